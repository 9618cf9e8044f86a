"""Pins for the oracle's ILU(0) factors, their application and the
right-preconditioned solve (Sec. 5, the tests on matrices from applications;
ILU(0) as Gaussian elimination restricted to A's pattern).

Each pin checks the oracle against something it does not compute itself: the
defining property (L U)_ij = a_ij on the pattern (through a sparse product,
not the elimination), LAPACK's LU where ILU(0) has no dropped fill, the
closed-form recurrence of ILU(0) for the 5-point Laplacian with its known
remainder, and dense solves."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from oracle.precond import ilu0, ilu0_apply, ZeroPivot

from paper_2208_09899_amd import workloads as w


def _pattern(M):
    """Stored (row, column) pairs, explicit zeros included."""
    M = sp.csr_matrix(M)
    r = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    return set(zip(r.tolist(), M.indices.tolist()))


def _random_pattern_matrix(n, density, seed, nonsym=True):
    """Random sparse matrix with a nonsymmetric pattern, every diagonal stored,
    diagonally dominant by rows (nonzero pivots)."""
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, format="csr")
    M.data = rng.standard_normal(M.data.shape[0])
    if not nonsym:
        M = M + M.T
    M = M.tolil()
    rowsum = np.asarray(abs(M).sum(axis=1)).ravel()
    for i in range(n):
        M[i, i] = rowsum[i] + 1.0 + rng.random()
    return M.tocsr()


@pytest.mark.parametrize("seed", range(4))
def test_ilu0_defining_property_nonsymmetric_pattern(seed):
    """L unit lower and U upper, both on A's pattern, and (L U)_ij = a_ij for
    every stored (i, j): the conditions that determine ILU(0) uniquely."""
    A = _random_pattern_matrix(80, 0.06, seed)
    L, U = ilu0(A)
    P = _pattern(A)
    assert np.array_equal(L.diagonal(), np.ones(80))
    assert sp.triu(L, 1).nnz == 0 and sp.tril(U, -1).nnz == 0
    for (i, j) in _pattern(L) | _pattern(U):
        assert (i, j) in P
    LU = (L @ U).tocsr()
    Ad = A.toarray()
    LUd = LU.toarray()
    scale = np.abs(Ad).max()
    worst = max(abs(LUd[i, j] - Ad[i, j]) for (i, j) in P)
    assert worst <= 1e-13 * scale
    # fill was dropped: L U differs from A somewhere off the pattern
    off = [(i, j) for i in range(80) for j in range(80) if (i, j) not in P]
    assert max(abs(LUd[i, j]) for (i, j) in off) > 1e-8


def test_ilu0_of_tridiagonal_is_lapack_lu():
    """A tridiagonal matrix has no fill: ILU(0) is its LU factorization,
    which LAPACK's getrf reproduces without row exchanges for the 1-D
    Laplacian (pivots (k+1)/k, column dominance)."""
    A = w.laplace_1d(60).to_scipy()
    L, U = ilu0(A)
    P, Ll, Ul = sla.lu(A.toarray())
    assert np.array_equal(P, np.eye(60))
    assert np.abs(L.toarray() - Ll).max() <= 1e-15
    assert np.abs(U.toarray() - Ul).max() <= 1e-14
    assert np.abs((L @ U - A).toarray()).max() <= 1e-14
    assert np.allclose(U.diagonal(), (np.arange(60) + 2) / (np.arange(60) + 1), rtol=1e-14)


def test_ilu0_of_full_pattern_is_lapack_lu():
    """With every entry stored nothing is dropped: ILU(0) = LU without
    pivoting, which getrf gives on a matrix that is diagonally dominant by
    columns (no row exchange)."""
    rng = np.random.default_rng(5)
    D = rng.standard_normal((25, 25))
    D += np.diag(np.abs(D).sum(axis=0) + 1.0)
    L, U = ilu0(sp.csr_matrix(D))
    P, Ll, Ul = sla.lu(D)
    assert np.array_equal(P, np.eye(25))
    assert np.abs(L.toarray() - Ll).max() <= 1e-14
    assert np.abs(U.toarray() - Ul).max() <= 1e-13 * np.abs(D).max()


@pytest.mark.parametrize("N", [3, 7, 16])
def test_ilu0_laplace2d_closed_form(N):
    """5-point Laplacian, natural ordering (i = x + N y): the ILU(0) pivots
    satisfy d_i = 4 - [x > 0] / d_{i-1} - [y > 0] / d_{i-N}, the multipliers
    are l_{i,i-1} = -1/d_{i-1}, l_{i,i-N} = -1/d_{i-N}, U keeps A's
    off-diagonal -1 entries, and the remainder L U - A is nonzero only at
    (i, i-N+1) (value 1/d_{i-N}, for y > 0, x < N-1) and (i, i+N-1) (value
    1/d_{i-1}, for x > 0, y < N-1).  N >= 3 (at N = 2 those positions are on
    the pattern).  The explicit zeros SciPy's kron stores for tiny grids are
    removed first, so that the pattern is the stencil's."""
    A = w.laplace_2d(N).to_scipy()
    A.eliminate_zeros()
    n = N * N
    d = np.zeros(n)
    Le = np.eye(n)
    Ue = np.zeros((n, n))
    Re = np.zeros((n, n))
    for i in range(n):
        x, y = i % N, i // N
        d[i] = 4.0
        if y > 0:
            d[i] -= 1.0 / d[i - N]
            Le[i, i - N] = -1.0 / d[i - N]
            if x < N - 1:
                Re[i, i - N + 1] = 1.0 / d[i - N]
        if x > 0:
            d[i] -= 1.0 / d[i - 1]
            Le[i, i - 1] = -1.0 / d[i - 1]
            if y < N - 1:
                Re[i, i + N - 1] = 1.0 / d[i - 1]
        Ue[i, i] = d[i]
        if x < N - 1:
            Ue[i, i + 1] = -1.0
        if y < N - 1:
            Ue[i, i + N] = -1.0
    L, U = ilu0(A)
    assert np.abs(L.toarray() - Le).max() <= 1e-15
    assert np.abs(U.toarray() - Ue).max() <= 4e-15
    R = (L @ U - A).toarray()
    assert np.abs(R - Re).max() <= 1e-14


def test_ilu0_apply_matches_dense_solve():
    A = _random_pattern_matrix(70, 0.08, 11)
    L, U = ilu0(A)
    Y = np.random.default_rng(2).standard_normal((70, 5))
    Z = ilu0_apply(L, U, Y)
    Zd = np.linalg.solve(L.toarray() @ U.toarray(), Y)
    assert np.abs(Z - Zd).max() <= 1e-13 * np.abs(Zd).max()


def test_ilu0_rejects_missing_diagonal_and_zero_pivot():
    M = sp.csr_matrix(np.array([[1.0, 2.0], [3.0, 0.0]]))
    M.eliminate_zeros()
    with pytest.raises(ValueError):
        ilu0(M)
    # explicit zero on the diagonal of row 1 after elimination: 6 - 3 * 2 = 0
    Z = sp.csr_matrix(np.array([[1.0, 2.0], [3.0, 6.0]]))
    with pytest.raises(ZeroPivot) as e:
        ilu0(Z)
    assert e.value.row == 1


def test_right_preconditioned_solve_with_exact_factors_takes_one_column():
    """Tridiagonal A: M = L U = A, so A M^{-1} = I and the first block
    column already solves the system; X is A^{-1} B."""
    A = w.laplace_1d(200).to_scipy()
    B = w.rhs(200, 3, seed=1)
    res = oracle.solve(A, B, method="gmres", skeleton="bcgsi_ls", m=10, tol=1e-10,
                       precond=ilu0(A))
    assert res.status == "ok" and res.iters == 1
    Xd = np.linalg.solve(A.toarray(), B)
    assert np.abs(res.X - Xd).max() <= 1e-10 * np.abs(Xd).max()


@pytest.mark.parametrize("skel", ["bcgsi_ls", "bmgs_cwy", "bmgs_svl"])
def test_right_preconditioned_convdiff_residual_and_error(skel):
    """Nonsymmetric convection-diffusion operator, BGMRES(10) with right
    ILU(0): the true residual B - A X of the returned X meets the tolerance
    (right preconditioning leaves the residual that of the original system),
    the estimates do not increase within a cycle (BGMRES minimises the
    residual over a growing space), the preconditioner cuts the iteration
    count, and X agrees with a dense solve within kappa times the residual."""
    A = w.convdiff_2d(12, 8.0, 0.4).to_scipy()
    B = w.rhs(A.shape[0], 4, seed=3)
    tol = 1e-9
    pre = oracle.solve(A, B, method="gmres", skeleton=skel, m=10, tol=tol, max_cycles=200,
                       precond=ilu0(A))
    plain = oracle.solve(A, B, method="gmres", skeleton=skel, m=10, tol=tol, max_cycles=400)
    assert pre.status == "ok" and plain.status == "ok"
    r = np.linalg.norm(B - A @ pre.X) / np.linalg.norm(B)
    assert r <= 1.01 * tol
    assert pre.iters < plain.iters
    pos = 0
    for cl in pre.cycle_len:
        h = pre.res_hist[pos:pos + cl]
        assert all(b <= a * (1 + 1e-12) for a, b in zip(h, h[1:]))
        pos += cl
    Ad = A.toarray()
    Xd = np.linalg.solve(Ad, B)
    kap = np.linalg.cond(Ad)
    assert np.linalg.norm(pre.X - Xd) / np.linalg.norm(Xd) <= kap * 2 * tol


@pytest.mark.parametrize("skel", ["bcgsi_ls", "bmgs_cwy", "bmgs_svl", "bmgs"])
def test_right_preconditioned_arnoldi_relation(skel):
    """One cycle on A M^{-1}: the block Arnoldi relation (Sec. 2.4, eq.
    block_arnoldi) holds for the operator formed independently as the dense
    product A (L U)^{-1} (a dense LU solve, not the oracle's triangular
    sweeps), to 1e-12.  (The basis's loss of orthogonality is the skeleton's
    own, O(u kappa) of the Krylov basis, and is not bounded here.)"""
    from oracle.precond import RightPreconditioned
    from oracle.skeletons import Counters, make_skeleton
    A = w.convdiff_2d(20, 6.0, 0.7).to_scipy()
    B = w.rhs(A.shape[0], 3, seed=4)
    L, U = ilu0(A)
    sk = make_skeleton(skel, RightPreconditioned(A, L, U), 3, 15, "cholqr", Counters())
    j = 0
    for jj in sk.run(B):
        j = jj
    assert j >= 14
    Md = (L @ U).toarray()
    AMinv = np.linalg.solve(Md.T, A.toarray().T).T       # A M^{-1}
    Vj, Vj1 = sk.Vcat(j), sk.Vcat(j + 1)
    lhs = AMinv @ Vj
    rel = np.linalg.norm(lhs - Vj1 @ sk.Hm1m(j)) / np.linalg.norm(lhs)
    assert rel <= 1e-12, rel
