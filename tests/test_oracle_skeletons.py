"""Pins for the oracle's block Arnoldi skeletons: invariants fixed by the
mathematics (Arnoldi relation, exact-arithmetic equality of skeletons,
closed-form spectrum)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle.skeletons import Counters, make_skeleton
from paper_2208_09899_amd import workloads as w

STABLE = ["bmgs", "bmgs_svl", "bmgs_lts", "bmgs_cwy", "bmgs_icwy", "bcgsi_ls"]
ALL = STABLE + ["bcgs_pip", "bcgs_pio"]


def _cycle(name, A, B, m, muscle="cholqr"):
    sk = make_skeleton(name, A, B.shape[1], m, muscle, Counters())
    last = 0
    for j in sk.run(B):
        last = j
    return sk, last


@pytest.mark.parametrize("muscle", ["cholqr", "houseqr"])
@pytest.mark.parametrize("name", ALL)
@pytest.mark.parametrize("case", ["lap1d", "lap2d", "convdiff"])
def test_block_arnoldi_relation(name, muscle, case):
    """A V_j = V_{j+1} H_{1:j+1,1:j} (Sec. 2.4, eq. block_arnoldi) to 1e-12."""
    if case == "lap1d":
        A, B, m = w.laplace_1d(1000).to_scipy(), w.rhs(1000, 4, 1), 20
    elif case == "lap2d":
        A, B, m = w.laplace_2d(32).to_scipy(), w.rhs(1024, 8, 2), 30
    else:
        A, B, m = w.convdiff_2d(40, 7.0, 0.8).to_scipy(), w.rhs(1600, 3, 9), 25
    sk, j = _cycle(name, A, B, m, muscle)
    assert j >= m - 1
    s = B.shape[1]
    Vj, Vj1 = sk.Vcat(j), sk.Vcat(j + 1)
    AV = A @ Vj
    rel = np.linalg.norm(AV - Vj1 @ sk.Hm1m(j)) / np.linalg.norm(AV)
    assert rel <= 1e-12, rel
    # the subdiagonal blocks are upper triangular Cholesky / R factors
    for k in range(1, j + 1):
        Hs = sk.H[k * s:(k + 1) * s, (k - 1) * s:k * s]
        assert np.allclose(np.tril(Hs, -1), 0.0)
        assert np.all(np.diag(Hs) > 0)
    # the first block of the basis spans B: B = V_1 Beta
    assert np.linalg.norm(sk.V[0] @ sk.Beta - B) <= 1e-13 * np.linalg.norm(B)


@pytest.mark.parametrize("name", ALL)
def test_skeletons_agree_in_exact_arithmetic(name):
    """All classical skeletons generate the same block QR, hence the same V and
    H (Sec. 2.4.2 remark); compared with textbook BMGS on the first columns of a
    well-conditioned problem."""
    A = (w.laplace_2d(24).to_scipy() + 3.0 * sp.identity(576)).tocsr()
    B = w.rhs(576, 4, 5)
    ref, _ = _cycle("bmgs", A, B, 8)
    sk, j = _cycle(name, A, B, 8)
    assert j == 8
    # BCGS-PIP's loss of orthogonality grows like eps * kappa^2 of the Krylov
    # basis (Table 2), which here gains about a factor 10 per block column.
    tol = 1e-6 if name in ("bcgs_pip", "bcgs_pio") else 1e-10
    assert np.linalg.norm(sk.Hm1m(8) - ref.Hm1m(8)) <= tol * np.linalg.norm(ref.Hm1m(8))
    assert np.linalg.norm(sk.Vcat(9) - ref.Vcat(9)) <= tol * 3


@pytest.mark.parametrize("name", ALL)
@pytest.mark.parametrize("n,s,m", [(64, 4, 16), (32, 4, 8)])
def test_hessenberg_spectrum_closed_form(name, n, s, m):
    """With n = m s the block Krylov space is the whole space, so H_m is similar
    to A = tridiag(-1,2,-1), whose eigenvalues are 2 - 2 cos(j pi/(n+1))."""
    A = w.laplace_1d(n).to_scipy()
    B = w.rhs(n, s, 11)
    sk, _ = _cycle(name, A, B, m)
    Hm = sk.H[: m * s, : m * s]
    ev = np.sort(np.linalg.eigvals(Hm).real)
    exact = np.sort(2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    # PIP / PIO: O(eps kappa^2) loss of orthogonality (Table 2)
    tol = 1e-7 if name in ("bcgs_pip", "bcgs_pio") else 1e-10
    assert np.max(np.abs(ev - exact)) <= tol


def test_delayed_skeletons_flag_two_columns_back():
    """A forced Cholesky flag at loop step k leaves k-2 final columns in the
    delayed skeletons (Algs. 6, 7) and k-1 in the others."""
    A = w.laplace_1d(300).to_scipy()
    B = w.rhs(300, 2, 3)
    for name in ALL:
        sk = make_skeleton(name, A, 2, 10, "cholqr", Counters(), force_steps={5})
        cols = list(sk.run(B))
        expect = 3 if sk.delayed else 4
        assert sk.flagged and sk.last == expect and cols == list(range(1, expect + 1))


@pytest.mark.parametrize("name", ALL)
def test_counters_per_cycle(name):
    """Per-cycle A-calls / basis applications / syncs of a full cycle of j
    columns, as implied by the appendix tables (Sec. 5 and Appendix A)."""
    A = w.laplace_1d(500).to_scipy()
    B = w.rhs(500, 3, 4)
    ct = Counters()
    sk = make_skeleton(name, A, 3, 12, "cholqr", ct)
    j = len(list(sk.run(B)))
    assert j == 12
    expect = {
        "bmgs": (j, 2 * j, j * (j + 1) // 2 + j + 1),
        "bcgs_pip": (j, 3 * j, j + 1),
        "bcgs_pio": (j, 2 * j, 2 * j + 1),
        "bmgs_svl": (j, 3 * j, 3 * j + 1),
        "bmgs_lts": (j, 3 * j, 3 * j + 1),
        "bmgs_cwy": (j + 1, 3 * j + 1, j + 2),
        "bmgs_icwy": (j + 1, 3 * j + 1, j + 2),
        "bcgsi_ls": (j + 1, 4 * j + 1, j + 2),
    }[name]
    assert ct.as_tuple() == expect


@pytest.mark.parametrize("muscle", ["cholqr", "houseqr"])
def test_pio_intraortho_of_block_diagonal(muscle):
    """Alg. 4's IntraOrtho of [W 0; 0 H]: the columns of the two blocks are
    orthogonal to each other, so R is block diagonal [R_W 0; 0 R_H] with
    R_W^T R_W = W^T W and R_H^T R_H = H^T H (the QR factors of each block)."""
    from oracle.primitives import intra_ortho
    rng = np.random.default_rng(7)
    n, k, s = 300, 5, 3
    W = rng.standard_normal((n, s))
    Hk = rng.standard_normal((k * s, s))
    D = np.zeros((n + k * s, 2 * s))
    D[:n, :s] = W
    D[n:, s:] = Hk
    Q, R, _, ok = intra_ortho(D, muscle)
    assert ok
    assert np.linalg.norm(R[:s, s:]) <= 1e-13 * np.linalg.norm(R)
    assert np.allclose(R[:s, :s].T @ R[:s, :s], W.T @ W, rtol=1e-12, atol=1e-12 * np.linalg.norm(W) ** 2)
    assert np.allclose(R[s:, s:].T @ R[s:, s:], Hk.T @ Hk, rtol=1e-12, atol=1e-12 * np.linalg.norm(Hk) ** 2)
    assert np.linalg.norm(Q @ R - D) <= 1e-13 * np.linalg.norm(D)


def test_pio_equals_pip_on_a_well_conditioned_cycle():
    """Algs. 3 and 4 compute H_{k+1,k} from the same quantity (Omega - H^T H
    = R_W^T R_W - R_H^T R_H in exact arithmetic), so their bases and
    Hessenberg matrices agree to rounding over the first columns.  Both have
    O(eps kappa^2) loss of orthogonality (Table 2) and kappa of the block
    Krylov basis grows with every column, so the rounding difference grows
    too: measured here 2e-14, 2e-13, 3e-12, 4e-11 after 2..5 columns; the
    check is on 3 columns."""
    A = (w.laplace_2d(20).to_scipy() + 4.0 * sp.identity(400)).tocsr()
    B = w.rhs(400, 3, 9)
    pip, _ = _cycle("bcgs_pip", A, B, 3)
    pio, _ = _cycle("bcgs_pio", A, B, 3)
    assert np.linalg.norm(pio.Hm1m(3) - pip.Hm1m(3)) <= 1e-11 * np.linalg.norm(pip.Hm1m(3))
    assert np.linalg.norm(pio.Vcat(4) - pip.Vcat(4)) <= 1e-11


@pytest.mark.parametrize("name", ["bmgs", "bmgs_svl", "bmgs_lts", "bmgs_cwy", "bmgs_icwy",
                                  "bcgsi_ls", "bcgs_pip"])
def test_global_paradigm_arnoldi_relation(name):
    """Global paradigm (Sec. 2.2, Table 1): A V_j = V_{j+1} H_{j+1,j} holds,
    the basis is orthonormal in the global inner product
    ((1/s) trace(V_i^T V_k) = delta_ik), and every s x s block of H is a
    multiple of I_s."""
    from oracle.primitives import ip_global
    A = w.convdiff_2d(20, 4.0, 0.5).to_scipy()
    B = w.rhs(400, 3, 17)
    sk, j = _cycle(name, A, B, 10, muscle="global")
    assert j == 10
    s = 3
    V = sk.Vcat(j + 1)
    H = sk.Hm1m(j)
    AV = A @ sk.Vcat(j)
    assert np.linalg.norm(AV - V @ H) <= 1e-12 * np.linalg.norm(AV)
    G = ip_global(V, V, s)
    tol = 1e-7 if name == "bcgs_pip" else 1e-12
    assert np.linalg.norm(np.eye(V.shape[1]) - G, 2) <= tol
    for a in range(j + 1):
        for b in range(j):
            blk = H[a * s:(a + 1) * s, b * s:(b + 1) * s]
            assert np.allclose(blk, blk[0, 0] * np.eye(s), rtol=0, atol=1e-14 * (1 + abs(blk[0, 0])))
