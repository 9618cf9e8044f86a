"""Right ILU(0) preconditioning (oracle, FP64).

TEST INFRASTRUCTURE ONLY: see the package docstring.

The paper's tests on matrices from applications (Sec. 5: the power-network,
circuit-simulation, near-singular and nonlinear-diffusion matrices) apply an
incomplete LU factorization with no fill, computed with MATLAB's ``ilu`` at
its default setting.  ILU(0) has a plain definition: L unit lower
triangular and U upper triangular, both supported on the sparsity pattern P
of A (L's strictly lower part on P's strictly lower part, U on P's upper part
including the diagonal), such that (L U)_ij = a_ij for every (i, j) in P.
Given nonzero pivots these conditions determine L and U uniquely; they are
obtained by Gaussian elimination in row (IKJ) order with every update outside
P dropped (Y. Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
Sec. 10.3.2, the ILU(0) algorithm), which is what ``ilu0`` does.

Readings (the paper does not state them):
  * the factorization uses the rows and columns in the order given (no
    reordering), and P is A's stored pattern (explicit zeros count as
    entries); every diagonal entry must be stored;
  * the preconditioner is applied on the right: the Krylov method runs on
    A M^{-1} with M = L U and the solution is X = M^{-1} Y.  The residual of
    A M^{-1} Y = B is then B - A X itself, so the stopping test (eq. normF_Rm
    over ||B||_F) measures the same quantity with and without M;
  * a zero (or non-finite) pivot u_ii is an error, reported with its row.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class ZeroPivot(ArithmeticError):
    """u_ii = 0 or not finite during ILU(0)."""

    def __init__(self, row: int):
        super().__init__(f"zero or non-finite pivot in row {row}")
        self.row = row


def ilu0(A):
    """ILU(0) factors (L, U) of a square sparse matrix A, as SciPy CSR.

    IKJ elimination restricted to A's pattern: for each row i in order, for
    each stored k < i in increasing order, l_ik = a_ik / u_kk and then
    a_ij <- a_ij - l_ik u_kj for the stored j > k of row i that row k also
    stores; fill-in outside the pattern is never formed."""
    M = sp.csr_matrix(A, dtype=np.float64, copy=True)
    M.sort_indices()
    n = M.shape[0]
    if M.shape[1] != n:
        raise ValueError("ILU(0) needs a square matrix")
    rows = []
    for i in range(n):
        a, b = M.indptr[i], M.indptr[i + 1]
        rows.append(dict(zip(M.indices[a:b].tolist(), M.data[a:b].tolist())))
    for i in range(n):
        ri = rows[i]
        if i not in ri:
            raise ValueError(f"row {i} stores no diagonal entry")
        for k in sorted(c for c in ri if c < i):
            rk = rows[k]
            lik = ri[k] / rk[k]
            ri[k] = lik
            for j, ukj in rk.items():
                if j > k and j in ri:
                    ri[j] = ri[j] - lik * ukj
        if ri[i] == 0.0 or not np.isfinite(ri[i]):
            raise ZeroPivot(i)
    Li, Lj, Lv, Ui, Uj, Uv = [], [], [], [], [], []
    for i, ri in enumerate(rows):
        for j, v in ri.items():
            if j < i:
                Li.append(i); Lj.append(j); Lv.append(v)
            else:
                Ui.append(i); Uj.append(j); Uv.append(v)
    Li.extend(range(n)); Lj.extend(range(n)); Lv.extend([1.0] * n)
    L = sp.csr_matrix((Lv, (Li, Lj)), shape=(n, n))
    U = sp.csr_matrix((Uv, (Ui, Uj)), shape=(n, n))
    L.sort_indices()
    U.sort_indices()
    return L, U


def ilu0_apply(L, U, Y):
    """M^{-1} Y = U^{-1} (L^{-1} Y) by forward and backward substitution."""
    Y = np.asarray(Y, dtype=np.float64)
    Z = spla.spsolve_triangular(L, Y, lower=True, unit_diagonal=True)
    return spla.spsolve_triangular(U, Z, lower=False)


class RightPreconditioned:
    """The operator A M^{-1} of the right-preconditioned system, applied as
    A (M^{-1} X); ``solution`` maps the Krylov solution Y to X = M^{-1} Y."""

    def __init__(self, A, L, U):
        self.A = A
        self.L = L
        self.U = U
        self.shape = A.shape

    def __matmul__(self, X):
        return self.A @ ilu0_apply(self.L, self.U, X)

    def solution(self, Y):
        return ilu0_apply(self.L, self.U, Y)
