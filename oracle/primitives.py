"""Block inner product and intra-orthogonalization muscles (oracle, FP64).

Test infrastructure only: see the package docstring.

Real arithmetic throughout, so the conjugate transpose of the paper is the
plain transpose.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


def ip(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Classical block inner product <X, Y> = X^T Y (Sec. 2.2, Table 1)."""
    return X.T @ Y


def ip_global(X: np.ndarray, Y: np.ndarray, s: int) -> np.ndarray:
    """Global block inner product (Sec. 2.2, Table 1): for n x s block vectors
    <X, Y> = (1/s) trace(X^T Y) I_s.  For concatenations [X_1 .. X_p] and
    [Y_1 .. Y_q] the result is the p s x q s matrix of the pairwise global
    products (each s x s block a multiple of I_s)."""
    G = X.T @ Y
    p, q = G.shape[0] // s, G.shape[1] // s
    out = np.zeros_like(G)
    for i in range(p):
        for j in range(q):
            t = np.trace(G[i * s:(i + 1) * s, j * s:(j + 1) * s]) / s
            out[i * s:(i + 1) * s, j * s:(j + 1) * s] = t * np.eye(s)
    return out


def chol_flag(Om: np.ndarray):
    """Cholesky factor with a breakdown flag (Sec. 4, the ``chol`` variant that
    raises the NaN-flag instead of failing).

    Returns (R, ok) with R upper triangular and R^T R = Om, computed from the
    upper triangle of Om by the unblocked column-by-column recurrence.

    Reading: the flag is raised iff some pivot Om_jj - sum_{i<j} R_ij^2 is
    not a positive finite number (the paper speaks of a matrix that is
    numerically not positive definite; no further threshold is applied).
    On a flag the returned R is incomplete and must not be used.
    """
    Om = np.asarray(Om, dtype=np.float64)
    s = Om.shape[0]
    R = np.zeros((s, s))
    for j in range(s):
        d = Om[j, j] - R[:j, j] @ R[:j, j]
        if not np.isfinite(d) or d <= 0.0:
            return R, False
        R[j, j] = math.sqrt(d)
        if j + 1 < s:
            R[j, j + 1:] = (Om[j, j + 1:] - R[:j, j] @ R[:j, j + 1:]) / R[j, j]
    return R, True


def right_solve_upper(X: np.ndarray, R: np.ndarray) -> np.ndarray:
    """X R^{-1} for upper-triangular R (a triangular solve, not an inverse)."""
    return sla.solve_triangular(R, X.T, trans="T", lower=False, check_finite=False).T


def left_solve_upper_t(R: np.ndarray, X: np.ndarray) -> np.ndarray:
    """R^{-T} X for upper-triangular R."""
    return sla.solve_triangular(R, X, trans="T", lower=False, check_finite=False)


def cholqr(X: np.ndarray):
    """CholQR muscle (Sec. 2.3 and the list of muscles in Sec. 5):
    G = X^T X (one sync), R = chol(G) with flag, Q = X R^{-1}.
    Returns (Q, R, ok)."""
    G = ip(X, X)
    R, ok = chol_flag(G)
    if not ok:
        return None, R, False
    return right_solve_upper(X, R), R, True


def houseqr(X: np.ndarray):
    """HouseQR muscle: Householder QR (LAPACK via numpy), the unconditionally
    stable muscle of Sec. 4.

    Reading: the signs are fixed so that diag(R) >= 0 (a zero diagonal entry
    gets sign +1), which makes the factorization unique for full-rank X.
    The flag is raised only for an exactly zero or non-finite diagonal."""
    Q, R = np.linalg.qr(X, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    Q = Q * d
    R = d[:, None] * R
    ok = bool(np.all(np.isfinite(R)) and np.all(np.diag(R) != 0.0))
    return Q, R, ok


def global_muscle(X: np.ndarray):
    """The global paradigm's muscle (Sec. 2.2, Table 1): N(X) = ||X||_F /
    sqrt(s) I_s, Q = X N(X)^{-1} -- a scaling, no intra-orthogonalization.
    It is CholQR under the global inner product (the Cholesky factor of
    (1/s) ||X||_F^2 I_s); the flag is raised when ||X||_F^2 is not a positive
    finite number.  Returns (Q, R, ok)."""
    s = X.shape[1]
    nu2 = float(np.sum(X * X)) / s
    if not np.isfinite(nu2) or nu2 <= 0.0:
        return None, np.zeros((s, s)), False
    nu = math.sqrt(nu2)
    return X / nu, nu * np.eye(s), True


def mgs_lowsync(X: np.ndarray, lts: bool):
    """Column-wise MGS-SVL / MGS-LTS muscles (Sec. 5 list of muscles; the
    column versions of Alg. 5): for column j, y = Q_{1:j-1}^T x_j,
    h = T^T y (SVL) or T^{-T} y (LTS), w = x_j - Q h, r = ||w|| (from w^T w),
    q_j = w / r, then z = Q_{1:j-1}^T q_j and the new column of T,
    -T z (SVL) or z (LTS), with T_jj = 1.  Syncs: 1 for the first column and
    3 for each later one, 3 s - 2 per call.  The flag is raised when some
    w^T w is not a positive finite number.  Returns (Q, R, T, ok)."""
    n, s = X.shape
    Q = np.zeros((n, s))
    R = np.zeros((s, s))
    T = np.eye(s)
    for j in range(s):
        x = X[:, j]
        if j > 0:
            y = Q[:, :j].T @ x
            Tj = T[:j, :j]
            h = sla.solve_triangular(Tj.T, y, lower=True, check_finite=False) if lts else Tj.T @ y
            w = x - Q[:, :j] @ h
            R[:j, j] = h
        else:
            w = x
        rr = float(w @ w)
        if not np.isfinite(rr) or rr <= 0.0:
            return None, R, T, False
        r = math.sqrt(rr)
        R[j, j] = r
        Q[:, j] = w / r
        if j > 0:
            z = Q[:, :j].T @ Q[:, j]
            T[:j, j] = z if lts else -(T[:j, :j] @ z)
    return Q, R, T, True


def muscle_syncs(muscle: str, s: int) -> int:
    """Syncs of one IntraOrtho call: one block inner product for CholQR,
    HouseQR (TSQR) and the global muscle; 3 s - 2 for the column-wise MGS
    muscles (Sec. 5 counts syncs inside the muscles; the appendix's totals
    imply 3 s - 2 = 1 + 3 (s - 1))."""
    return 3 * s - 2 if muscle in ("mgs_svl", "mgs_lts") else 1


def intra_ortho(X: np.ndarray, muscle: str):
    """IntraOrtho(X) -> (Q, R, T, ok).  T is the auxiliary factor the
    SVL/LTS skeletons expect from the muscle (Alg. 5, lines 2 and 7).

    Reading: CholQR, HouseQR and the global muscle carry no such factor;
    T = I_s, its value for an exactly orthonormal Q.  muscle = "global"
    selects the global paradigm as a whole (the skeletons then use the global
    inner product too; the paper forces the global muscle there, Sec. 5)."""
    if muscle == "cholqr":
        Q, R, ok = cholqr(X)
    elif muscle == "houseqr":
        Q, R, ok = houseqr(X)
    elif muscle == "global":
        Q, R, ok = global_muscle(X)
    elif muscle in ("mgs_svl", "mgs_lts"):
        return mgs_lowsync(X, muscle == "mgs_lts")
    else:
        raise ValueError(f"unknown muscle {muscle!r}")
    return Q, R, np.eye(X.shape[1]), ok
