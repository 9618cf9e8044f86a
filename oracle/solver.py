"""Restarted BFOM / BGMRES with cospatial restarts and adaptive restarting (oracle, FP64).

Test infrastructure only: see the package docstring.

Follows Sec. 2.4.1 (eq. Xm: X_m = V_m (H_m + M)^{-1} E_1 B, with M = 0 for
BFOM and M = H_m^{-T} (E_m H_{m+1,m}^T H_{m+1,m}) E_m^T for BGMRES),
Sec. 2.4.2 (Theorem 1: R_m = U_m (E_m^T Xi_m) with
U_m = V_{m+1} [M; -H_{m+1,m}], the residual-norm identity eq. normF_Rm, and
the restart X <- X + D) and Sec. 4 (adaptive restarting on a Cholesky
breakdown: keep the last final column, restart from there, shrink m).

Readings (where the paper is silent or ambiguous):
  * X_0 = 0; the first cycle starts from R_0 = B with cospatial factor C = I.
  * Convergence is tested after every final block column j against the
    residual estimate of eq. normF_Rm divided by ||B||_F (Sec. 5); a cycle
    therefore has m columns unless it converges or breaks down.
  * Each restart builds K(A, U_j) from the restart block U_j (formed
    explicitly) and carries the cospatial factor C = E_j^T Xi_j, so the next
    cycle's right-hand side is E_1 B' C with B' the factor of IntraOrtho(U_j).
  * On a Cholesky flag with j >= 1 final columns: X is updated with Xi_j,
    the restart uses V_{j+1}, and m <- j for all later cycles (m never
    grows).  With j = 0 the solve stops with status "breakdown".
  * A singular H_j (possible for nonsymmetric A) gives an infinite BFOM
    estimate for that column; BGMRES then falls back to the least-squares
    form of its iterate (identical in exact arithmetic).  If the last column
    of a BFOM cycle has a singular H_j (no BFOM iterate exists), the cycle
    ends with the least-squares iterate of that column instead.  After a
    least-squares iterate the next cycle restarts from its residual block
    V_{j+1} (E_1 B C - H_{j+1,j} Xi) with C = I (the factor M of Thm. 1 needs
    H_j^{-T}).
  * ``max_cycles`` bounds the number of cycles; exhausting it returns the
    last iterate with status "not_converged".
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .precond import RightPreconditioned
from .skeletons import Counters, make_skeleton


@dataclasses.dataclass
class OracleResult:
    X: np.ndarray
    status: str                      # "ok" | "not_converged" | "breakdown"
    iters: int
    res_hist: list
    loo_hist: list
    cycle_len: list
    m_after: list
    counts: tuple                    # (a_calls, v_apps, syncs)
    cycles: list = dataclasses.field(default_factory=list)   # per-cycle data if keep_cycles


def small_solve(method: str, Hj1: np.ndarray, BC: np.ndarray, s: int):
    """Coefficients of the (modified) BFOM iterate for j final columns.

    Hj1 is H_{1:j+1,1:j} ((j+1)s x js), BC = B C (s x s).  Returns
    (Xi, M, est) with Xi = (H_j + M E_j^T)^{-1} E_1 B C (eq. Xm), M the
    modification's s-column factor and est the residual norm of eq. normF_Rm,
    ||[M; -H_{j+1,j}] E_j^T Xi||_F."""
    js = Hj1.shape[1]
    j = js // s
    Hj = Hj1[:js, :]
    Hsub = Hj1[js:, (j - 1) * s:]
    rhs = np.zeros((js, s))
    rhs[:s] = BC
    M = np.zeros((js, s))
    try:
        if method == "gmres":
            E = np.zeros((js, s))
            E[(j - 1) * s:] = Hsub.T @ Hsub
            M = np.linalg.solve(Hj.T, E)
        Hmod = Hj.copy()
        Hmod[:, (j - 1) * s:] += M
        Xi = np.linalg.solve(Hmod, rhs)
    except np.linalg.LinAlgError:
        if method == "fom":
            return None, M, np.inf
        # least-squares form of the BGMRES iterate: min ||E_1 B C - H_{j+1,j} Xi||_F
        g = np.zeros(((j + 1) * s, s))
        g[:s] = BC
        Xi = np.linalg.lstsq(Hj1, g, rcond=None)[0]
        res = g - Hj1 @ Xi
        return Xi, None, float(np.linalg.norm(res))
    last = Xi[(j - 1) * s:]
    est = float(np.linalg.norm(np.vstack([M, -Hsub]) @ last))
    return Xi, M, est


def solve(A, B, method: str = "gmres", skeleton: str = "bcgsi_ls", muscle: str = "cholqr",
          m: int = 20, tol: float = 1e-8, max_cycles: int = 50, record_loo: bool = False,
          force_flag=(), keep_cycles: bool = False, max_iters: int | None = None,
          x_star=None, precond=None) -> OracleResult:
    """Restarted block solve of A X = B (Secs. 2.4, 4).

    Stopping: by default after the first column whose residual estimate
    (eq. normF_Rm) divided by ||B||_F is <= tol.  If ``x_star`` is given the
    test is instead ||X_j - X_*||_F / ||X_*||_F <= tol, the relative error the
    paper's benchmarks measure when a ground truth is available (Sec. 5).
    ``max_iters`` (optional) stops after that many final columns in total,
    with status "not_converged"; it is used to sample a bounded amount of work.

    ``force_flag`` is a collection of (cycle, step) pairs (1-based cycle,
    skeleton loop step k; k = 0 is the cycle's first IntraOrtho) at which the
    Cholesky breakdown flag is raised regardless of the data -- a test hook for
    the adaptive-restart path.

    ``precond`` (optional) is a pair (L, U) of ILU(0) factors
    (``oracle.precond.ilu0``): the cycles then run on A M^{-1}, M = L U
    (right preconditioning), and the returned X is M^{-1} Y for the Krylov
    solution Y; the per-cycle data kept by ``keep_cycles`` stays in terms
    of Y."""
    if precond is not None:
        Aop = RightPreconditioned(A, *precond)
        res = _solve(Aop, B, method, skeleton, muscle, m, tol, max_cycles, record_loo,
                     force_flag, keep_cycles, max_iters, x_star, Aop.solution)
        res.X = Aop.solution(res.X)
        return res
    return _solve(A, B, method, skeleton, muscle, m, tol, max_cycles, record_loo, force_flag,
                  keep_cycles, max_iters, x_star, lambda Y: Y)


def _solve(A, B, method, skeleton, muscle, m, tol, max_cycles, record_loo, force_flag,
           keep_cycles, max_iters, x_star, sol) -> OracleResult:
    B = np.asarray(B, dtype=np.float64)
    n, s = B.shape
    X = np.zeros((n, s))
    nB = float(np.linalg.norm(B))
    ct = Counters()
    res_hist, loo_hist, cycle_len, m_after, cycles = [], [], [], [], []
    if nB == 0.0:
        return OracleResult(X, "ok", 0, res_hist, loo_hist, cycle_len, m_after, ct.as_tuple())
    forced = {}
    for (c, k) in force_flag:
        forced.setdefault(c, set()).add(k)
    C = np.eye(s)
    R0 = B
    for c in range(1, max_cycles + 1):
        sk = make_skeleton(skeleton, A, s, m, muscle, ct, forced.get(c, ()))
        conv = False
        j = 0
        Xi = M = None
        for jj in sk.run(R0):
            j = jj
            Hj1 = sk.Hm1m(j)
            Xi, M, est = small_solve(method, Hj1, sk.Beta @ C, s)
            res_hist.append(est / nB)
            if record_loo:
                Vc = sk.Vcat(j + 1)
                loo_hist.append(float(np.linalg.norm(np.eye((j + 1) * s) - sk.ip(Vc, Vc), 2)))
            if x_star is None:
                crit = est / nB
            elif Xi is None:
                crit = np.inf
            else:
                crit = np.linalg.norm(sol(X + sk.Vcat(j) @ Xi) - x_star) / np.linalg.norm(x_star)
            if crit <= tol:
                conv = True
                break
            if max_iters is not None and len(res_hist) >= max_iters:
                break
        if not conv and sk.flagged:
            j = sk.last
            if j == 0:
                cycle_len.append(0)
                m_after.append(m)
                return OracleResult(X, "breakdown", len(res_hist), res_hist, loo_hist,
                                    cycle_len, m_after, ct.as_tuple(), cycles)
            m = j
            # Xi / M of column j are the last ones computed (columns are final in order)
        if Xi is None:
            # BFOM with a singular H_j at the cycle's last column: least-squares iterate
            g = np.zeros(((j + 1) * s, s))
            g[:s] = sk.Beta @ C
            Xi = np.linalg.lstsq(sk.Hm1m(j), g, rcond=None)[0]
            M = None
        Vj = sk.Vcat(j)
        X = X + Vj @ Xi
        cycle_len.append(j)
        m_after.append(m)
        if keep_cycles:
            cycles.append(dict(V=[v.copy() for v in sk.V[: j + 1]], H=sk.Hm1m(j).copy(),
                               Xi=Xi.copy(), M=None if M is None else M.copy(),
                               Beta=sk.Beta.copy(), C=C.copy(), X=X.copy(), j=j))
        if conv:
            return OracleResult(X, "ok", len(res_hist), res_hist, loo_hist, cycle_len,
                                m_after, ct.as_tuple(), cycles)
        if max_iters is not None and len(res_hist) >= max_iters:
            break
        Hsub = sk.H[j * s:(j + 1) * s, (j - 1) * s:j * s]
        if M is None:   # least-squares fallback above: restart from the residual itself
            g = np.zeros(((j + 1) * s, s)); g[:s] = sk.Beta @ C
            U = sk.Vcat(j + 1) @ (g - sk.Hm1m(j) @ Xi)
            C = np.eye(s)
        else:
            U = sk.Vcat(j + 1) @ np.vstack([M, -Hsub])
            C = Xi[(j - 1) * s:].copy()
        if keep_cycles:
            cycles[-1]["U"] = U.copy()
            cycles[-1]["C_next"] = C.copy()
        R0 = U
    return OracleResult(X, "not_converged", len(res_hist), res_hist, loo_hist, cycle_len,
                        m_after, ct.as_tuple(), cycles)
