"""The precision form on the GPU: inner BFOM/BGMRES with FP32 block vectors
(SpMM, Gram products, fused updates), FP64 small dense steps with the
shifted-Cholesky fallback, and outer iterative refinement on the FP64
residual B - A X.

Each test solves to a relative residual of 1e-8 and reports the error of X
against the FP64 oracle's solution of the same seeded problem.  The bound on
that error follows from the residuals: for X and X_o with relative residuals
r and r_o, ||X - X_o|| / ||X_o|| <= kappa(A) (r + r_o) / (1 - kappa(A) r_o)."""
import numpy as np
import pytest

from paper_2208_09899_amd import workloads as w

from gpu_common import gpu_solve, oracle_solve

pytestmark = pytest.mark.gpu


def kappa_laplace2d(N):
    """Spectral condition number of the 5-point Dirichlet Laplacian on an N x N
    grid: eigenvalues 4 - 2 cos(i pi/(N+1)) - 2 cos(j pi/(N+1))."""
    c = np.cos(np.pi / (N + 1))
    return (4 + 4 * c) / (4 - 4 * c)


def true_relres(csr, X, B):
    return np.linalg.norm(B - csr.to_scipy() @ X) / np.linalg.norm(B)


@pytest.mark.parametrize("method,skel", [("gmres", "bcgsi_ls"), ("fom", "bcgsi_ls"),
                                         ("gmres", "bmgs_cwy"), ("gmres", "bmgs_svl"),
                                         ("gmres", "bmgs_icwy"), ("gmres", "bmgs_lts")])
def test_mixed_reaches_tolerance_laplace2d(method, skel):
    N, s, tol = 48, 8, 1e-8
    A = w.laplace_2d(N)
    B = w.rhs(A.n, s, seed=11)
    g = gpu_solve(A, B, method=method, skeleton=skel, m=20, tol=tol, max_cycles=200,
                  precision="mixed", max_refine=20, inner_tol=1e-4)
    o = oracle_solve(A, B, method, skel, m=20, tol=tol, max_cycles=1000)
    assert g.status == "ok"
    assert g.refine_steps >= 2          # FP32 inner solves cannot reach 1e-8 alone
    r = true_relres(A, g.X, B)
    assert abs(r - g.true_relres) <= 1e-12
    assert r <= tol
    r_o = true_relres(A, o.X, B)
    kap = kappa_laplace2d(N)
    err = np.linalg.norm(g.X - o.X) / np.linalg.norm(o.X)
    print(f"mixed {method}/{skel}: refinement steps {g.refine_steps}, inner block "
          f"iterations {g.iters}, true relres {r:.2e}, error vs FP64 oracle {err:.2e}")
    assert err <= kap * (r + r_o) / (1 - kap * r_o)


def test_mixed_graph_laplacian_restarts():
    """Random geometric graph Laplacian + 1e-3 I (n = 2^13, kappa ~ 2e4),
    s = 16, m = 25, many restarts per inner solve: the refined solution
    reaches 1e-8 and agrees with the FP64 GPU solve within the residual bound
    (kappa ~ 2e4 from the largest degree and the shift)."""
    A = w.rgg_laplacian(1 << 13, seed=3, degree=4, shift=1e-3)
    B = w.rhs(A.n, 16, seed=4)
    tol = 1e-8
    g = gpu_solve(A, B, method="gmres", skeleton="bcgsi_ls", m=25, tol=tol, max_cycles=400,
                  precision="mixed", max_refine=30, inner_tol=1e-4)
    assert g.status == "ok", (g.status, g.refine_steps, g.true_relres)
    r = true_relres(A, g.X, B)
    assert r <= tol
    g64 = gpu_solve(A, B, method="gmres", skeleton="bcgsi_ls", m=25, tol=tol, max_cycles=4000)
    r64 = true_relres(A, g64.X, B)
    err = np.linalg.norm(g.X - g64.X) / np.linalg.norm(g64.X)
    print(f"mixed rgg: refinement steps {g.refine_steps}, inner block iterations {g.iters}, "
          f"FP64 block iterations {g64.iters}, true relres {r:.2e} / {r64:.2e}, "
          f"difference to FP64 solve {err:.2e}")
    assert g64.status == "ok"
    assert err <= 1e5 * (r + r64)
