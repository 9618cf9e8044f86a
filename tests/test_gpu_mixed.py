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


def test_mixed_kappa_1e6_graph_laplacian():
    """The precision form on an ill-conditioned operator of the random
    geometric graph class: n = 2^14 points, mean degree 8 (above the 2-D
    percolation threshold: 16 components, the largest 16355 nodes) + 1e-5 I.
    lambda_min is exactly the shift (the constant vector of each component)
    and lambda_max = 13.1, so kappa = 1.3e6.  BGMRES(25) with BCGSI+LS,
    s = 16: FP32 inner solves with u_32 kappa ~ 0.08 each win only about
    one digit, so refinement does the rest; the solve must reach a true
    relative residual of 1e-8.  Its error against a direct FP64 solution is
    formed by the library (lsba_result_err_vs_ref) and must satisfy the
    residual bound kappa r (plus the direct solve's own rounding)."""
    import scipy.sparse.linalg as sla
    A = w.rgg_laplacian(1 << 14, seed=3, degree=8.0, shift=1e-5)
    B = w.rhs(A.n, 16, seed=4)
    As = A.to_scipy().tocsc()
    X_ref = sla.spsolve(As, B)
    tol = 1e-8
    g = gpu_solve(A, B, method="gmres", skeleton="bcgsi_ls", m=25, tol=tol, max_cycles=3000,
                  precision="mixed", max_refine=40, inner_tol=1e-4, x_ref=X_ref)
    r = true_relres(A, g.X, B)
    print(f"mixed kappa 1.3e6: status {g.status}, refinement steps {g.refine_steps}, inner block "
          f"iterations {g.iters}, true relres {r:.2e}, error vs direct {g.err_vs_ref:.2e}")
    assert g.status == "ok", (g.status, g.refine_steps, g.true_relres)
    assert r <= tol
    kappa = 13.13 / 1e-5
    assert g.err_vs_ref <= kappa * (r + 1e-12)


@pytest.mark.parametrize("s", [16, 32])
def test_mixed_wide_blocks_keep_fp32_accuracy(s):
    """s = 16 and 32 take the FP32 Gram and update on the BF16 matrix cores
    with three-part splits.  Their products must keep FP32 accuracy: the
    inner solves' loss of orthogonality stays at the FP32 level (a product
    at bfloat16 accuracy, 2^-8, would leave it near 1e-2), and the refined
    solve needs about as many block iterations as the FP64 solve to the
    same tolerance.  3-D Laplacian 16^3, BGMRES(20) with BCGSI+LS."""
    A = w.laplace_3d(16)
    B = w.rhs(A.n, s, seed=21)
    tol = 1e-8
    g = gpu_solve(A, B, method="gmres", skeleton="bcgsi_ls", m=20, tol=tol, max_cycles=200,
                  precision="mixed", max_refine=20, inner_tol=1e-4, record_loo=True)
    g64 = gpu_solve(A, B, method="gmres", skeleton="bcgsi_ls", m=20, tol=tol, max_cycles=200)
    r = true_relres(A, g.X, B)
    loo = np.asarray(g.loo_hist)
    loo = loo[np.isfinite(loo)]
    print(f"mixed s={s}: refinement steps {g.refine_steps}, inner block iterations {g.iters}, "
          f"FP64 iterations {g64.iters}, true relres {r:.2e}, max LOO {loo.max():.2e}")
    assert g.status == "ok" and g64.status == "ok"
    assert r <= tol
    assert loo.size > 0 and loo.max() <= 1e-3
    assert g.iters <= 1.5 * g64.iters + 10
