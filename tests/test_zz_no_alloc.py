"""lsba_solve_noalloc (the entry point that allocates no device memory)
against lsba_solve through the C ABI: two calls in a row, the second on a
smaller problem, each bitwise equal to lsba_solve on the same inputs (same
kernels and launch shapes, fixed-order reductions; only the workspace
addresses differ).  Also: a problem beyond the fixed workspace is rejected."""
import numpy as np
import pytest

from paper_2208_09899_amd import lsba, workloads as w

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert a.status == b.status
    assert a.iters == b.iters
    assert list(a.cycle_len) == list(b.cycle_len)
    assert list(a.m_after) == list(b.m_after)
    assert tuple(a.counts) == tuple(b.counts)
    assert np.array_equal(np.asarray(a.res_hist), np.asarray(b.res_hist))
    assert a.true_relres == b.true_relres


def test_noalloc_matches_solve_twice_then_smaller():
    import torch
    torch.cuda.set_device(0)
    ctx = lsba.Context(0)
    cases = [
        # (operator, s, params): tridiag n = 1000, s = 4, m = 20 (the small
        # BGMRES workload), then a smaller 2-D problem with another skeleton
        (w.laplace_1d(1000), 4, dict(method="gmres", skeleton="bcgsi_ls", m=20, tol=1e-8,
                                     max_cycles=50, true_res=True)),
        (w.laplace_2d(17), 2, dict(method="fom", skeleton="bmgs_cwy", m=10, tol=1e-10,
                                   max_cycles=200, true_res=True)),
    ]
    try:
        for (A, s, kw), status in zip(cases, ("not_converged", "ok")):
            op = lsba.Operator(ctx, A)
            try:
                B = torch.from_numpy(w.rhs(A.n, s, 7)).cuda()
                X1 = torch.full_like(B, np.nan)
                X2 = torch.full_like(B, np.nan)
                r_ref = lsba.solve(ctx, op, B, X=X1, **kw)
                r_na = lsba.solve_noalloc(ctx, op, B, X=X2, **kw)
                torch.cuda.synchronize()
                _same(r_na, r_ref)
                assert torch.equal(X1, X2)
                # restarted BGMRES(20) on tridiag(-1, 2, -1), n = 1000 (kappa ~ 4e5)
                # reaches the 50-cycle cap; the 2-D problem converges
                assert r_na.status == status
            finally:
                op.close()
    finally:
        ctx.close()


def test_noalloc_rejects_problem_beyond_workspace():
    import torch
    torch.cuda.set_device(0)
    ctx = lsba.Context(0)
    try:
        A = w.laplace_1d(1 << 18)
        op = lsba.Operator(ctx, A)
        try:
            B = torch.ones((A.n, 32), dtype=torch.float64, device="cuda")
            with pytest.raises(lsba.LsbaError) as ei:
                lsba.solve_noalloc(ctx, op, B, m=20)
            assert ei.value.status == -1
            assert "workspace" in str(ei.value)
        finally:
            op.close()
    finally:
        ctx.close()
