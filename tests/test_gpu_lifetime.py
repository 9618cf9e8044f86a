"""Handle lifetimes through the C ABI: an operator may be destroyed after its
context (a garbage collector may finalize them in either order); the context
then releases the operator's device memory and the later operator destroy
frees only the handle."""
import pytest

from paper_2208_09899_amd import lsba, workloads as w

pytestmark = pytest.mark.gpu


def test_operator_destroyed_after_its_context():
    lib = lsba.load()
    ctx = lsba.Context(0)
    op = lsba.Operator(ctx, w.laplace_1d(64))
    ctx.close()          # context first ...
    op.close()           # ... then the operator: must not touch the freed context
    # a fresh context still works afterwards
    ctx2 = lsba.Context(0)
    op2 = lsba.Operator(ctx2, w.laplace_1d(64))
    r = lsba.solve(ctx2, op2, w.rhs(64, 1, 3), m=10, tol=1e-10, max_cycles=20)
    assert r.status in ("ok", "not_converged") and r.iters > 0
    assert r.res_hist[-1] < 1e-2 * r.res_hist[0]
    op2.close()
    ctx2.close()
    assert lib is lsba.load()
