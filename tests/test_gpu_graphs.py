"""Captured cycles: replaying a cycle's hipGraph gives bitwise the results of
launching its kernels one by one, on every replay.

Each case solves once with individual launches, then several times with
graph replay (later solves reuse the graphs the first one captured), with
eager work and synchronisations of the program's own between the replays."""
import numpy as np
import pytest

from paper_2208_09899_amd import lsba, workloads as w

from gpu_common import ctx

pytestmark = pytest.mark.gpu

CASES = [
    dict(method="gmres", skeleton="bcgsi_ls"),
    dict(method="fom", skeleton="bmgs_cwy"),
    dict(method="gmres", skeleton="bmgs_icwy"),
    dict(method="gmres", skeleton="bmgs_svl"),
    dict(method="fom", skeleton="bmgs_lts", muscle="houseqr"),
    dict(method="gmres", skeleton="bcgsi_ls", precision="mixed"),
    # a forced Cholesky flag shortens one cycle: a second graph (restart length j)
    dict(method="gmres", skeleton="bcgsi_ls", force_flag=(2, 11)),
    dict(method="gmres", skeleton="bmgs_svl", record_loo=True),
]


def _same(a, b):
    assert a.status == b.status and a.iters == b.iters
    assert list(a.cycle_len) == list(b.cycle_len) and list(a.m_after) == list(b.m_after)
    assert tuple(a.counts) == tuple(b.counts)
    assert np.array_equal(np.asarray(a.X), np.asarray(b.X))
    assert np.array_equal(a.res_hist, b.res_hist)
    assert (a.loo_hist is None) == (b.loo_hist is None)
    if a.loo_hist is not None:
        assert np.array_equal(a.loo_hist, b.loo_hist, equal_nan=True)


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(str(v) for v in c.values()))
def test_replay_matches_individual_launches(case):
    A = w.convdiff_2d(40, 2.0, 0.3)
    B = w.rhs(A.n, 4, seed=11)
    kw = dict(m=12, tol=1e-8, max_cycles=300, **case)
    c = ctx()
    op = lsba.Operator(c, A)
    try:
        c.set_graphs(False)
        ref = lsba.solve(c, op, B, **kw)
        assert ref.status in ("ok", "breakdown")
        c.set_graphs(True)
        for rep in range(3):
            g = lsba.solve(c, op, B, **kw)
            _same(g, ref)
            # eager work of the program's own between replays
            e = lsba.solve(c, op, 2.0 * B, method="gmres", skeleton="bcgsi_ls", m=7, tol=1e-6,
                           max_cycles=300)
            assert e.status == "ok"
    finally:
        c.set_graphs(False)
        op.close()


def test_graphs_survive_a_workspace_reallocation():
    """A larger solve frees and reallocates the cached buffers; the graphs
    captured before are dropped, and the smaller solve still replays right."""
    c = ctx()
    small, big = w.convdiff_2d(32, 1.0, 0.2), w.convdiff_2d(64, 1.0, 0.2)
    Bs, Bb = w.rhs(small.n, 4, seed=1), w.rhs(big.n, 8, seed=2)
    kw = dict(method="gmres", skeleton="bmgs_cwy", m=10, tol=1e-8, max_cycles=300)
    ops = lsba.Operator(c, small)
    opb = lsba.Operator(c, big)
    try:
        c.set_graphs(False)
        ref_s = lsba.solve(c, ops, Bs, **kw)
        ref_b = lsba.solve(c, opb, Bb, **kw)
        c.set_graphs(True)
        for _ in range(2):
            _same(lsba.solve(c, ops, Bs, **kw), ref_s)
            _same(lsba.solve(c, opb, Bb, **kw), ref_b)
    finally:
        c.set_graphs(False)
        ops.close()
        opb.close()
