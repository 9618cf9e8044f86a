"""The serving form: continuous batching of independent BGMRES solves.

A request computes exactly what a standalone solve computes (same kernels,
fixed-order reductions), so its X, history and counts must be identical
whether it runs alone or admitted beside others; the admission rule (free
slot and summed footprints within the byte budget) must hold at every
moment."""
import time

import numpy as np
import pytest

from paper_2208_09899_amd import lsba, workloads as w

from gpu_common import ctx, gpu_solve

pytestmark = pytest.mark.gpu

PARAMS = dict(method="gmres", skeleton="bcgsi_ls", m=20, tol=1e-8, max_cycles=500)


def small_stream(count, seed=6):
    """Requests shaped like the serving stream, at grid sides 24..72."""
    return w.serving_stream(count=count, rate=1000.0, seed=seed, side_lo=24, side_hi=72)


def drain(srv, tickets, timeout_s=120.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in srv.poll():
            done[t] = srv.fetch(t)
        assert time.time() - t0 < timeout_s, "serving loop made no progress"
    return done


def test_each_result_same_alone_and_in_the_mix():
    reqs = small_stream(10)
    problems = [w.request_problem(r) for r in reqs]
    alone = [gpu_solve(A, B, **PARAMS) for A, B in problems]
    ops = [lsba.Operator(ctx(), A) for A, _ in problems]
    srv = lsba.Server(ctx(), budget_bytes=8 << 30, max_slots=4)
    try:
        tickets = [srv.submit(op, B, **PARAMS) for op, (_, B) in zip(ops, problems)]
        done = drain(srv, tickets)
        assert srv.stats()["peak_active"] >= 2      # requests did overlap
    finally:
        srv.close()
        for op in ops:
            op.close()
    for t, a, (A, B) in zip(tickets, alone, problems):
        g = done[t]
        assert g.status == a.status == "ok"
        assert g.iters == a.iters and g.cycle_len == a.cycle_len
        assert tuple(g.counts) == tuple(a.counts)
        assert np.array_equal(np.asarray(g.X), np.asarray(a.X))
        assert np.array_equal(g.res_hist, a.res_hist)
        relres = np.linalg.norm(B - A.to_scipy() @ g.X) / np.linalg.norm(B)
        assert relres <= 1.01e-8 + 1e-12


def test_admission_respects_the_byte_budget():
    reqs = small_stream(8, seed=7)
    problems = [w.request_problem(r) for r in reqs]
    fps = [lsba.footprint(A.n, B.shape[1], **PARAMS) for A, B in problems]
    budget = 2 * max(fps)                      # at most two of the largest at once
    ops = [lsba.Operator(ctx(), A) for A, _ in problems]
    srv = lsba.Server(ctx(), budget_bytes=budget, max_slots=8)
    try:
        tickets = [srv.submit(op, B, **PARAMS) for op, (_, B) in zip(ops, problems)]
        done = {}
        t0 = time.time()
        while len(done) < len(tickets):
            st = srv.stats()
            assert st["bytes_in_use"] <= budget
            for t in srv.poll():
                done[t] = srv.fetch(t)
            assert time.time() - t0 < 120.0
        assert all(r.status == "ok" for r in done.values())
        assert srv.stats()["bytes_in_use"] == 0
    finally:
        srv.close()
        for op in ops:
            op.close()


def test_oversized_request_and_early_fetch():
    A = w.convdiff_2d(40, 2.0, 0.3)
    B = w.rhs(A.n, 8, seed=3)
    op = lsba.Operator(ctx(), A)
    fp = lsba.footprint(A.n, 8, **PARAMS)
    small = lsba.Server(ctx(), budget_bytes=fp - 1, max_slots=2)
    try:
        with pytest.raises(lsba.LsbaError):
            small.submit(op, B, **PARAMS)        # can never be admitted: LSBA_ERR_OOM
    finally:
        small.close()
    srv = lsba.Server(ctx(), budget_bytes=fp, max_slots=1)
    try:
        t = srv.submit(op, B, **PARAMS)
        with pytest.raises(lsba.LsbaError):
            srv.fetch(t)                         # not finished yet: LSBA_ERR_BUSY
        r = drain(srv, [t])[t]
        assert r.status == "ok"
    finally:
        srv.close()
        op.close()
