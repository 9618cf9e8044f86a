"""HouseQR muscle on the GPU (Householder TSQR, diag(R) >= 0) against the
oracle's HouseQR (LAPACK QR with the same sign fix): the factors are unique
for a full-rank block, so X, iteration counts, restart points and counts
must agree as for CholQR."""
import numpy as np
import pytest

from paper_2208_09899_amd import workloads as w

from gpu_common import pip_hist_atol, assert_parity, gpu_solve, oracle_solve

pytestmark = pytest.mark.gpu

SKELETONS = ["bcgsi_ls", "bmgs_svl", "bmgs_lts", "bmgs_cwy", "bmgs_icwy", "bcgs_pip", "bmgs", "bcgs_pio"]


@pytest.mark.parametrize("method", ["fom", "gmres"])
@pytest.mark.parametrize("skel", SKELETONS)
def test_houseqr_laplace2d_32(method, skel):
    wl = w.workload("laplace2d", 32)
    g = gpu_solve(wl.A, wl.B, method=method, skeleton=skel, muscle="houseqr", m=30, tol=1e-8,
                  max_cycles=1000)
    o = oracle_solve(wl.A, wl.B, method, skel, m=30, tol=1e-8, max_cycles=1000, muscle="houseqr")
    assert_parity(g, o, hist_atol=pip_hist_atol(440.0) if skel in ("bcgs_pip", "bcgs_pio") else 1e-12)


@pytest.mark.parametrize("skel", ["bcgsi_ls", "bmgs_svl", "bmgs_cwy"])
@pytest.mark.parametrize("s", [1, 3, 8, 16])
def test_houseqr_convdiff_ragged(skel, s):
    A = w.convdiff_2d(45, 3.0, 0.7)
    B = w.rhs(A.n, s, seed=21 + s)
    g = gpu_solve(A, B, method="gmres", skeleton=skel, muscle="houseqr", m=15, tol=1e-8,
                  max_cycles=2000)
    o = oracle_solve(A, B, "gmres", skel, m=15, tol=1e-8, max_cycles=2000, muscle="houseqr")
    assert_parity(g, o)


@pytest.mark.parametrize("s,skel", [(32, "bcgsi_ls"), (32, "bmgs_lts"), (8, "bmgs_svl")])
def test_houseqr_multilevel_tsqr(s, skel):
    """n = 65536: at s = 32 the TSQR has three stack levels above the row
    chunks, at s = 8 one; one restart cycle plus a few columns of the next."""
    A = w.laplace_2d(256)
    B = w.rhs(A.n, s, seed=31)
    g = gpu_solve(A, B, method="gmres", skeleton=skel, muscle="houseqr", m=6, tol=1e-12,
                  max_cycles=10, max_iters=9)
    o = oracle_solve(A, B, "gmres", skel, m=6, tol=1e-12, max_cycles=10, max_iters=9,
                     muscle="houseqr")
    assert_parity(g, o, hist_atol=1e-11)


@pytest.mark.parametrize("skel", ["bcgsi_ls", "bmgs_svl"])
def test_houseqr_rank_deficient_start_breaks_down(skel):
    """An exactly zero column gives an exactly zero diagonal entry of R: the
    flag at the cycle start ends the solve with a breakdown, as in the oracle."""
    A = w.laplace_2d(20)
    B = w.rhs(A.n, 4, seed=5)
    B[:, 2] = 0.0
    g = gpu_solve(A, B, method="gmres", skeleton=skel, muscle="houseqr", m=10, tol=1e-8)
    o = oracle_solve(A, B, "gmres", skel, m=10, tol=1e-8, muscle="houseqr")
    assert g.status == o.status == "breakdown"
    assert g.iters == o.iters == 0
    assert not np.any(np.asarray(g.X))


@pytest.mark.parametrize("skel", ["bmgs_svl", "bmgs_lts", "bcgsi_ls"])
def test_houseqr_forced_flag_adaptive_restart(skel):
    A = w.convdiff_2d(30, 1.0, 0.2)
    B = w.rhs(A.n, 4, seed=8)
    g = gpu_solve(A, B, method="gmres", skeleton=skel, muscle="houseqr", m=12, tol=1e-8,
                  max_cycles=500, force_flag=(1, 6))
    o = oracle_solve(A, B, "gmres", skel, m=12, tol=1e-8, max_cycles=500, force_flag=(1, 6),
                     muscle="houseqr")
    assert_parity(g, o)
    assert g.m_after[0] < 12
