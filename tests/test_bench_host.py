"""Host-side checks of the benchmark driver (no GPU): the one-GPU guard, the
workload table, the stored traffic records' match with the kernel sources,
and the CPU-baseline leg's fields."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2208_09899_amd import workloads as w  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


@pytest.mark.parametrize("name", sorted(bench.WORKLOADS))
def test_workload_table_builds_small_cases(name):
    entry = bench.WORKLOADS[name]
    key, _, solves, precision = entry[:4]
    assert precision in ("fp64", "mixed")
    assert all(m in ("fom", "gmres") for m, _ in solves)
    if len(entry) > 4:
        assert entry[4] == "ilu0"
    small = {"tridiag1000": 50, "laplace2d": 12, "rgg": 1 << 10, "laplace3d": 6,
             "convdiff2d": 12}[key]
    wl = w.workload(key, small)
    assert wl.B.shape[0] == wl.A.n and wl.A.nnz == int(wl.A.row_ptr[-1])


def test_stored_traffic_matches_current_kernel_sources():
    """The committed counter records apply only while the kernels they
    measured are unchanged: the default workload's record must match the
    current sources of the update, Gram and SpMM kernels."""
    rec = json.load(open(bench.traffic_file("laplace3d")))
    assert rec["workload"] == "laplace3d"
    for kind in ("update", "gram", "spmm"):
        k = bench.stored_traffic(kind, "laplace3d")
        assert k is not None, kind
        assert 1.0 <= k["traffic_over_alg"] <= 2.5
    assert bench.stored_traffic("precond", "laplace3d") is None


def test_cpu_baseline_fields_with_and_without_preconditioner():
    wl = w.workload("laplace2d", 12)
    for pre in (None, "ilu0"):
        cb = bench.cpu_baseline(wl, [("gmres", "bcgsi_ls")], [40], budget_s=0.5,
                                precond=pre)
        assert cb["kind"] == "oracle" and cb["unit"] == "solves/s"
        assert cb["value"] > 0 and cb["cores"] >= 1
        assert ("ILU(0)" in cb["sample"]) == (pre is not None)
