"""The host side of the ILU(0) preconditioner on the CPU: the sorted pattern,
the dependency levels of both sweeps, their level-order layout (with the
padded copy of the first entries) and the launch plans for every lane count
and for the factorization, checked by `tests/ilu_plan_check.cpp` built with
g++ against the library's own header (`csrc/ilu_plan.h`).  The checker
verifies that every row depends only on rows of earlier levels and sits at
the lowest such level, that the plans tile the levels, that a chained run
fits one workgroup (rows times lanes, columns per lane, levels per run) and
that one-level launches cover their rows; and that invalid patterns are
rejected with their reason."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2208_09899_amd import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2208_09899_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "ilu_plan_check.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.fail("g++ is needed to build the ILU(0) plan checker")
    exe = str(tmp_path_factory.mktemp("ilu_plan") / "ilu_plan_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC, SRC, "-o", exe],
                   check=True, capture_output=True, text=True)
    return exe


def _run(checker, tmp_path, n, rp, ci):
    path = tmp_path / "pattern.bin"
    with open(path, "wb") as f:
        np.array([n, len(ci)], dtype=np.int64).tofile(f)
        np.asarray(rp, dtype=np.int64).tofile(f)
        np.asarray(ci, dtype=np.int32).tofile(f)
    p = subprocess.run([checker, str(path)], capture_output=True, text=True, timeout=120)
    return p.returncode, p.stdout.strip()


def _csr(M):
    M = sp.csr_matrix(M)
    return M.shape[0], M.indptr, M.indices


def _shuffled(n, seed):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=6.0 / n, random_state=rng, format="csr") + sp.identity(n)
    M = sp.csr_matrix(M)
    rp, ci = M.indptr.copy(), M.indices.copy()
    for i in range(n):
        a, b = rp[i], rp[i + 1]
        ci[a:b] = ci[a:b][rng.permutation(b - a)]
    return n, rp, ci


def _bidiag(n, lower):
    M = sp.diags([np.ones(n), np.ones(n - 1)], [0, -1 if lower else 1], format="csr")
    return _csr(M)


CASES = {
    "laplace2d_64": lambda: _csr(w.laplace_2d(64).to_scipy()),
    "laplace3d_24": lambda: _csr(w.laplace_3d(24).to_scipy()),
    "convdiff_40": lambda: _csr(w.convdiff_2d(40, 8.0, 0.4).to_scipy()),
    "rgg_2pow16": lambda: _csr(w.rgg_laplacian(1 << 16, seed=3, degree=4.0).to_scipy()),
    "random_shuffled_3000": lambda: _shuffled(3000, 7),
    "lower_bidiagonal_5000": lambda: _bidiag(5000, True),
    "upper_bidiagonal_5000": lambda: _bidiag(5000, False),
    "diagonal_1000": lambda: _csr(sp.identity(1000, format="csr")),
    "full_40": lambda: _csr(np.ones((40, 40))),
    "one_row": lambda: (1, np.array([0, 1]), np.array([0])),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_ilu_host_analysis_invariants(checker, tmp_path, case):
    n, rp, ci = CASES[case]()
    rc, out = _run(checker, tmp_path, n, rp, ci)
    assert rc == 0 and out.startswith("OK"), out
    lo, up = (int(x) for x in out.split()[1:3])
    if case.endswith("bidiagonal_5000"):
        # one sweep is a chain of 5000 single-row levels (three chained runs)
        assert sorted((lo, up)) == [1, 5000]
    if case == "laplace2d_64":
        assert lo == up == 127          # the grid's anti-diagonals
    if case == "full_40":
        assert lo == up == 40


def test_ilu_host_analysis_rejects_bad_patterns(checker, tmp_path):
    # row 1 stores no diagonal entry
    rc, out = _run(checker, tmp_path, 2, [0, 2, 3], [0, 1, 0])
    assert rc == 0 and out == "ERROR row 1 stores no diagonal entry", out
    # row 0 stores column 1 twice
    rc, out = _run(checker, tmp_path, 2, [0, 3, 4], [1, 0, 1, 1])
    assert rc == 0 and out == "ERROR row 0 stores column 1 twice", out
