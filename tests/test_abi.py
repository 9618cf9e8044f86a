"""The C-ABI library loads and exports every function include/lsba.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2208_09899_amd import lsba

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "lsba.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lsba_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libh():
    if not os.path.exists(lsba.LIB_PATH):
        pytest.fail("liblsba.so is not built: run `python -m paper_2208_09899_amd.build`")
    return lsba.load()


def test_header_and_binding_agree():
    assert _declared() == sorted(lsba.EXPORTS)


def test_library_exports_every_declared_symbol(libh):
    for name in _declared():
        assert hasattr(libh, name), name


def test_params_default_and_status_strings(libh):
    p = lsba.Params()
    assert libh.lsba_params_default(ctypes.byref(p)) == 0
    assert p.struct_size == ctypes.sizeof(lsba.Params)
    assert (p.method, p.skeleton, p.muscle, p.precision, p.m) == (1, 0, 0, 0, 20)
    assert p.tol == 1e-8 and p.max_cycles == 50 and p.force_flag_step == -1
    assert libh.lsba_params_default(None) == -1
    for st in range(-5, 3):
        assert libh.lsba_status_string(st)


def test_null_handles_are_rejected(libh):
    assert libh.lsba_context_create(0, None, None) == -1
    assert libh.lsba_solve(None, None, None, 1, None, 1, None, 1, 0, None) == -1
    assert libh.lsba_operator_create_csr(None, 1, 0, None, None, None, 0, None) == -1
    # getters tolerate a NULL result
    assert libh.lsba_result_iters(None) == 0
    libh.lsba_result_destroy(None)
    libh.lsba_context_destroy(None)
    libh.lsba_operator_destroy(None)
    assert libh.lsba_precond_create_ilu0(None, None, None) == -1
    assert libh.lsba_precond_apply(None, None, 1, None, 1, None, 1, 0) == -1
    assert libh.lsba_precond_factors(None, None, None, None) == -1
    assert libh.lsba_precond_info(None, None, None, None, None) == -1
    assert libh.lsba_solve_precond(None, None, None, None, 1, None, 1, None, 1, 0, None) == -1
    libh.lsba_precond_destroy(None)


def test_params_struct_layout_matches_header():
    # field order and types of lsba_params (x86-64 SysV layout)
    offs = {name: getattr(lsba.Params, name).offset for name, _ in lsba.Params._fields_}
    assert offs["tol"] == 24 and offs["max_iters"] == 40 and offs["inner_tol"] == 56
    assert ctypes.sizeof(lsba.Params) == 80


def test_solve_footprint_counts_the_basis(lib):
    """lsba_solve_footprint is host-only arithmetic: at least B, X, U, W and the
    m + 1 basis blocks, growing with n, s and m; invalid shapes give 0."""
    from paper_2208_09899_amd import lsba
    n, s, m = 10000, 8, 20
    fp = lsba.footprint(n, s, m=m)
    assert fp >= (m + 1 + 4) * n * s * 8
    assert lsba.footprint(2 * n, s, m=m) > fp
    assert lsba.footprint(n, 2 * s, m=m) > fp
    assert lsba.footprint(n, s, m=m + 5) > fp
    assert lsba.footprint(n, 33, m=m) == 0
