import os
import sys

# The oracle works on small dense blocks; BLAS threading only adds overhead there.
for _v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-only oracle checks")


@pytest.fixture(scope="session")
def lib():
    """The loaded C-ABI library (product path).  GPU tests only."""
    from paper_2208_09899_amd import lsba
    return lsba.load()
