"""Plain FP64 CPU oracle for the adaptively restarted block Krylov solvers
(BFOM / BGMRES with low-synchronization block Gram-Schmidt skeletons) of
K. Lund, "Adaptively restarted block Krylov subspace methods with
low-synchronization skeletons".

TEST INFRASTRUCTURE ONLY.  This package is a slow, obviously correct
restatement of the paper's algorithms in NumPy/SciPy, used to check the GPU
library.  Only the test-suite, the smoke entry point and the benchmark's
CPU-baseline leg may import it; the product path never does.  It shares no
code with the HIP library or its Python binding.

Modules:
  primitives -- block inner product, Cholesky with breakdown flag, CholQR, HouseQR
  skeletons  -- block Arnoldi skeletons (Algs. 2, 3, 5, 6, 7)
  solver     -- restarted BFOM / BGMRES driver with cospatial restarts and
                the adaptive restart heuristic (Secs. 2.4.1, 2.4.2, 4)
  precond    -- ILU(0) factors and their application, right preconditioning
                (Sec. 5, the tests on matrices from applications)

Every public function cites the passage of the paper it follows.  Readings
taken where the paper is silent or ambiguous are listed in the docstrings
of the functions that make them.
"""
from .primitives import ip, chol_flag, cholqr, houseqr, intra_ortho
from .skeletons import SKELETONS, make_skeleton
from .solver import solve, OracleResult, small_solve
from .precond import ilu0, ilu0_apply, ZeroPivot

__all__ = ["ip", "chol_flag", "cholqr", "houseqr", "intra_ortho", "SKELETONS",
           "make_skeleton", "solve", "OracleResult", "small_solve", "ilu0", "ilu0_apply",
           "ZeroPivot"]
