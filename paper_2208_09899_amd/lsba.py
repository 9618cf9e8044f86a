"""Python binding of liblsba (include/lsba.h): argument marshalling only.

Every step of a solve runs in the HIP library; this module converts Python
arguments (NumPy host arrays or torch CUDA tensors) into the C ABI's plain
pointers and sizes and copies the result arrays back.  It raises
``LibraryMissing`` when the built library is absent -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblsba.so")

METHODS = {"fom": 0, "gmres": 1}
SKELETONS = {"bcgsi_ls": 0, "bmgs_svl": 1, "bmgs_lts": 2, "bmgs_cwy": 3, "bmgs_icwy": 4,
             "bcgs_pip": 5, "bmgs": 6, "bcgs_pio": 7}
MUSCLES = {"cholqr": 0, "houseqr": 1, "global": 2, "mgs_svl": 3, "mgs_lts": 4}
PRECISIONS = {"fp64": 0, "mixed": 1}
REC_LOO, REC_TRUE_RES = 1, 2

STATUS = {0: "ok", 1: "not_converged", 2: "breakdown", -1: "err_arg", -2: "err_oom",
          -3: "err_hip", -4: "err_unsupported", -5: "err_busy"}

# Symbols declared in include/lsba.h
EXPORTS = [
    "lsba_params_default", "lsba_context_create", "lsba_context_destroy", "lsba_last_error",
    "lsba_status_string", "lsba_operator_create_csr", "lsba_operator_destroy", "lsba_solve",
    "lsba_result_status", "lsba_result_iters", "lsba_result_res_hist", "lsba_result_loo_hist",
    "lsba_result_cycles", "lsba_result_cycle_len", "lsba_result_m_after", "lsba_result_counts",
    "lsba_result_true_relres", "lsba_result_refine_steps", "lsba_result_gpu_ms",
    "lsba_result_destroy", "lsba_context_set_timing", "lsba_context_kernel_stats",
    "lsba_solve_footprint", "lsba_server_create", "lsba_server_submit", "lsba_server_poll",
    "lsba_server_fetch", "lsba_server_stats", "lsba_server_destroy", "lsba_context_set_graphs",
    "lsba_solve_noalloc", "lsba_context_kernel_flops", "lsba_result_set_err_vs_ref",
    "lsba_result_err_vs_ref", "lsba_precond_create_ilu0", "lsba_precond_destroy",
    "lsba_precond_apply", "lsba_precond_factors", "lsba_precond_info", "lsba_solve_precond",
]

KERNEL_KINDS = {"spmm": 0, "gram": 1, "gram_reduce": 2, "update": 3, "small": 4, "residual": 5,
                "precond": 6}
TIME_ALL = 0x7F


class LibraryMissing(RuntimeError):
    pass


class LsbaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("method", ctypes.c_int32),
        ("skeleton", ctypes.c_int32),
        ("muscle", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("max_cycles", ctypes.c_int32),
        ("max_iters", ctypes.c_int64),
        ("max_refine", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("record", ctypes.c_uint32),
        ("force_flag_cycle", ctypes.c_int32),
        ("force_flag_step", ctypes.c_int32),
    ]


_lib = None


def _init_torch_runtime_first():
    """PyTorch wheels for ROCm ship their own HIP and HSA runtimes, so a
    process that uses torch and this library holds two of each (device
    pointers are shared: both map the process's one GPU address space).  If
    the library's runtime opens the GPU first, torch's later initialisation
    can find no device; initialising torch's first makes either order of use
    work.  Nothing happens when torch is absent or sees no GPU."""
    try:
        import torch
    except ImportError:
        return
    try:
        if torch.cuda.is_available():
            torch.cuda.init()
    except Exception:
        pass


def load(path: str | None = None) -> ctypes.CDLL:
    """Load liblsba.so (built by ``paper_2208_09899_amd.build``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise LibraryMissing(f"{p} not found: build it with `python -m paper_2208_09899_amd.build`")
    _init_torch_runtime_first()
    lib = ctypes.CDLL(p)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "lsba_params_default": (i32, [ctypes.POINTER(Params)]),
        "lsba_context_create": (i32, [ctypes.c_int, vp, ctypes.POINTER(vp)]),
        "lsba_context_destroy": (None, [vp]),
        "lsba_last_error": (ctypes.c_char_p, [vp]),
        "lsba_status_string": (ctypes.c_char_p, [i32]),
        "lsba_operator_create_csr": (i32, [vp, i64, i64, vp, vp, vp, ctypes.c_int,
                                           ctypes.POINTER(vp)]),
        "lsba_operator_destroy": (None, [vp]),
        "lsba_solve": (i32, [vp, vp, ctypes.POINTER(Params), i32, vp, i64, vp, i64,
                             ctypes.c_int, ctypes.POINTER(vp)]),
        "lsba_solve_noalloc": (i32, [vp, vp, ctypes.POINTER(Params), i32, vp, i64, vp, i64,
                                     ctypes.POINTER(vp)]),
        "lsba_result_status": (i32, [vp]),
        "lsba_result_iters": (i64, [vp]),
        "lsba_result_res_hist": (ctypes.POINTER(dbl), [vp]),
        "lsba_result_loo_hist": (ctypes.POINTER(dbl), [vp]),
        "lsba_result_cycles": (i32, [vp]),
        "lsba_result_cycle_len": (ctypes.POINTER(i32), [vp]),
        "lsba_result_m_after": (ctypes.POINTER(i32), [vp]),
        "lsba_result_counts": (None, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64)]),
        "lsba_result_true_relres": (dbl, [vp]),
        "lsba_result_refine_steps": (i32, [vp]),
        "lsba_result_set_err_vs_ref": (i32, [vp, vp, i64, i32, vp, i64, vp, i64, ctypes.c_int]),
        "lsba_result_err_vs_ref": (dbl, [vp]),
        "lsba_result_gpu_ms": (dbl, [vp]),
        "lsba_result_destroy": (None, [vp]),
        "lsba_context_set_timing": (i32, [vp, ctypes.c_uint32]),
        "lsba_context_set_graphs": (i32, [vp, ctypes.c_int]),
        "lsba_context_kernel_stats": (i32, [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                            ctypes.POINTER(dbl)]),
        "lsba_context_kernel_flops": (i32, [vp, i32, ctypes.POINTER(dbl)]),
        "lsba_solve_footprint": (ctypes.c_uint64, [i64, i32, vp]),
        "lsba_server_create": (i32, [vp, ctypes.c_uint64, i32, ctypes.POINTER(vp)]),
        "lsba_server_submit": (i32, [vp, vp, vp, i32, vp, i64, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_uint64)]),
        "lsba_server_poll": (i32, [vp, ctypes.POINTER(ctypes.c_uint64), i32, ctypes.POINTER(i32)]),
        "lsba_server_fetch": (i32, [vp, ctypes.c_uint64, vp, i64, ctypes.c_int,
                                    ctypes.POINTER(vp)]),
        "lsba_server_stats": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(i32)]),
        "lsba_server_destroy": (None, [vp]),
        "lsba_precond_create_ilu0": (i32, [vp, vp, ctypes.POINTER(vp)]),
        "lsba_precond_destroy": (None, [vp]),
        "lsba_precond_apply": (i32, [vp, vp, i32, vp, i64, vp, i64, ctypes.c_int]),
        "lsba_precond_factors": (i32, [vp, vp, vp, vp]),
        "lsba_precond_info": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                    ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "lsba_solve_precond": (i32, [vp, vp, vp, ctypes.POINTER(Params), i32, vp, i64, vp, i64,
                                     ctypes.c_int, ctypes.POINTER(vp)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class Context:
    """A library context on one GPU.  ``stream``: a hipStream_t handle (int),
    ``"torch"`` for torch's current stream on ``device``, or None for a
    library-owned stream."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = load()
        if stream == "torch":
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        st = self.lib.lsba_context_create(device, ctypes.c_void_p(stream) if stream else None,
                                          ctypes.byref(h))
        if st != 0:
            raise LsbaError(st, self.lib.lsba_last_error(None).decode())
        self.h = h
        self.device = device

    def error(self) -> str:
        return self.lib.lsba_last_error(self.h).decode()

    def set_timing(self, enable: bool = True, kinds=None):
        """Time every kernel class (enable=True), the named classes (kinds, a
        subset of KERNEL_KINDS), or nothing (enable=False)."""
        if not enable:
            mask = 0
        elif kinds is None:
            mask = TIME_ALL
        else:
            mask = 0
            for k in kinds:
                mask |= 1 << KERNEL_KINDS[k]
        st = self.lib.lsba_context_set_timing(self.h, mask)
        if st != 0:
            raise LsbaError(st, self.error())

    def set_graphs(self, enable: bool = True):
        """Replay captured cycles (enable=True) or launch every kernel
        individually (enable=False, the default)."""
        st = self.lib.lsba_context_set_graphs(self.h, 1 if enable else 0)
        if st != 0:
            raise LsbaError(st, self.error())

    def kernel_stats(self) -> dict:
        """{kind: (launches, total_ms, total_algorithmic_bytes)} since timing was enabled."""
        out = {}
        for name, kind in KERNEL_KINDS.items():
            n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            self.lib.lsba_context_kernel_stats(self.h, kind, ctypes.byref(n), ctypes.byref(ms),
                                               ctypes.byref(by))
            out[name] = (n.value, ms.value, by.value)
        return out

    def kernel_flops(self) -> dict:
        """{kind: total algorithmic flops} of the timed launches since timing was enabled."""
        out = {}
        for name, kind in KERNEL_KINDS.items():
            f = ctypes.c_double()
            self.lib.lsba_context_kernel_flops(self.h, kind, ctypes.byref(f))
            out[name] = f.value
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.lsba_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """A CSR operator copied into device memory (``csr``: an object with
    ``n``, ``row_ptr`` (int64), ``col_idx`` (int32), ``values`` (float64) as
    NumPy arrays or torch CUDA tensors)."""

    def __init__(self, ctx: Context, csr):
        self.ctx = ctx
        rp, ci, va = csr.row_ptr, csr.col_idx, csr.values
        on_dev = _is_torch(rp)
        if on_dev:
            args = [ctypes.c_void_p(t.data_ptr()) for t in (rp, ci, va)]
            n, nnz = int(rp.numel()) - 1, int(ci.numel())
        else:
            rp = np.ascontiguousarray(rp, dtype=np.int64)
            ci = np.ascontiguousarray(ci, dtype=np.int32)
            va = np.ascontiguousarray(va, dtype=np.float64)
            self._keep = (rp, ci, va)
            args = [a.ctypes.data_as(ctypes.c_void_p) for a in (rp, ci, va)]
            n, nnz = rp.shape[0] - 1, ci.shape[0]
        h = ctypes.c_void_p()
        st = ctx.lib.lsba_operator_create_csr(ctx.h, n, nnz, *args, 1 if on_dev else 0,
                                              ctypes.byref(h))
        if st != 0:
            raise LsbaError(st, ctx.error())
        self.h = h
        self.n = n
        self.nnz = nnz

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.lsba_operator_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Precond:
    """ILU(0) factors of an operator's matrix, computed on the device
    (lsba_precond_create_ilu0); pass as ``precond=`` to ``solve`` for right
    preconditioning."""

    def __init__(self, ctx: Context, op: Operator):
        self.ctx = ctx
        h = ctypes.c_void_p()
        st = ctx.lib.lsba_precond_create_ilu0(ctx.h, op.h, ctypes.byref(h))
        if st != 0:
            raise LsbaError(st, ctx.error())
        self.h = h
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        lo, up = ctypes.c_int32(), ctypes.c_int32()
        ctx.lib.lsba_precond_info(h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(lo),
                                  ctypes.byref(up))
        self.n, self.nnz = n.value, nnz.value
        self.levels = (lo.value, up.value)

    def factors(self):
        """(row_ptr, col_idx, values) of the factors on A's pattern, columns
        ascending: left of the diagonal L's multipliers, the rest U."""
        rp = np.empty(self.n + 1, dtype=np.int64)
        ci = np.empty(self.nnz, dtype=np.int32)
        va = np.empty(self.nnz, dtype=np.float64)
        st = self.ctx.lib.lsba_precond_factors(self.h, rp.ctypes.data_as(ctypes.c_void_p),
                                               ci.ctypes.data_as(ctypes.c_void_p),
                                               va.ctypes.data_as(ctypes.c_void_p))
        if st != 0:
            raise LsbaError(st, self.ctx.error())
        return rp, ci, va

    def apply(self, Y, Z=None):
        """Z = U^{-1} L^{-1} Y (NumPy n x s, or torch CUDA tensors)."""
        on_dev = _is_torch(Y)
        if on_dev:
            assert Y.stride(1) == 1
            if Z is None:
                import torch
                Z = torch.empty_like(Y)
            yp, ly = ctypes.c_void_p(Y.data_ptr()), Y.stride(0)
            zp, lz = ctypes.c_void_p(Z.data_ptr()), Z.stride(0)
            s = Y.shape[1]
        else:
            Y = np.ascontiguousarray(Y, dtype=np.float64)
            s = Y.shape[1]
            if Z is None:
                Z = np.empty_like(Y)
            yp, ly = Y.ctypes.data_as(ctypes.c_void_p), s
            zp, lz = Z.ctypes.data_as(ctypes.c_void_p), s
        st = self.ctx.lib.lsba_precond_apply(self.ctx.h, self.h, s, yp, ly, zp, lz,
                                             1 if on_dev else 0)
        if st != 0:
            raise LsbaError(st, self.ctx.error())
        return Z

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.lsba_precond_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class Result:
    status: str
    X: object
    iters: int
    res_hist: np.ndarray
    loo_hist: np.ndarray | None
    cycle_len: list
    m_after: list
    counts: tuple
    true_relres: float
    refine_steps: int
    gpu_ms: float
    err_vs_ref: float = float("nan")


def make_params(method="gmres", skeleton="bcgsi_ls", muscle="cholqr", precision="fp64", m=20,
                tol=1e-8, max_cycles=50, max_iters=0, max_refine=20, inner_tol=1e-4,
                record_loo=False, true_res=False, force_flag=None) -> Params:
    lib = load()
    p = Params()
    lib.lsba_params_default(ctypes.byref(p))
    p.method = METHODS[method]
    p.skeleton = SKELETONS[skeleton]
    p.muscle = MUSCLES[muscle]
    p.precision = PRECISIONS[precision]
    p.m = m
    p.tol = tol
    p.max_cycles = max_cycles
    p.max_iters = max_iters
    p.max_refine = max_refine
    p.inner_tol = inner_tol
    p.record = (REC_LOO if record_loo else 0) | (REC_TRUE_RES if true_res else 0)
    if force_flag is not None:
        p.force_flag_cycle, p.force_flag_step = force_flag
    return p


def solve(ctx: Context, op: Operator, B, X=None, x_ref=None, precond: Precond | None = None,
          **kw) -> Result:
    """Solve A X = B (B: n x s, row-major NumPy array or torch CUDA tensor).
    Keyword arguments are those of ``make_params``.  ``x_ref``: a reference
    solution (same kind of array as B, e.g. the FP64 oracle's X); the result
    then carries ||X - x_ref||_F / ||x_ref||_F, formed by the library.
    ``precond``: ILU(0) factors for right preconditioning (lsba_solve_precond)."""
    lib = ctx.lib
    p = make_params(**kw)
    on_dev = _is_torch(B)
    if on_dev:
        import torch
        assert B.dtype == torch.float64 and B.dim() == 2
        n, s = B.shape
        ldb = B.stride(0)
        assert B.stride(1) == 1
        if X is None:
            X = torch.empty_like(B)
        bptr, xptr, ldx = ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()), X.stride(0)
    else:
        B = np.ascontiguousarray(B, dtype=np.float64)
        n, s = B.shape
        ldb = s
        if X is None:
            X = np.empty_like(B)
        bptr, xptr, ldx = B.ctypes.data_as(ctypes.c_void_p), X.ctypes.data_as(ctypes.c_void_p), s
    h = ctypes.c_void_p()
    if precond is None:
        st = lib.lsba_solve(ctx.h, op.h, ctypes.byref(p), s, bptr, ldb, xptr, ldx,
                            1 if on_dev else 0, ctypes.byref(h))
    else:
        st = lib.lsba_solve_precond(ctx.h, op.h, precond.h, ctypes.byref(p), s, bptr, ldb, xptr,
                                    ldx, 1 if on_dev else 0, ctypes.byref(h))
    if st < 0:
        raise LsbaError(st, ctx.error())
    if x_ref is not None:
        if on_dev:
            assert x_ref.shape == B.shape and x_ref.stride(1) == 1
            rptr, ldr = ctypes.c_void_p(x_ref.data_ptr()), x_ref.stride(0)
        else:
            x_ref = np.ascontiguousarray(x_ref, dtype=np.float64)
            rptr, ldr = x_ref.ctypes.data_as(ctypes.c_void_p), s
        st2 = lib.lsba_result_set_err_vs_ref(ctx.h, h, n, s, xptr, ldx, rptr, ldr,
                                             1 if on_dev else 0)
        if st2 < 0:
            lib.lsba_result_destroy(h)
            raise LsbaError(st2, ctx.error())
    return _take_result(lib, h, X)


def solve_noalloc(ctx: Context, op: Operator, B, X=None, **kw) -> Result:
    """lsba_solve_noalloc: solve A X = B with the library's fixed device
    workspace (B: n x s float64 torch CUDA tensor, row-major rows)."""
    import torch
    lib = ctx.lib
    p = make_params(**kw)
    assert _is_torch(B) and B.dtype == torch.float64 and B.dim() == 2 and B.stride(1) == 1
    n, s = B.shape
    if X is None:
        X = torch.empty_like(B)
    h = ctypes.c_void_p()
    st = lib.lsba_solve_noalloc(ctx.h, op.h, ctypes.byref(p), s, ctypes.c_void_p(B.data_ptr()),
                                B.stride(0), ctypes.c_void_p(X.data_ptr()), X.stride(0),
                                ctypes.byref(h))
    if st < 0:
        raise LsbaError(st, ctx.error())
    return _take_result(lib, h, X)


def _take_result(lib, h, X) -> Result:
    """Read a library result into a Result and destroy the handle."""
    try:
        it = lib.lsba_result_iters(h)
        rp = lib.lsba_result_res_hist(h)
        res = np.array(rp[:it], dtype=np.float64) if it and rp else np.zeros(0)
        lp = lib.lsba_result_loo_hist(h)
        loo = np.array(lp[:it], dtype=np.float64) if (it and lp) else None
        nc = lib.lsba_result_cycles(h)
        cl = lib.lsba_result_cycle_len(h)
        ma = lib.lsba_result_m_after(h)
        a, v, sy = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        lib.lsba_result_counts(h, ctypes.byref(a), ctypes.byref(v), ctypes.byref(sy))
        return Result(status=STATUS[lib.lsba_result_status(h)], X=X, iters=it, res_hist=res,
                      loo_hist=loo, cycle_len=list(cl[:nc]) if nc else [],
                      m_after=list(ma[:nc]) if nc else [], counts=(a.value, v.value, sy.value),
                      true_relres=lib.lsba_result_true_relres(h),
                      refine_steps=lib.lsba_result_refine_steps(h),
                      gpu_ms=lib.lsba_result_gpu_ms(h),
                      err_vs_ref=lib.lsba_result_err_vs_ref(h))
    finally:
        lib.lsba_result_destroy(h)


def footprint(n: int, s: int, **kw) -> int:
    """Device bytes a solve of an n-row operator with s right-hand sides holds."""
    p = make_params(**kw)
    return int(load().lsba_solve_footprint(n, s, ctypes.byref(p)))


class Server:
    """Continuous batching of FP64 solves on one device (see lsba_server_* in
    include/lsba.h): submit() queues a request, poll() advances every running
    request by the cycles whose device work has completed and admits queued
    ones within the byte budget, fetch() returns a finished request's result."""

    def __init__(self, ctx: Context, budget_bytes: int, max_slots: int = 8):
        self.ctx = ctx
        self.lib = ctx.lib
        h = ctypes.c_void_p()
        st = self.lib.lsba_server_create(ctx.h, int(budget_bytes), int(max_slots), ctypes.byref(h))
        if st != 0:
            raise LsbaError(st, ctx.error())
        self.h = h
        self._shape = {}

    def submit(self, op: Operator, B, **kw) -> int:
        p = make_params(**kw)
        B = np.ascontiguousarray(B, dtype=np.float64)
        n, s = B.shape
        t = ctypes.c_uint64()
        st = self.lib.lsba_server_submit(self.h, op.h, ctypes.byref(p), s,
                                         B.ctypes.data_as(ctypes.c_void_p), s, 0, ctypes.byref(t))
        if st != 0:
            raise LsbaError(st, self.ctx.error())
        self._shape[t.value] = (n, s)
        return t.value

    def poll(self, cap: int = 256) -> list:
        buf = (ctypes.c_uint64 * cap)()
        k = ctypes.c_int32()
        st = self.lib.lsba_server_poll(self.h, buf, cap, ctypes.byref(k))
        if st != 0:
            raise LsbaError(st, self.ctx.error())
        return [int(buf[i]) for i in range(k.value)]

    def fetch(self, ticket: int) -> Result:
        n, s = self._shape[ticket]
        X = np.empty((n, s), dtype=np.float64)
        h = ctypes.c_void_p()
        st = self.lib.lsba_server_fetch(self.h, ticket, X.ctypes.data_as(ctypes.c_void_p), s, 0,
                                        ctypes.byref(h))
        if st < 0:
            raise LsbaError(st, self.ctx.error())
        del self._shape[ticket]
        return _take_result(self.lib, h, X)

    def stats(self) -> dict:
        a, q, pk = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        b = ctypes.c_uint64()
        self.lib.lsba_server_stats(self.h, ctypes.byref(a), ctypes.byref(q), ctypes.byref(b),
                                   ctypes.byref(pk))
        return {"active": a.value, "queued": q.value, "bytes_in_use": b.value,
                "peak_active": pk.value}

    def close(self):
        if getattr(self, "h", None):
            self.lib.lsba_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
