"""Thin Python binding of libboys.so (argument marshalling only).

Every function here checks tensor shapes, dtypes and devices, passes raw
device pointers and the current torch stream to the C-ABI entry point of the
same name, and raises :class:`BoysError` on a non-zero status.  All arithmetic
runs in the library's HIP kernels; there is no fallback: if libboys.so is
missing or the device is not gfx950 the call fails.
"""
from __future__ import annotations

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libboys.so")
_lib = None

F64_KMAX = 32        # the paper's tables: every FP64 entry point
F64_KMAX_EVAL = 40   # boys_eval_f64(_tol): orders 33..40 use the high-order tables
F64_KMAX_BACKWARD = 39  # boys_backward recomputes order kmax+1 <= 40
F32_KMAX = 16

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_INT = ctypes.c_int

_SIGNATURES = {
    "boys_strerror": ([_INT], ctypes.c_char_p),
    "boys_last_hip_error": ([], _INT),
    "boys_eval_f64": ([_P, _I64, _INT, _P, _I64, _P], _INT),
    "boys_eval_f64_tol": ([_P, _I64, _INT, ctypes.c_double, _P, _I64, _P], _INT),
    "boys_eval_f32": ([_P, _I64, _INT, _P, _I64, _P], _INT),
    "boys_weighted_sum": ([_P, _P, _P, _P, _P, _P, _I32, _P, _P], _INT),
    "boys_weighted_sum_tol": ([_P, _P, _P, _P, _P, _P, _I32, ctypes.c_double, _P, _P], _INT),
    "boys_weighted_sum_noalloc": ([_P, _P, _P, _P, _P, _P, _I32, _P, _P], _INT),
    "boys_backward_tol": ([_P, _P, _I64, _INT, _I64, ctypes.c_double, _P, _P], _INT),
    "boys_tune_weighted_sum": ([_P, _P, _P, _P, _P, _P, _I32, _P, _P,
                                ctypes.POINTER(_INT), ctypes.POINTER(ctypes.c_float)], _INT),
    "boys_weighted_sum_num_configs": ([], _INT),
    "boys_weighted_sum_config_name": ([_INT], ctypes.c_char_p),
    "boys_weighted_sum_get_config": ([], _INT),
    "boys_weighted_sum_set_config": ([_INT], _INT),
    "boys_backward": ([_P, _P, _I64, _INT, _I64, _P, _P], _INT),
    "boys_pairsum": ([_P, _P, _I64, _P, _INT, _P, _P], _INT),
    "boys_pairsum_tol": ([_P, _P, _I64, _P, _INT, ctypes.c_double, _P, _P], _INT),
    "boys_finalize": ([], None),
    "boys_set_tables": ([_INT], _INT),
    "boys_get_tables": ([], _INT),
}

# Variants of the 5e-14 tables for orders up to 32 (boys_set_tables).
TABLES_PAPER = 0
TABLES_PER_KMAX = 1
TABLES_CENTRE = 2


class BoysError(RuntimeError):
    pass


def library_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded libboys.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise BoysError(f"{_LIB_PATH} is not built (run __graft_entry__.build()); "
                            "there is no CPU fallback")
        handle = ctypes.CDLL(_LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(handle, name, None)
            if fn is None:
                continue
            fn.argtypes = args
            fn.restype = res
        _lib = handle
    return _lib


def _check(status: int, name: str):
    if status != 0:
        L = lib()
        msg = L.boys_strerror(status).decode()
        raise BoysError(f"{name} failed: {msg} (status {status}, hip error {L.boys_last_hip_error()})")


def _ptr(t: torch.Tensor):
    return _P(t.data_ptr())


def _stream(dev: torch.device):
    return _P(torch.cuda.current_stream(dev).cuda_stream)


def _vector(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise BoysError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise BoysError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 1 or not t.is_contiguous():
        raise BoysError(f"{name} must be a contiguous 1-D tensor")


def _rows(out: torch.Tensor, n: int, ncol: int, dtype, device, name: str) -> int:
    """Validates an (n, >= ncol) row-major output and returns its row stride."""
    if not out.is_cuda or out.device != device or out.dtype != dtype:
        raise BoysError(f"{name} must be a {dtype} tensor on {device}")
    if out.dim() != 2 or out.shape[0] != n or out.shape[1] < ncol or (n > 0 and out.stride(1) != 1):
        raise BoysError(f"{name} must have shape ({n}, >={ncol}) with unit column stride")
    if n > 1 and out.stride(0) < ncol:
        raise BoysError(f"{name} rows overlap (row stride {out.stride(0)} < {ncol}); "
                        "pass a contiguous tensor")
    return out.stride(0) if n > 1 else max(out.shape[1], ncol)


def _eval(name: str, x: torch.Tensor, kmax: int, out, dtype, limit: int):
    _vector(x, dtype, "x")
    if not 0 <= kmax <= limit:
        raise BoysError(f"kmax must be in [0, {limit}]")
    n = x.numel()
    if out is None:
        out = torch.empty((n, kmax + 1), dtype=dtype, device=x.device)
    ld = _rows(out, n, kmax + 1, dtype, x.device, "out")
    with torch.cuda.device(x.device):
        _check(getattr(lib(), name)(_ptr(x), n, kmax, _ptr(out), ld, _stream(x.device)), name)
    return out


def boys_eval_f64(x: torch.Tensor, kmax: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """F_0..F_kmax(x) in FP64 as an (n, kmax+1) tensor (or into ``out``)."""
    return _eval("boys_eval_f64", x, kmax, out, torch.float64, F64_KMAX_EVAL)


def boys_eval_f64_tol(x: torch.Tensor, kmax: int, tol: float,
                      out: torch.Tensor | None = None) -> torch.Tensor:
    """boys_eval_f64 with the cheaper table set whose guarantee is at most tol
    (tol >= 1e-10: the screening set; tol >= 5e-14: the paper's)."""
    _vector(x, torch.float64, "x")
    if not 0 <= kmax <= F64_KMAX_EVAL:
        raise BoysError(f"kmax must be in [0, {F64_KMAX_EVAL}]")
    n = x.numel()
    if out is None:
        out = torch.empty((n, kmax + 1), dtype=torch.float64, device=x.device)
    ld = _rows(out, n, kmax + 1, torch.float64, x.device, "out")
    with torch.cuda.device(x.device):
        _check(lib().boys_eval_f64_tol(_ptr(x), n, kmax, float(tol), _ptr(out), ld,
                                       _stream(x.device)), "boys_eval_f64_tol")
    return out


def boys_eval_f32(x: torch.Tensor, kmax: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """F_0..F_kmax(x) for FP32 x, FP32 results, as an (n, kmax+1) tensor."""
    return _eval("boys_eval_f32", x, kmax, out, torch.float32, F32_KMAX)


def _batch_args(x, batch_off, batch_n, batch_kmax, w, w_off):
    _vector(x, torch.float64, "x")
    _vector(w, torch.float64, "w")
    _vector(batch_off, torch.int64, "batch_off")
    _vector(w_off, torch.int64, "w_off")
    _vector(batch_n, torch.int32, "batch_n")
    _vector(batch_kmax, torch.int32, "batch_kmax")
    nb = batch_off.numel()
    if not (batch_n.numel() == batch_kmax.numel() == w_off.numel() == nb):
        raise BoysError("batch_off, batch_n, batch_kmax and w_off must have the same length")
    for t in (w, batch_off, batch_n, batch_kmax, w_off):
        if t.device != x.device:
            raise BoysError("all tensors must be on one device")
    return nb


def boys_weighted_sum(x, batch_off, batch_n, batch_kmax, w, w_off, out=None,
                      tol=None) -> torch.Tensor:
    """out[i] = sum_l w[w_off[b]+l] F_l(x[i]) for every argument i of batch b.

    tol: None for the 5e-14 tables of the current variant (set_tables), else
    as boys_eval_f64_tol (1e-10 or more takes the screening tables)."""
    nb = _batch_args(x, batch_off, batch_n, batch_kmax, w, w_off)
    if out is None:
        out = torch.zeros_like(x)
    _vector(out, torch.float64, "out")
    args = (_ptr(x), _ptr(batch_off), _ptr(batch_n), _ptr(batch_kmax), _ptr(w), _ptr(w_off), nb)
    with torch.cuda.device(x.device):
        if tol is None:
            _check(lib().boys_weighted_sum(*args, _ptr(out), _stream(x.device)),
                   "boys_weighted_sum")
        else:
            _check(lib().boys_weighted_sum_tol(*args, float(tol), _ptr(out), _stream(x.device)),
                   "boys_weighted_sum_tol")
    return out


def boys_weighted_sum_noalloc(x, batch_off, batch_n, batch_kmax, w, w_off,
                              out: torch.Tensor) -> torch.Tensor:
    """boys_weighted_sum through the entry point that allocates nothing (fixed
    per-device scratch, kernels launched directly; capturable).  ``out`` is
    required, so that this wrapper allocates nothing either."""
    nb = _batch_args(x, batch_off, batch_n, batch_kmax, w, w_off)
    _vector(out, torch.float64, "out")
    with torch.cuda.device(x.device):
        _check(lib().boys_weighted_sum_noalloc(_ptr(x), _ptr(batch_off), _ptr(batch_n),
                                               _ptr(batch_kmax), _ptr(w), _ptr(w_off), nb,
                                               _ptr(out), _stream(x.device)),
               "boys_weighted_sum_noalloc")
    return out


def boys_tune_weighted_sum(x, batch_off, batch_n, batch_kmax, w, w_off, out=None):
    """Autotunes the batched kernel on these arguments; returns (config, ms, name)."""
    nb = _batch_args(x, batch_off, batch_n, batch_kmax, w, w_off)
    if out is None:
        out = torch.zeros_like(x)
    cfg, ms = _INT(-1), ctypes.c_float(0.0)
    with torch.cuda.device(x.device):
        _check(lib().boys_tune_weighted_sum(_ptr(x), _ptr(batch_off), _ptr(batch_n),
                                            _ptr(batch_kmax), _ptr(w), _ptr(w_off), nb, _ptr(out),
                                            _stream(x.device), ctypes.byref(cfg), ctypes.byref(ms)),
               "boys_tune_weighted_sum")
    return cfg.value, ms.value, weighted_sum_config_name(cfg.value)


def weighted_sum_config_name(config: int) -> str:
    return lib().boys_weighted_sum_config_name(config).decode()


def weighted_sum_num_configs() -> int:
    return int(lib().boys_weighted_sum_num_configs())


def weighted_sum_get_config() -> int:
    return int(lib().boys_weighted_sum_get_config())


def weighted_sum_set_config(config: int):
    _check(lib().boys_weighted_sum_set_config(config), "boys_weighted_sum_set_config")


def set_tables(variant: int):
    """Process-wide choice of the 5e-14 tables for orders up to 32:
    TABLES_PAPER, TABLES_PER_KMAX or TABLES_CENTRE (boys_set_tables)."""
    _check(lib().boys_set_tables(int(variant)), "boys_set_tables")


def get_tables() -> int:
    return int(lib().boys_get_tables())


class table_variant:
    """Context manager: calls inside use `variant`; the previous one is
    restored on exit."""

    def __init__(self, variant: int):
        self.variant = int(variant)

    def __enter__(self):
        self.prev = get_tables()
        set_tables(self.variant)
        return self

    def __exit__(self, *exc):
        set_tables(self.prev)
        return False


def boys_backward(x: torch.Tensor, grad_f: torch.Tensor, kmax: int | None = None,
                  out: torch.Tensor | None = None, tol: float | None = None) -> torch.Tensor:
    """grad_x[i] = -sum_k grad_f[i,k] F_{k+1}(x[i]) for k = 0..kmax.

    tol: None for the paper's tables, else as boys_backward_tol."""
    _vector(x, torch.float64, "x")
    n = x.numel()
    if kmax is None:
        kmax = grad_f.shape[1] - 1
    if not 0 <= kmax <= F64_KMAX_BACKWARD:
        raise BoysError(f"kmax must be in [0, {F64_KMAX_BACKWARD}]")
    ld = _rows(grad_f, n, kmax + 1, torch.float64, x.device, "grad_f")
    if out is None:
        out = torch.empty_like(x)
    _vector(out, torch.float64, "grad_x")
    with torch.cuda.device(x.device):
        if tol is None:
            _check(lib().boys_backward(_ptr(x), _ptr(grad_f), n, kmax, ld, _ptr(out),
                                       _stream(x.device)), "boys_backward")
        else:
            _check(lib().boys_backward_tol(_ptr(x), _ptr(grad_f), n, kmax, ld, float(tol),
                                           _ptr(out), _stream(x.device)), "boys_backward_tol")
    return out


def boys_pairsum(x: torch.Tensor, y: torch.Tensor, c, out: torch.Tensor | None = None,
                 tol: float | None = None) -> torch.Tensor:
    """z_i = sum_l c_l sum_j F_l(x_i + x_j) y_j (the paper's benchmark workload).

    x, y: FP64 vectors on the GPU; c: the kmax+1 weights (host sequence).
    tol: None for the paper's tables, else as boys_eval_f64_tol."""
    import numpy as np
    _vector(x, torch.float64, "x")
    _vector(y, torch.float64, "y")
    if y.numel() != x.numel() or y.device != x.device:
        raise BoysError("x and y must have the same length and device")
    ch = np.ascontiguousarray(np.asarray(c.cpu() if isinstance(c, torch.Tensor) else c, dtype=np.float64))
    kmax = ch.size - 1
    if not 0 <= kmax <= F64_KMAX_EVAL:
        raise BoysError(f"c must hold 1..{F64_KMAX_EVAL + 1} weights")
    if out is None:
        out = torch.empty_like(x)
    _vector(out, torch.float64, "out")
    with torch.cuda.device(x.device):
        if tol is None:
            _check(lib().boys_pairsum(_ptr(x), _ptr(y), x.numel(), _P(ch.ctypes.data), kmax,
                                      _ptr(out), _stream(x.device)), "boys_pairsum")
        else:
            _check(lib().boys_pairsum_tol(_ptr(x), _ptr(y), x.numel(), _P(ch.ctypes.data), kmax,
                                          float(tol), _ptr(out), _stream(x.device)),
                   "boys_pairsum_tol")
    return out


class BoysFunction(torch.autograd.Function):
    """F_0..F_kmax(x) with a backward pass through boys_backward.

    ``BoysFunction.apply(x, kmax)`` returns the (n, kmax+1) FP64 tensor of
    boys_eval_f64; its gradient with respect to x uses dF_k/dx = -F_{k+1},
    which the backward kernel recomputes at order kmax+1.
    ``BoysFunction.apply(x, kmax, tol)`` does the same at a chosen accuracy
    (boys_eval_f64_tol forward, boys_backward_tol backward).
    """

    @staticmethod
    def forward(ctx, x, kmax: int, tol: float | None = None):
        if kmax > F64_KMAX_BACKWARD:
            raise BoysError(f"differentiable evaluation needs kmax <= {F64_KMAX_BACKWARD}")
        ctx.save_for_backward(x)
        ctx.kmax = kmax
        ctx.tol = tol
        return boys_eval_f64(x, kmax) if tol is None else boys_eval_f64_tol(x, kmax, tol)

    @staticmethod
    def backward(ctx, grad_f):
        (x,) = ctx.saved_tensors
        grad_x = None
        if ctx.needs_input_grad[0]:
            # An upstream gradient may be a broadcast view (row stride 0, e.g.
            # from F.sum(0) @ v); the kernel needs disjoint rows.
            rows_ok = grad_f.stride(1) == 1 and (grad_f.shape[0] <= 1 or
                                                 grad_f.stride(0) >= grad_f.shape[1])
            g = grad_f if rows_ok else grad_f.contiguous()
            grad_x = boys_backward(x, g, ctx.kmax, tol=ctx.tol)
        return grad_x, None, None


def finalize():
    lib().boys_finalize()
