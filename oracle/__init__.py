"""CPU oracle for the Boys functions -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never uses it and it
uses nothing of the GPU library: the arithmetic lives in ``boys_oracle.c``
(long double, see its header for the method and its citations), and this
module only marshals arrays and composes the exact functions into the
quantities the hot path produces:

* :func:`boys`            F_0..F_kmax(x), definition Sec. I eq. 3.
* :func:`weighted_sum`    sum_l w_l F_l(x) per argument, the consumer of the
                          paper's benchmark (Sec. III, Algorithm 2), with one
                          (kmax, w) per batch of arguments.
* :func:`backward`        dL/dx = -sum_k G_k F_{k+1}(x) for L = sum_k G_k F_k(x),
                          from dF_k/dx = -F_{k+1} (differentiate eq. 3 under
                          the integral sign).
* :func:`central_difference`  the same gradient by a long-double central
                          difference of L, independent of the derivative rule.
* :func:`pairsum`         z_i = sum_l c_l sum_j F_l(x_i + x_j) y_j, the paper's
                          benchmark quantity (Sec. III, Algorithm 2), for
                          selected rows i.

Pins: ``tests/oracle_pins.py`` ties the long-double F_k to mpmath, quadrature
and the closed forms; ``tests/oracle_composition_pins.py`` ties each composed
quantity above to values built from mpmath's incomplete gamma function (not
from this module's F), with planted mistakes in this file that must be caught.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

KMAX_LIMIT = 40


class OracleLib:
    """ctypes view of one build of ``boys_oracle.c`` (the default build lives
    next to this file; tests also load deliberately broken builds)."""

    def __init__(self, path: str):
        if not os.path.exists(path):
            raise RuntimeError(f"oracle library {path} is not built; run __graft_entry__.build()")
        assert np.finfo(np.longdouble).nmant >= 63, "the oracle needs x87 long double"
        lib = ctypes.CDLL(path)
        for name in ("oracle_boys_ld", "oracle_boys_f64"):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
            fn.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        self._lib = lib
        self.path = path

    def max_threads(self) -> int:
        return int(self._lib.oracle_max_threads())

    def boys_ld(self, x, kmax: int, threads: int = 0) -> np.ndarray:
        """F_0..F_kmax at every x, as an (n, kmax+1) long-double array."""
        xa = np.ascontiguousarray(np.asarray(x, dtype=np.longdouble).reshape(-1))
        out = np.empty((xa.size, kmax + 1), dtype=np.longdouble)
        rc = self._lib.oracle_boys_ld(xa.ctypes.data, xa.size, int(kmax), out.ctypes.data, int(threads))
        if rc != 0:
            raise ValueError(f"oracle_boys_ld rejected n={xa.size} kmax={kmax}")
        return out

    def boys(self, x, kmax: int, threads: int = 0) -> np.ndarray:
        """F_0..F_kmax at every x (taken as float64), rounded to float64, shape (n, kmax+1)."""
        xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
        out = np.empty((xa.size, kmax + 1), dtype=np.float64)
        rc = self._lib.oracle_boys_f64(xa.ctypes.data, xa.size, int(kmax), out.ctypes.data, int(threads))
        if rc != 0:
            raise ValueError(f"oracle_boys_f64 rejected n={xa.size} kmax={kmax}")
        return out


_default = None


def lib() -> OracleLib:
    global _default
    if _default is None:
        _default = OracleLib(_LIB_PATH)
    return _default


def max_threads() -> int:
    return lib().max_threads()


def boys_ld(x, kmax: int, threads: int = 0) -> np.ndarray:
    return lib().boys_ld(x, kmax, threads)


def boys(x, kmax: int, threads: int = 0) -> np.ndarray:
    return lib().boys(x, kmax, threads)


def weighted_sum(x, batch_off, batch_n, batch_kmax, w, w_off, threads: int = 0) -> np.ndarray:
    """out[i] = sum_{l=0..kmax_b} w[w_off_b + l] F_l(x[i]) for every i in batch b.

    Batch b covers x[batch_off_b : batch_off_b + batch_n_b]; arguments outside
    every batch get 0.  Evaluated in long double, returned as float64.
    """
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    out = np.zeros(x.size, dtype=np.float64)
    for off, n, k, wo in zip(batch_off, batch_n, batch_kmax, w_off):
        off, n, k, wo = int(off), int(n), int(k), int(wo)
        if n == 0:
            continue
        F = boys_ld(x[off:off + n], k, threads)
        wl = w[wo:wo + k + 1].astype(np.longdouble)
        out[off:off + n] = (F * wl[None, :]).sum(axis=1).astype(np.float64)
    return out


def backward_ld(x, G, threads: int = 0) -> np.ndarray:
    """-sum_{k=0..K} G[i,k] F_{k+1}(x[i]) in long double; G has shape (n, K+1)."""
    G = np.asarray(G)
    K = G.shape[1] - 1
    F = boys_ld(x, K + 1, threads)
    return -(G.astype(np.longdouble) * F[:, 1:]).sum(axis=1)


def backward(x, G, threads: int = 0) -> np.ndarray:
    return backward_ld(x, G, threads).astype(np.float64)


def central_difference(x, G, rel_step: float = 1e-6, threads: int = 0) -> np.ndarray:
    """(L(x+h) - L(x-h)) / 2h with L = sum_k G[i,k] F_k(x) and h = rel_step*max(1,x).

    Everything in long double, so the difference itself loses only about
    1e-19/h of relative accuracy; the O(h^2) truncation is about 1e-13 of F.
    """
    G = np.asarray(G).astype(np.longdouble)
    K = G.shape[1] - 1
    xl = np.asarray(x, dtype=np.float64).astype(np.longdouble)
    h = np.longdouble(rel_step) * np.maximum(np.longdouble(1), xl)
    Fp = boys_ld(xl + h, K, threads)
    Fm = boys_ld(xl - h, K, threads)
    Lp = (G * Fp).sum(axis=1)
    Lm = (G * Fm).sum(axis=1)
    return ((Lp - Lm) / (2 * h)).astype(np.float64)


def pairsum(x, y, c, rows=None, threads: int = 0):
    """z_i = sum_l c_l sum_j F_l(x_i + x_j) y_j for i in ``rows`` (default all).

    The argument x_i + x_j is formed in float64 (as the GPU forms it), then
    everything else is long double.  Returns (z, scale) as float64 arrays
    where scale_i = sum_j |y_j| sum_l |c_l F_l(x_i + x_j)| bounds the
    magnitude of the summands (for rounding bounds)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64).astype(np.longdouble)
    c = np.asarray(c, dtype=np.float64).astype(np.longdouble)
    k = c.size - 1
    rows = range(x.size) if rows is None else rows
    z, scale = [], []
    for i in rows:
        F = boys_ld(x[int(i)] + x, k, threads)
        w = (F * c[None, :]).sum(axis=1)
        z.append((y * w).sum())
        scale.append((np.abs(y) * (np.abs(F * c[None, :])).sum(axis=1)).sum())
    return np.array(z, dtype=np.float64), np.array(scale, dtype=np.float64)
