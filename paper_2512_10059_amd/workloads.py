"""Seeded synthetic inputs for the Boys-function workloads.

This module draws random numbers and nothing else: it holds none of the
method's arithmetic, so the GPU path, the CPU oracle, the tests and the
benchmark can all take their inputs from it.  Every generator uses numpy's
PCG64 ``default_rng(seed)``.

The paper's own benchmark draws arguments uniformly from [0, 30] (Sec. III).
The workloads here follow the shapes in which Boys functions arise in
Gaussian-orbital integrals: for two primitive exponents a, b and a distance R
between centres, the argument is x = a*b/(a+b) * R^2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

N_MIXED = 65536            # plain FP64 correctness workload
N_WRITEOUT = 1 << 26       # write-out workload (FP64 and FP32)
N_BACKWARD = 1 << 24       # differentiation workload
N_BATCHES = 8192           # batched fused workload


def mixed_arguments(n: int = N_MIXED, seed: int = 1) -> np.ndarray:
    """Four equal parts, shuffled: U[0,1]; U[1,30]; log-uniform[30,1e4]; and a
    part that is half exactly 0.0 and half U[0,1e-6] (the tiny-x corner)."""
    rng = np.random.default_rng(seed)
    q = n // 4
    sizes = [q, q, q, n - 3 * q]
    p0 = rng.uniform(0.0, 1.0, sizes[0])
    p1 = rng.uniform(1.0, 30.0, sizes[1])
    p2 = np.exp(rng.uniform(np.log(30.0), np.log(1e4), sizes[2]))
    z = sizes[3] // 2
    p3 = np.concatenate([np.zeros(z), rng.uniform(0.0, 1e-6, sizes[3] - z)])
    x = np.concatenate([p0, p1, p2, p3])
    rng.shuffle(x)
    return x


def gaussian_pair_arguments(n: int = N_WRITEOUT, seed: int = 2) -> np.ndarray:
    """x = a*b/(a+b) * R^2 with a, b log-uniform on [0.05, 1e4] and R uniform
    on [0, 8] bohr.  Range about 1e-12 .. 3e5, median about 18."""
    rng = np.random.default_rng(seed)
    lo, hi = np.log(0.05), np.log(1e4)
    a = np.exp(rng.uniform(lo, hi, n))
    b = np.exp(rng.uniform(lo, hi, n))
    R = rng.uniform(0.0, 8.0, n)
    return (a * b / (a + b)) * (R * R)


@dataclass
class Batches:
    x: np.ndarray            # float64[sum n_b]
    batch_off: np.ndarray    # int64[nbatch]  first argument of batch b
    batch_n: np.ndarray      # int32[nbatch]  number of arguments of batch b
    batch_kmax: np.ndarray   # int32[nbatch]  highest order of batch b
    w: np.ndarray            # float64[sum (kmax_b+1)] weights w_{b,0..kmax_b}
    w_off: np.ndarray        # int64[nbatch]  first weight of batch b

    @property
    def total(self) -> int:
        return int(self.x.size)


def batched_workload(nbatch: int = N_BATCHES, seed: int = 3, mean_size: float = 4096.0,
                     sigma: float = 1.5, max_size: int = 1 << 18, kmax_hi: int = 32) -> Batches:
    """Batch sizes lognormal with mean ``mean_size`` (so mu = ln(mean) - sigma^2/2)
    and shape ``sigma``, rounded and clipped to [1, max_size]; per-batch kmax
    uniform on {0..kmax_hi}; weights N(0,1); arguments as gaussian_pair_arguments."""
    rng = np.random.default_rng(seed)
    mu = np.log(mean_size) - 0.5 * sigma * sigma
    n = np.clip(np.rint(rng.lognormal(mu, sigma, nbatch)), 1, max_size).astype(np.int32)
    kmax = rng.integers(0, kmax_hi + 1, nbatch).astype(np.int32)
    off = np.zeros(nbatch, dtype=np.int64)
    off[1:] = np.cumsum(n.astype(np.int64))[:-1]
    w_off = np.zeros(nbatch, dtype=np.int64)
    w_off[1:] = np.cumsum(kmax.astype(np.int64) + 1)[:-1]
    w = rng.standard_normal(int((kmax.astype(np.int64) + 1).sum()))
    x = gaussian_pair_arguments(int(n.astype(np.int64).sum()), seed=seed + 1000)
    return Batches(x=x, batch_off=off, batch_n=n, batch_kmax=kmax, w=w, w_off=w_off)


def backward_workload(n: int = N_BACKWARD, kmax: int = 16, seed: int = 5):
    """Arguments as gaussian_pair_arguments and upstream gradients G ~ N(0,1)
    of shape (n, kmax+1)."""
    x = gaussian_pair_arguments(n, seed=seed)
    rng = np.random.default_rng(seed + 1000)
    G = rng.standard_normal((n, kmax + 1))
    return x, G


def pair_workload(n: int = 1 << 19, kmax: int = 12, seed: int = 6, x_max: float = 30.0):
    """The paper's benchmark inputs (Sec. III): x uniform on [0, 30], and y and
    the kmax+1 weights c drawn N(0,1) (the paper leaves their distribution
    open).  Its GPU run used n = 2^19 and kmax = 12."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, x_max, n)
    y = rng.standard_normal(n)
    c = rng.standard_normal(kmax + 1)
    return x, y, c
