"""boys_eval_f32 on the GPU against the FP64 oracle evaluated at the FP32
arguments (tolerance 1e-6 absolute), with the maximum error reported per
region A' = [0, x0'), B' = [x0', x1'), C' = [x1', inf)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_10059_amd as boys
from paper_2512_10059_amd import workloads
from tests.test_coeff_tables_f32 import X0F, X1F

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-6
F32 = np.float32


def run(x32: np.ndarray, kmax: int) -> np.ndarray:
    xt = torch.from_numpy(np.ascontiguousarray(x32, dtype=F32)).to(DEV)
    F = boys.boys_eval_f32(xt, kmax)
    torch.cuda.synchronize()
    return F.cpu().numpy().astype(np.float64)


def region_errors(x32, F, ref):
    err = np.abs(F - ref).max(axis=1)
    A = x32 < X0F
    C = x32 >= X1F
    B = ~A & ~C
    return {name: float(err[m].max()) if m.any() else 0.0 for name, m in (("A", A), ("B", B), ("C", C))}


def edge_f32():
    pts = [F32(0), F32(1e-30), F32(1e-6), X0F, X1F]
    out = []
    for p in pts:
        v = p
        for _ in range(3):
            v = np.nextafter(v, F32(-np.inf)) if v > 0 else v
        for _ in range(7):
            out.append(v)
            v = np.nextafter(v, F32(np.inf))
    out += [F32(30.0), F32(1e4), F32(3e38)]
    return np.array([v for v in out if v >= 0], F32)


@pytest.mark.parametrize("kmax", range(17))
def test_every_order_per_region(kmax):
    rng = np.random.default_rng(300 + kmax)
    x = np.concatenate([edge_f32(), rng.uniform(0, float(X0F), 2000).astype(F32),
                        rng.uniform(float(X0F), float(X1F), 2000).astype(F32),
                        np.exp(rng.uniform(np.log(float(X1F)), np.log(1e5), 1000)).astype(F32),
                        workloads.gaussian_pair_arguments(3000, seed=400 + kmax).astype(F32)])
    F = run(x, kmax)
    ref = oracle.boys(x.astype(np.float64), kmax)
    errs = region_errors(x, F, ref)
    print(f"kmax={kmax} max abs err per region: {errs}")
    assert max(errs.values()) <= TOL, errs


@pytest.mark.parametrize("n", [1, 63, 65, 257, 4099])
def test_ragged_sizes(n):
    x = workloads.gaussian_pair_arguments(n, seed=n).astype(F32)
    assert np.abs(run(x, 16) - oracle.boys(x.astype(np.float64), 16)).max() <= TOL


def test_padded_and_unaligned_output():
    x = workloads.gaussian_pair_arguments(777, seed=3).astype(F32)
    ref = oracle.boys(x.astype(np.float64), 9)
    xt = torch.from_numpy(x).to(DEV)
    big = torch.full((777, 12), -3.0, dtype=torch.float32, device=DEV)
    boys.boys_eval_f32(xt, 9, out=big[:, :10])
    buf = torch.full((777 * 10 + 1,), -3.0, dtype=torch.float32, device=DEV)
    odd = buf[1:].view(777, 10)
    boys.boys_eval_f32(xt, 9, out=odd)
    torch.cuda.synchronize()
    b = big.cpu().numpy().astype(np.float64)
    assert np.abs(b[:, :10] - ref).max() <= TOL and np.all(b[:, 10:] == -3.0)
    assert np.abs(odd.cpu().numpy().astype(np.float64) - ref).max() <= TOL
    assert buf[0].item() == -3.0


def test_domain_values():
    x = np.array([-1.0, np.nan, np.inf, 0.0], F32)
    F = run(x, 16)
    assert np.all(np.isnan(F[:2])) and np.all(F[2] == 0.0)
    assert np.abs(F[3] - 1.0 / (2 * np.arange(17) + 1)).max() <= TOL


def test_invalid_arguments_raise():
    x = torch.ones(4, dtype=torch.float32, device=DEV)
    with pytest.raises(boys.BoysError):
        boys.boys_eval_f32(x, 17)
    with pytest.raises(boys.BoysError):
        boys.boys_eval_f32(x.double(), 3)


def test_full_precision_workload_sampled():
    """The 2^26 write-out arguments rounded to FP32, kmax=16 (the launch the
    benchmark times): 2^17 sampled rows plus the first and last 4096 against
    the oracle, per region; and FP64 agreement within 1e-6 on the sample."""
    x = workloads.gaussian_pair_arguments().astype(F32)
    xt = torch.from_numpy(x).to(DEV)
    F = boys.boys_eval_f32(xt, 16)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    n = x.size
    idx = np.unique(np.concatenate([rng.integers(0, n, 1 << 17), np.arange(4096), np.arange(n - 4096, n)]))
    Fs = F[torch.from_numpy(idx).to(DEV)].cpu().numpy().astype(np.float64)
    ref = oracle.boys(x[idx].astype(np.float64), 16)
    errs = region_errors(x[idx], Fs, ref)
    print(f"full workload sample, max abs err per region: {errs}")
    assert max(errs.values()) <= TOL, errs
    assert bool(torch.isfinite(F).all())
