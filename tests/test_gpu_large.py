"""More than 2^31 arguments in one call: the 64-bit index paths of the
write-out (FP64 and FP32), backward and batched kernels.  Arguments are drawn
on the device (uniform on [0, 40), which covers all three regions); rows near
the start, around index 2^31, at the end and at random are compared with the
oracle.  Each test frees its buffers (about 50 GB at most) before the next."""
import gc

import numpy as np
import pytest
import torch

import oracle
import paper_2512_10059_amd as boys

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N = (1 << 31) + 77
EPS_TOL = 5e-14


def sample_rows(n, seed):
    rng = np.random.default_rng(seed)
    edge = (1 << 31)
    idx = np.concatenate([np.arange(64), np.arange(edge - 64, edge + 64), np.arange(n - 64, n),
                          rng.integers(0, n, 4096)])
    return np.unique(idx)


def device_arguments(n, seed, dtype=torch.float64):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    return torch.rand(n, dtype=dtype, device=DEV, generator=g) * 40.0


def release():
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_eval_f64_beyond_2_31():
    x = device_arguments(N, 1)
    F = boys.boys_eval_f64(x, 1)
    torch.cuda.synchronize()
    idx = sample_rows(N, 2)
    it = torch.from_numpy(idx).to(DEV)
    xs, Fs = x[it].cpu().numpy(), F[it].cpu().numpy()
    del x, F
    release()
    assert np.abs(Fs - oracle.boys(xs, 1)).max() <= EPS_TOL


def test_eval_f32_beyond_2_31():
    x = device_arguments(N, 3, torch.float32)
    F = boys.boys_eval_f32(x, 0)
    torch.cuda.synchronize()
    idx = sample_rows(N, 4)
    it = torch.from_numpy(idx).to(DEV)
    xs, Fs = x[it].double().cpu().numpy(), F[it].double().cpu().numpy()
    del x, F
    release()
    assert np.abs(Fs - oracle.boys(xs, 0)).max() <= 1e-6


def test_backward_beyond_2_31():
    x = device_arguments(N, 5)
    g = torch.Generator(device=DEV)
    g.manual_seed(6)
    G = torch.randn((N, 1), dtype=torch.float64, device=DEV, generator=g)
    grad = boys.boys_backward(x, G, 0)
    torch.cuda.synchronize()
    idx = sample_rows(N, 7)
    it = torch.from_numpy(idx).to(DEV)
    xs, Gs, gs = x[it].cpu().numpy(), G[it].cpu().numpy(), grad[it].cpu().numpy()
    del x, G, grad
    release()
    ref = -Gs[:, 0] * oracle.boys(xs, 1)[:, 1]
    assert np.all(np.abs(gs - ref) <= EPS_TOL * np.abs(Gs[:, 0]) + 1e-15 * np.abs(ref))


def test_weighted_sum_beyond_2_31():
    """Three batches of 2^30, 2^30 and 4173 arguments (orders 3, 9 and 32):
    offsets past 2^31 in the batch table and in the kernel's addressing."""
    sizes = np.array([1 << 30, 1 << 30, 4173], dtype=np.int32)
    kmax = np.array([3, 9, 32], dtype=np.int32)
    off = np.array([0, 1 << 30, 1 << 31], dtype=np.int64)
    w_off = np.array([0, 4, 14], dtype=np.int64)
    w = np.random.default_rng(8).standard_normal(int((kmax + 1).sum()))
    n = int(sizes.astype(np.int64).sum())
    x = device_arguments(n, 9)
    t = lambda a: torch.from_numpy(a).to(DEV)
    out = boys.boys_weighted_sum(x, t(off), t(sizes), t(kmax), t(w), t(w_off))
    torch.cuda.synchronize()
    idx = sample_rows(n, 10)
    it = torch.from_numpy(idx).to(DEV)
    xs, got = x[it].cpu().numpy(), out[it].cpu().numpy()
    del x, out
    release()
    b = np.searchsorted(off, idx, side="right") - 1
    for bb in range(3):
        m = b == bb
        k = int(kmax[bb])
        wl = w[w_off[bb]:w_off[bb] + k + 1]
        ref = oracle.boys(xs[m], k) @ wl
        tol = EPS_TOL * np.abs(wl).sum() + 4 * (k + 1) * 2.0**-53 * (oracle.boys(xs[m], k) @ np.abs(wl))
        assert np.all(np.abs(got[m] - ref) <= tol), bb
