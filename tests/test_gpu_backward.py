"""boys_backward and the autograd function on the GPU.

The gradient of L = sum_k G_k F_k(x) is checked against the oracle's
-sum_k G_k F_{k+1}(x) and against a long-double central difference of L with
h = 1e-6 max(1, x), to 1e-10 relative.  "Relative" is taken against the
scale S = sum_k |G_k| F_{k+1}(x) of the sum (the sum itself can cancel to
zero).  Where the method's absolute guarantee, 5e-14 per F_{k+1}, exceeds
1e-10 S (orders whose F_{k+1} is below about 5e-4 of the others), the bound
is that guarantee: tol = max(1e-10 S, 5e-14 sum_k |G_k|)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_10059_amd as boys
from paper_2512_10059_amd import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
REL = 1e-10
EPS_TOL = 5e-14


def gpu_backward(x, G, kmax=None):
    xt = torch.from_numpy(x).to(DEV)
    Gt = torch.from_numpy(np.ascontiguousarray(G)).to(DEV)
    return boys.boys_backward(xt, Gt, kmax).cpu().numpy()


def bounds(x, G):
    K = G.shape[1] - 1
    F = oracle.boys(x, K + 1)
    S = (np.abs(G) * F[:, 1:]).sum(1)
    return S, np.maximum(REL * S, EPS_TOL * np.abs(G).sum(1))


def test_gradient_vs_oracle_and_central_difference():
    x, G = workloads.backward_workload(n=20000, kmax=16, seed=21)
    x[:5] = [0.0, 1e-9, 11.899848152108484, 28.98933773882074, 1e4]
    g = gpu_backward(x, G)
    S, tol = bounds(x, G)
    ref = oracle.backward(x, G)
    fd = oracle.central_difference(x, G)
    e_ref = np.abs(g - ref)
    e_fd = np.abs(g - fd)
    assert np.all(e_ref <= tol), f"vs oracle: worst {np.max(e_ref / tol):.3f} of bound"
    assert np.all(e_fd <= tol + 1e-12 * S), f"vs central difference: worst {np.max(e_fd / tol):.3f}"
    # Report how much of the sample meets the strict 1e-10 * S bound.
    strict = np.mean(e_ref <= REL * S)
    assert strict > 0.99, f"only {strict:.4f} within 1e-10 S"


@pytest.mark.parametrize("kmax", [0, 1, 5, 8, 15, 16, 24, 31, 32, 33, 36, 38, 39])
def test_every_order(kmax):
    """Orders up to 31 recompute F_{kmax+1} with the paper's tables, 32..39
    with the high-order set; even and odd row lengths, full and partial
    waves."""
    x, G = workloads.backward_workload(n=3000, kmax=kmax, seed=40 + kmax)
    g = gpu_backward(x, G)
    S, tol = bounds(x, G)
    assert np.all(np.abs(g - oracle.backward(x, G)) <= tol)


@pytest.mark.parametrize("kmax", [16, 24])
def test_padded_gradient_rows_and_ragged_sizes(kmax):
    """Row stride kmax+5 and sizes with partial waves; kmax 24 is an order
    whose packed rows would go to LDS by DMA, so this covers its fallback."""
    for n in (1, 63, 65, 257, 1000):
        x, Gfull = workloads.backward_workload(n=n, kmax=kmax + 4, seed=n)
        G = Gfull[:, :kmax + 1]
        xt = torch.from_numpy(x).to(DEV)
        Gt = torch.from_numpy(Gfull).to(DEV)[:, :kmax + 1]  # row stride kmax+5
        g = boys.boys_backward(xt, Gt, kmax).cpu().numpy()
        S, tol = bounds(x, G)
        assert np.all(np.abs(g - oracle.backward(x, G)) <= tol), n


@pytest.mark.parametrize("kmax", [15, 16, 18, 24, 30])
def test_packed_rows_aligned_and_unaligned(kmax):
    """Packed rows (ld = kmax+1) take 16-byte loads (kmax <= 16, or an even
    row length) or LDS-DMA loads (odd row lengths from 19) when G is 16-byte
    aligned, and 8-byte loads when it is not; all give the same gradient bit
    for bit.  Even and odd row lengths (a 16-byte unit straddles two rows
    when odd)."""
    n = 64 * 37 + 29
    x, G = workloads.backward_workload(n=n, kmax=kmax, seed=70 + kmax)
    xt = torch.from_numpy(x).to(DEV)
    buf = torch.zeros(n * (kmax + 1) + 1, dtype=torch.float64, device=DEV)
    Ga = buf[:-1].view(n, kmax + 1)
    Ga.copy_(torch.from_numpy(G))
    Gu = buf[1:].view(n, kmax + 1)  # 8 bytes off 16-byte alignment
    ga = boys.boys_backward(xt, Ga, kmax).cpu().numpy()
    Gu.copy_(torch.from_numpy(G))
    gu = boys.boys_backward(xt, Gu, kmax).cpu().numpy()
    assert np.array_equal(ga, gu)
    S, tol = bounds(x, G)
    assert np.all(np.abs(ga - oracle.backward(x, G)) <= tol)


def test_autograd_at_high_orders():
    """BoysFunction at kmax 36 and 39 (forward and backward through the
    high-order tables) against the oracle."""
    for kmax in (36, 39):
        x, G = workloads.backward_workload(n=3000, kmax=kmax, seed=80 + kmax)
        xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
        F = boys.BoysFunction.apply(xt, kmax)
        F.backward(torch.from_numpy(G).to(DEV))
        S, tol = bounds(x, G)
        assert np.all(np.abs(xt.grad.cpu().numpy() - oracle.backward(x, G)) <= tol), kmax
        assert np.abs(F.detach().cpu().numpy() - oracle.boys(x, kmax)).max() <= EPS_TOL


def test_autograd_matches_kernel_and_oracle():
    x, G = workloads.backward_workload(n=5000, kmax=16, seed=3)
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    Gt = torch.from_numpy(G).to(DEV)
    F = boys.BoysFunction.apply(xt, 16)
    loss = (F * Gt).sum()
    loss.backward()
    g = xt.grad.cpu().numpy()
    direct = boys.boys_backward(xt.detach(), Gt, 16).cpu().numpy()
    assert np.array_equal(g, direct)
    S, tol = bounds(x, G)
    assert np.all(np.abs(g - oracle.backward(x, G)) <= tol)
    Fo = oracle.boys(x, 16)
    assert np.abs(F.detach().cpu().numpy() - Fo).max() <= EPS_TOL


def test_autograd_broadcast_upstream_gradient():
    """A loss (F.sum(0) @ v) whose upstream gradient reaches BoysFunction as a
    broadcast view (row stride 0): the gradient is -sum_k v_k F_{k+1}(x) per
    argument, as the oracle gives for G = v in every row."""
    x, _ = workloads.backward_workload(n=4000, kmax=16, seed=31)
    v = np.random.default_rng(32).standard_normal(17)
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    F = boys.BoysFunction.apply(xt, 16)
    (F.sum(0) @ torch.from_numpy(v).to(DEV)).backward()
    G = np.broadcast_to(v, (x.size, 17))
    S, tol = bounds(x, G)
    assert np.all(np.abs(xt.grad.cpu().numpy() - oracle.backward(x, np.ascontiguousarray(G))) <= tol)
    # The direct entry point refuses overlapping rows instead of misreading them.
    with pytest.raises(boys.BoysError):
        boys.boys_backward(xt.detach(), torch.from_numpy(v).to(DEV).expand(x.size, 17), 16)


def test_empty_and_invalid():
    x = torch.empty(0, dtype=torch.float64, device=DEV)
    G = torch.empty((0, 17), dtype=torch.float64, device=DEV)
    assert boys.boys_backward(x, G, 16).numel() == 0
    x = torch.ones(4, dtype=torch.float64, device=DEV)
    with pytest.raises(boys.BoysError):
        boys.boys_backward(x, torch.ones((4, 41), dtype=torch.float64, device=DEV), 40)
    with pytest.raises(boys.BoysError):
        boys.boys_backward(x, torch.ones((4, 3), dtype=torch.float64, device=DEV), 5)


def test_full_differentiation_workload_sampled():
    """2^24 arguments, kmax=16: forward plus backward at full size, 2^15
    sampled gradients against the oracle and the central difference."""
    x, G = workloads.backward_workload()
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    Gt = torch.from_numpy(G).to(DEV)
    F = boys.BoysFunction.apply(xt, 16)
    F.backward(Gt)
    g = xt.grad
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    idx = np.unique(rng.integers(0, x.size, 1 << 15))
    gs = g[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    S, tol = bounds(x[idx], G[idx])
    assert np.all(np.abs(gs - oracle.backward(x[idx], G[idx])) <= tol)
    assert np.all(np.abs(gs - oracle.central_difference(x[idx], G[idx])) <= tol + 1e-12 * S)
    Fs = F.detach()[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    assert np.abs(Fs - oracle.boys(x[idx], 16)).max() <= EPS_TOL


def _around(points, steps=2):
    out = []
    for p in points:
        v = p
        for _ in range(steps):
            v = np.nextafter(v, -np.inf) if v > 0 else v
        for _ in range(2 * steps + 1):
            out.append(v)
            v = np.nextafter(v, np.inf)
    return np.array(out)


@pytest.mark.parametrize("kmax", [16, 36])
def test_domain_values_and_region_boundaries(kmax):
    """Outside the domain the gradient is NaN (x < 0, NaN) or zero (x = +inf,
    where every F_{k+1} is 0).  At the region boundaries of both table sets
    (the paper's x0, x1 for orders up to 32; the high-order set's for 33..40,
    which kmax 36 recomputes at order 37), +-2 ulps, the gradient matches
    the oracle within the bound of the other tests."""
    rng = np.random.default_rng(77 + kmax)
    pts = _around([0.0, 5e-324, 11.899848152108484, 28.98933773882074,
                   14.842842360917231, 30.455574446774907, 1e300])
    x = np.concatenate([pts, [-1.0, -1e-300, np.nan, np.inf]])
    G = rng.standard_normal((x.size, kmax + 1))
    g = gpu_backward(x, G)
    m = pts.size
    assert np.all(np.isnan(g[m:m + 3])), g[m:m + 3]
    assert g[m + 3] == 0.0
    S, tol = bounds(pts, G[:m])
    assert np.all(np.abs(g[:m] - oracle.backward(pts, G[:m])) <= tol)
