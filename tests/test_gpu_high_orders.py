"""Orders 33..40 through boys_eval_f64 (the high-order table set: the
method's construction at eps_tol = 5e-14 for kmax = 40) on the GPU against
the long-double oracle.  Bar: 5e-14 absolute, as for the paper's tables."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_10059_amd as boys
from paper_2512_10059_amd import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
EPS_TOL = 5e-14
X0H, X1H = 14.842842360917231, 30.455574446774907   # the high-order set's x0, x1
X0, X1 = 11.899848152108484, 28.98933773882074       # the paper's


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def edge_arguments():
    pts = [0.0, 5e-324, 1e-300, 1e-9, 0.5, 1.0, 40.0, 1e3, 1e6, 1e300]
    for b in (X0, X1, X0H, X1H):
        v = b
        for _ in range(3):
            v = np.nextafter(v, -np.inf)
        for _ in range(7):
            pts.append(v)
            v = np.nextafter(v, np.inf)
    return np.array(pts)


@pytest.mark.parametrize("kmax", range(33, 41))
def test_every_high_order(kmax):
    rng = np.random.default_rng(500 + kmax)
    x = np.concatenate([edge_arguments(), rng.uniform(0, X0H, 900), rng.uniform(X0H, X1H, 600),
                        rng.uniform(X1H, 60, 300), workloads.gaussian_pair_arguments(700, seed=600 + kmax)])
    F = boys.boys_eval_f64(dev(x), kmax).cpu().numpy()
    err = np.abs(F - oracle.boys(x, kmax))
    i = np.unravel_index(err.argmax(), err.shape)
    assert err.max() <= EPS_TOL, f"kmax={kmax}: {err.max():.3e} at x={x[i[0]]!r}, k={i[1]}"


def test_padded_and_unaligned_output_at_order_40():
    x = workloads.gaussian_pair_arguments(1000, seed=61)
    ref = oracle.boys(x, 40)
    big = torch.full((1000, 48), -7.0, dtype=torch.float64, device=DEV)
    boys.boys_eval_f64(dev(x), 40, out=big[:, :41])
    buf = torch.full((1000 * 41 + 1,), -7.0, dtype=torch.float64, device=DEV)
    odd = buf[1:].view(1000, 41)
    boys.boys_eval_f64(dev(x), 40, out=odd)
    b = big.cpu().numpy()
    assert np.abs(b[:, :41] - ref).max() <= EPS_TOL
    assert np.all(b[:, 41:] == -7.0)
    assert np.abs(odd.cpu().numpy() - ref).max() <= EPS_TOL
    assert buf[0].item() == -7.0


@pytest.mark.parametrize("tol", [5e-14, 1e-10, 1.0])
def test_high_orders_take_the_high_set_for_any_valid_tolerance(tol):
    x = dev(workloads.gaussian_pair_arguments(5000, seed=62))
    a = boys.boys_eval_f64(x, 36).cpu().numpy()
    b = boys.boys_eval_f64_tol(x, 36, tol).cpu().numpy()
    assert np.array_equal(a, b)


def test_order_41_is_rejected():
    with pytest.raises(boys.BoysError):
        boys.boys_eval_f64(dev(np.ones(4)), 41)


def test_order_40_sampled_at_2_24():
    """2^24 Gaussian-pair arguments at kmax = 40 (a 5.5 GB output): 2^15
    sampled rows and the first and last 1024 against the oracle."""
    x = workloads.gaussian_pair_arguments(1 << 24, seed=63)
    F = boys.boys_eval_f64(dev(x), 40)
    torch.cuda.synchronize()
    n = x.size
    rng = np.random.default_rng(64)
    idx = np.unique(np.concatenate([rng.integers(0, n, 1 << 15), np.arange(1024), np.arange(n - 1024, n)]))
    Fs = F[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    assert np.abs(Fs - oracle.boys(x[idx], 40)).max() <= EPS_TOL
    assert bool(torch.isfinite(F).all())
    del F
    torch.cuda.empty_cache()
