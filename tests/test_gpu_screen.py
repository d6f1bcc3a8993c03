"""The screening table set (eps_tol = 1e-10) through boys_eval_f64_tol,
boys_pairsum_tol and boys_weighted_sum_tol on the GPU, against the
long-double oracle.

Bar: 1e-10 absolute per F_k (the set's guarantee; the FP64 rounding of the
evaluation adds ~1e-16), and for the pair sums 1e-10 sum_l |c_l| sum_j |y_j|
plus the rounding allowance of the paper-set pair test.  Tolerances the
paper's set meets (5e-14 <= tol < 1e-10) must give exactly boys_eval_f64."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_10059_amd as boys
from paper_2512_10059_amd import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
EPS = 1e-10
TOL = EPS * (1 + 1e-4)
X0 = 11.899848152108484
X1S = 23.149988540679747   # screening x1
X1 = 28.98933773882074     # the paper's x1
U = 2.0 ** -53


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def edge_arguments():
    pts = [0.0, 5e-324, 1e-300, 1e-9, 0.5, 1.0, 30.0, 1e3, 1e6, 1e300]
    for b in (X0, X1S, X1):
        v = b
        for _ in range(3):
            v = np.nextafter(v, -np.inf)
        for _ in range(7):
            pts.append(v)
            v = np.nextafter(v, np.inf)
    return np.array(pts)


@pytest.mark.parametrize("kmax", range(33))
def test_every_order_within_1e10(kmax):
    rng = np.random.default_rng(300 + kmax)
    x = np.concatenate([edge_arguments(), rng.uniform(0, X0, 700), rng.uniform(X0, X1S, 500),
                        rng.uniform(X1S, 40, 300), workloads.gaussian_pair_arguments(800, seed=400 + kmax)])
    F = boys.boys_eval_f64_tol(dev(x), kmax, 1e-10).cpu().numpy()
    err = np.abs(F - oracle.boys(x, kmax))
    assert err.max() <= TOL, f"kmax={kmax}: {err.max():.3e} at x={x[np.unravel_index(err.argmax(), err.shape)[0]]!r}"


@pytest.mark.parametrize("tol", [5e-14, 1e-12, 9.99e-11])
def test_tolerances_the_paper_set_meets_give_boys_eval_f64(tol):
    x = dev(workloads.gaussian_pair_arguments(20000, seed=31))
    a = boys.boys_eval_f64(x, 20).cpu().numpy()
    b = boys.boys_eval_f64_tol(x, 20, tol).cpu().numpy()
    assert np.array_equal(a, b)


def test_looser_tolerances_use_the_screening_set():
    x = dev(workloads.gaussian_pair_arguments(20000, seed=32))
    a = boys.boys_eval_f64_tol(x, 16, 1e-10).cpu().numpy()
    b = boys.boys_eval_f64_tol(x, 16, 1e-6).cpu().numpy()
    c = boys.boys_eval_f64(x, 16).cpu().numpy()
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)   # a different table set


def test_invalid_tolerance_raises():
    x = dev(np.ones(8))
    for tol in (1e-14, 0.0, float("nan")):
        with pytest.raises(boys.BoysError):
            boys.boys_eval_f64_tol(x, 4, tol)


def test_full_writeout_workload_sampled():
    """2^26 arguments, kmax = 32, the launch the benchmark times: 2^16 sampled
    rows and the first and last 2048 against the oracle."""
    x = workloads.gaussian_pair_arguments()
    xt = dev(x)
    F = boys.boys_eval_f64_tol(xt, 32, 1e-10)
    torch.cuda.synchronize()
    n = x.size
    rng = np.random.default_rng(78)
    idx = np.unique(np.concatenate([rng.integers(0, n, 1 << 16), np.arange(2048), np.arange(n - 2048, n)]))
    Fs = F[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    err = np.abs(Fs - oracle.boys(x[idx], 32))
    assert err.max() <= TOL
    assert bool(torch.isfinite(F).all())
    del F
    torch.cuda.empty_cache()


def pair_check(x, y, c, z, rows, eps):
    ref, scale = oracle.pairsum(x, y, c, rows)
    k = len(c) - 1
    tol = eps * (1 + 1e-4) * np.abs(c).sum() * np.abs(y).sum() + ((k + 2) + 512 + x.size / 512 + 2) * U * scale
    err = np.abs(z[rows] - ref)
    assert np.all(err <= tol), f"worst {np.max(err / tol):.3f} of the bound"


@pytest.mark.parametrize("kmax", [0, 7, 12, 32])
def test_pairsum_screening_set(kmax):
    x, y, c = workloads.pair_workload(n=700, kmax=kmax, seed=50 + kmax)
    z = boys.boys_pairsum(dev(x), dev(y), c, tol=1e-10).cpu().numpy()
    pair_check(x, y, c, z, np.arange(x.size), EPS)


def test_pairsum_paper_tolerance_is_boys_pairsum():
    x, y, c = workloads.pair_workload(n=900, kmax=12, seed=60)
    a = boys.boys_pairsum(dev(x), dev(y), c).cpu().numpy()
    b = boys.boys_pairsum(dev(x), dev(y), c, tol=5e-14).cpu().numpy()
    assert np.array_equal(a, b)


# --- the batched consumer (boys_weighted_sum_tol) -----------------------------

def _batches(seed, nbatch=240):
    """Small batches of every order 0..32 over the write-out distribution,
    with empty batches and the region boundaries of both sets planted."""
    bt = workloads.batched_workload(nbatch=nbatch, seed=seed, mean_size=300.0, sigma=1.2,
                                    max_size=4000)
    bt.batch_n[5::41] = 0
    edges = edge_arguments()
    b = int(np.argmax(bt.batch_n))
    assert bt.batch_n[b] >= edges.size
    bt.x[int(bt.batch_off[b]):int(bt.batch_off[b]) + edges.size] = edges
    return bt


def _ws(bt, tol=None, out=None):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return boys.boys_weighted_sum(t(bt.x), t(bt.batch_off), t(bt.batch_n), t(bt.batch_kmax),
                                  t(bt.w), t(bt.w_off), out=out, tol=tol).cpu().numpy()


def _ws_bound(bt, eps):
    tol = np.zeros(bt.x.size)
    mask = np.zeros(bt.x.size, bool)
    for b in range(bt.batch_off.size):
        off, n, k, wo = (int(bt.batch_off[b]), int(bt.batch_n[b]), int(bt.batch_kmax[b]),
                         int(bt.w_off[b]))
        if n <= 0:
            continue
        wl = bt.w[wo:wo + k + 1]
        F = oracle.boys(bt.x[off:off + n], k)
        tol[off:off + n] = eps * np.abs(wl).sum() + 4 * (k + 1) * U * (np.abs(wl) * F).sum(1)
        mask[off:off + n] = True
    return tol, mask


def test_weighted_sum_screening_set_every_config():
    """tol = 1e-10: every argument within 1e-10 sum_l |w_l| plus the
    accumulation's rounding, and every configuration bitwise equal."""
    bt = _batches(seed=90)
    ref = oracle.weighted_sum(bt.x, bt.batch_off, bt.batch_n, bt.batch_kmax, bt.w, bt.w_off)
    tol, mask = _ws_bound(bt, TOL)
    saved = boys.weighted_sum_get_config()
    try:
        first = None
        for cfg in range(boys.weighted_sum_num_configs()):
            boys.weighted_sum_set_config(cfg)
            got = _ws(bt, tol=1e-10)
            err = np.abs(got - ref)
            assert np.all(err[mask] <= tol[mask]), (cfg, float(np.max(err[mask] - tol[mask])))
            if first is None:
                first = got
            else:
                assert np.array_equal(got[mask], first[mask]), cfg
    finally:
        boys.weighted_sum_set_config(saved)
    paper = _ws(bt)
    assert not np.array_equal(paper[mask], first[mask])  # a different table set ran


@pytest.mark.parametrize("tol", [5e-14, 1e-12, 9.9e-11])
def test_weighted_sum_paper_tolerances_give_boys_weighted_sum(tol):
    bt = _batches(seed=91)
    _, mask = _ws_bound(bt, EPS)
    assert np.array_equal(_ws(bt, tol=tol)[mask], _ws(bt)[mask])


def test_weighted_sum_invalid_tolerance_raises():
    bt = _batches(seed=92, nbatch=8)
    for tol in (1e-15, float("nan")):
        with pytest.raises(boys.BoysError):
            _ws(bt, tol=tol)


# --- the backward pass (boys_backward_tol, BoysFunction with tol) ------------

def _grad_bound(x, G, eps):
    kmax = G.shape[1] - 1
    F = oracle.boys(x, kmax + 1)[:, 1:]
    return eps * np.abs(G).sum(1) + 4 * (kmax + 2) * U * (np.abs(G) * F).sum(1)


@pytest.mark.parametrize("kmax", [0, 8, 16, 31])
def test_backward_screening_set(kmax):
    x, G = workloads.backward_workload(n=4000, kmax=kmax, seed=300 + kmax)
    x[:edge_arguments().size] = edge_arguments()
    g = boys.boys_backward(dev(x), dev(G), kmax, tol=1e-10).cpu().numpy()
    err = np.abs(g - oracle.backward(x, G))
    tol = _grad_bound(x, G, TOL)
    assert np.all(err <= tol), float(np.max(err / tol))


@pytest.mark.parametrize("kmax,tol", [(16, 5e-14), (16, 9.9e-11), (36, 1e-10), (39, 1.0)])
def test_backward_tolerances_that_select_the_paper_or_high_set(kmax, tol):
    x, G = workloads.backward_workload(n=3000, kmax=kmax, seed=400 + kmax)
    a = boys.boys_backward(dev(x), dev(G), kmax).cpu().numpy()
    b = boys.boys_backward(dev(x), dev(G), kmax, tol=tol).cpu().numpy()
    assert np.array_equal(a, b)


def test_autograd_with_screening_tolerance():
    x, G = workloads.backward_workload(n=3000, kmax=12, seed=500)
    xt = dev(x).requires_grad_(True)
    F = boys.BoysFunction.apply(xt, 12, 1e-10)
    F.backward(dev(G))
    assert np.abs(F.detach().cpu().numpy() - oracle.boys(x, 12)).max() <= TOL
    err = np.abs(xt.grad.cpu().numpy() - oracle.backward(x, G))
    assert np.all(err <= _grad_bound(x, G, TOL))
