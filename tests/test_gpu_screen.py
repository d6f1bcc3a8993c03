"""The screening table set (eps_tol = 1e-10) through boys_eval_f64_tol and
boys_pairsum_tol on the GPU, against the long-double oracle.

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
