"""The per-kmax and centre-of-anti-diagonal table variants (boys_set_tables)
on the GPU against the CPU oracle, through every forward entry point that
takes them: the write-out (boys_eval_f64), the batched consumer
(boys_weighted_sum and its allocation-free twin) and the pair sums.

Bars: 5e-14 absolute per value for the write-out (each variant's
guarantee); the weighted-sum and pair-sum bounds of test_gpu_weighted_sum and
test_gpu_pairsum.  Arguments include each variant's own region ends x0(K)
and x1(K) with their neighbouring doubles, where the per-kmax set switches
regions at other points than the paper's."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_10059_amd as boys
from paper_2512_10059_amd import workloads
from tests.test_coeff_tables_perk import CT, PK
from tests.test_gpu_pairsum import check as pair_check
from tests.test_gpu_weighted_sum import check as ws_check
from tests.test_gpu_weighted_sum import small_batches, to_dev

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
EPS_TOL = 5e-14
VARIANTS = {"per_kmax": 1, "centre": 2}


def around(v, steps=3):
    out = []
    for _ in range(steps):
        v = np.nextafter(v, 0.0)
    for _ in range(2 * steps + 1):
        out.append(v)
        v = np.nextafter(v, np.inf)
    return out


def edges(K):
    pts = [0.0, 5e-324, 1e-12, 0.5, 1.0, 2.0, 30.0, 1e3, 1e300]
    for b in (PK[K]["x0"], PK[K]["x1"], CT["x0"], CT["x1"]):
        pts += around(b)
    return np.array(pts)


def eval_f64(x, kmax):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    F = boys.boys_eval_f64(xt, kmax)
    torch.cuda.synchronize()
    return F.cpu().numpy()


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kmax", [0, 1, 2, 3, 4, 5, 7, 8, 12, 16, 20, 23, 27, 31, 32])
def test_writeout_parity(variant, kmax):
    x = np.concatenate([workloads.mixed_arguments(n=8192, seed=40 + kmax), edges(kmax),
                        np.linspace(0.0, 35.0, 4001)])
    with boys.table_variant(VARIANTS[variant]):
        F = eval_f64(x, kmax)
    err = np.abs(F - oracle.boys(x, kmax))
    i = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= EPS_TOL, f"{variant} kmax={kmax}: {err.max():.3e} at x={x[i[0]]!r}, order {i[1]}"


def test_writeout_variants_differ_only_within_the_bound():
    """The three variants give different roundings, not different functions:
    per value within 1e-13 of each other, and the paper's variant is the
    default after the context manager."""
    x = workloads.gaussian_pair_arguments(n=20000, seed=11)
    ref = eval_f64(x, 9)
    for v in VARIANTS.values():
        with boys.table_variant(v):
            assert np.abs(eval_f64(x, 9) - ref).max() <= 2 * EPS_TOL
    assert boys.get_tables() == 0
    assert np.array_equal(eval_f64(x, 9), ref)


def boundary_batches(rng):
    """One batch per order 0..32 holding the per-kmax and the paper's region
    ends of that order with their neighbours, plus random arguments."""
    xs, off, n, k = [], [], [], []
    pos = 0
    for K in range(33):
        pts = np.concatenate([edges(K), rng.uniform(0.0, 35.0, 200)])
        xs.append(pts)
        off.append(pos)
        n.append(pts.size)
        k.append(K)
        pos += pts.size
    kk = np.array(k, np.int32)
    w_off = np.zeros(33, np.int64)
    w_off[1:] = np.cumsum(kk.astype(np.int64) + 1)[:-1]
    return workloads.Batches(x=np.concatenate(xs), batch_off=np.array(off, np.int64),
                             batch_n=np.array(n, np.int32), batch_kmax=kk,
                             w=rng.standard_normal(int((kk + 1).sum())), w_off=w_off)


@pytest.mark.parametrize("variant", VARIANTS)
def test_weighted_sum_parity(variant):
    rng = np.random.default_rng(7)
    for bt in (small_batches(seed=21), boundary_batches(rng)):
        args = to_dev(bt)
        with boys.table_variant(VARIANTS[variant]):
            out = boys.boys_weighted_sum(*args)
            torch.cuda.synchronize()
        ws_check(bt, out.cpu().numpy())


@pytest.mark.parametrize("variant", VARIANTS)
def test_weighted_sum_every_configuration(variant):
    bt = small_batches(seed=22)
    args = to_dev(bt)
    prev = boys.weighted_sum_get_config()
    try:
        with boys.table_variant(VARIANTS[variant]):
            for cfg in range(boys.weighted_sum_num_configs()):
                boys.weighted_sum_set_config(cfg)
                out = boys.boys_weighted_sum(*args)
                torch.cuda.synchronize()
                ws_check(bt, out.cpu().numpy())
    finally:
        boys.weighted_sum_set_config(prev)


def test_weighted_sum_switching_variants_rebuilds_nothing_stale():
    """Calls on the same buffers alternating between variants each give that
    variant's result (the cached graphs are kept per table set), and the
    allocation-free entry point follows the variant too, bit for bit."""
    bt = small_batches(seed=23)  # with empty batches: their arguments stay untouched
    args = to_dev(bt)
    fresh = {}
    for v in (0, 1, 2):
        with boys.table_variant(v):
            fresh[v] = boys.boys_weighted_sum(*args, out=torch.full_like(args[0], -1.0)).cpu().numpy()
    assert not np.array_equal(fresh[0], fresh[1])
    out = torch.empty_like(args[0])
    for v in (1, 0, 2, 1, 0):
        with boys.table_variant(v):
            out.fill_(-1.0)
            boys.boys_weighted_sum(*args, out=out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), fresh[v]), v
            out.fill_(-1.0)
            boys.boys_weighted_sum_noalloc(*args, out=out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), fresh[v]), ("noalloc", v)


def test_weighted_sum_screening_ignores_the_variant():
    bt = small_batches(seed=24)
    args = to_dev(bt)
    ref = boys.boys_weighted_sum(*args, tol=1e-10).cpu().numpy()
    with boys.table_variant(1):
        assert np.array_equal(boys.boys_weighted_sum(*args, tol=1e-10).cpu().numpy(), ref)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kmax", [0, 2, 5, 7, 12, 20, 31, 32])
def test_pairsum_parity(variant, kmax):
    x, y, c = workloads.pair_workload(n=600, kmax=kmax, seed=60 + kmax, x_max=20.0)
    x = np.concatenate([x, np.array(edges(kmax)[:30]) / 2])
    y = np.concatenate([y, np.ones(30)])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)
    with boys.table_variant(VARIANTS[variant]):
        z = boys.boys_pairsum(t(x), t(y), c)
        torch.cuda.synchronize()
    pair_check(x, y, c, z.cpu().numpy(), np.arange(0, x.size, 3))
