"""boys_weighted_sum on the GPU against the CPU oracle.

Tolerance: the method's guarantee |F_l - F~_l| <= 5e-14 carried through the
weighted sum, |out - ref| <= 5e-14 * sum_l |w_l|, plus the rounding of the
(k+1)-term FP64 accumulation, 4 (k+1) 2^-53 sum_l |w_l F_l|."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_10059_amd as boys
from paper_2512_10059_amd import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
EPS_TOL = 5e-14


def to_dev(bt):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return (t(bt.x), t(bt.batch_off), t(bt.batch_n), t(bt.batch_kmax), t(bt.w), t(bt.w_off))


def tolerance(bt, batches=None):
    """Per-argument bound for the batches listed (default: all)."""
    tol = np.zeros(bt.x.size)
    idx = range(bt.batch_off.size) if batches is None else batches
    for b in idx:
        off, n, k, wo = (int(bt.batch_off[b]), int(bt.batch_n[b]), int(bt.batch_kmax[b]),
                         int(bt.w_off[b]))
        if n <= 0:
            continue
        wl = bt.w[wo:wo + k + 1]
        F = oracle.boys(bt.x[off:off + n], k)
        tol[off:off + n] = EPS_TOL * np.abs(wl).sum() + 4 * (k + 1) * 2.0**-53 * (np.abs(wl) * F).sum(1)
    return tol


def _configs():
    """Every configuration the library offers (read from it at collection;
    one placeholder when the library is not built, where every GPU test
    fails at its first call anyway)."""
    try:
        return range(boys.weighted_sum_num_configs())
    except Exception:  # library not built: collection must still succeed
        return range(1)


CONFIGS = _configs()


def small_batches(seed=0, nbatch=300, with_empty=True):
    bt = workloads.batched_workload(nbatch=nbatch, seed=seed, mean_size=300.0, sigma=1.2,
                                    max_size=5000)
    if with_empty:
        bt.batch_n[::37] = 0  # empty batches inside the table
    return bt


def check(bt, out, batches=None):
    ref = oracle.weighted_sum(bt.x, bt.batch_off, bt.batch_n, bt.batch_kmax, bt.w, bt.w_off)
    tol = tolerance(bt, batches)
    mask = np.zeros(bt.x.size, bool)
    for b in (range(bt.batch_off.size) if batches is None else batches):
        mask[int(bt.batch_off[b]):int(bt.batch_off[b]) + max(int(bt.batch_n[b]), 0)] = True
    err = np.abs(out - ref)
    bad = mask & ~(err <= tol)
    assert not bad.any(), f"{bad.sum()} outside bound; worst excess {np.max((err - tol)[mask]):.3e}"
    return err[mask].max()


def test_small_batches_default_config():
    bt = small_batches()
    args = to_dev(bt)
    out = boys.boys_weighted_sum(*args).cpu().numpy()
    check(bt, out)
    # arguments of empty batches are not written (output was zero-filled)
    for b in range(0, bt.batch_off.size, 37):
        assert np.all(out[int(bt.batch_off[b]):int(bt.batch_off[b]) + 1] == 0.0) or bt.batch_n[b] != 0


@pytest.mark.parametrize("config", CONFIGS)
def test_every_config_bitwise_equal(config):
    """Every tile/binning/carry-over configuration runs the same arithmetic per
    argument, so the results are bitwise identical across configurations."""
    bt = small_batches(seed=1)
    args = to_dev(bt)
    boys.weighted_sum_set_config(0)
    ref = boys.boys_weighted_sum(*args).cpu().numpy()
    boys.weighted_sum_set_config(config)
    try:
        out = boys.boys_weighted_sum(*args).cpu().numpy()
    finally:
        boys.weighted_sum_set_config(-1)
    assert np.array_equal(out, ref, equal_nan=True)
    if config == 0:
        check(bt, out)


def test_orders_and_domain_edges():
    """Batches of one argument, orders 0 and 32, region boundaries, x = 0,
    +inf (0), NaN and negative x (NaN)."""
    X0, X1 = 11.899848152108484, 28.98933773882074
    xs = np.array([0.0, 1e-300, X0, np.nextafter(X0, 0), X1, np.nextafter(X1, 99), 30.0, 1e6,
                   np.inf, np.nan, -1.0])
    m = xs.size
    nb = 2 * m
    x = np.concatenate([xs, xs])
    off = np.arange(nb, dtype=np.int64)
    n = np.ones(nb, dtype=np.int32)
    k = np.array([0] * m + [32] * m, dtype=np.int32)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(m * 1 + m * 33)
    w_off = np.concatenate([np.arange(m), m + 33 * np.arange(m)]).astype(np.int64)
    bt = workloads.Batches(x=x, batch_off=off, batch_n=n, batch_kmax=k, w=w, w_off=w_off)
    out = boys.boys_weighted_sum(*to_dev(bt)).cpu().numpy()
    finite = np.isfinite(x) & (x >= 0)
    ok = np.ones(nb, bool)
    ok[~finite] = False
    ref = oracle.weighted_sum(x, off, n, k, w, w_off)
    tol = tolerance(bt)
    assert np.all(np.abs(out - ref)[ok] <= tol[ok])
    assert np.all(out[np.isposinf(x)] == 0.0)
    assert np.all(np.isnan(out[np.isnan(x) | (x < 0)]))


def test_graph_reuse_and_in_place_table_change():
    """The cached graph is reused for identical arguments and reads the batch
    table on the device, so an in-place change of the orders is honoured."""
    bt = small_batches(seed=2, with_empty=False)
    args = list(to_dev(bt))
    out = torch.zeros_like(args[0])
    boys.boys_weighted_sum(*args, out=out)
    a = out.cpu().numpy().copy()
    boys.boys_weighted_sum(*args, out=out)
    assert np.array_equal(out.cpu().numpy(), a)
    newk = np.minimum(bt.batch_kmax, 3).astype(np.int32)
    args[3].copy_(torch.from_numpy(newk))
    boys.boys_weighted_sum(*args, out=out)
    bt.batch_kmax = newk
    check(bt, out.cpu().numpy())


def test_workspace_growth_leaves_enqueued_work_intact():
    """A call that has to grow the workspace, enqueued right behind one that
    uses the old workspace (no synchronisation in between): the library
    retires the old workspace instead of waiting for the device, and both
    results are right."""
    boys.finalize()  # start from no workspace
    small = small_batches(seed=6, nbatch=300)
    large = small_batches(seed=7, nbatch=5000)
    a_small, a_large = to_dev(small), to_dev(large)
    out_small = boys.boys_weighted_sum(*a_small)
    out_large = boys.boys_weighted_sum(*a_large)  # 5001 > 1024 prefix entries: grows
    # Another output array: the cached graph is replaced while the previous
    # launches may still be queued (the old graph is retired behind an event).
    out_again = boys.boys_weighted_sum(*a_large)
    check(small, out_small.cpu().numpy())
    check(large, out_large.cpu().numpy())
    assert torch.equal(out_again, out_large)


def test_capturing_stream_is_refused():
    """Under graph capture the graph-cached entry point enqueues nothing and
    returns BOYS_ECAPTURE (its workspace and graph are per device, so a
    captured replay would share them with later calls)."""
    bt = small_batches(seed=9)
    args = to_dev(bt)
    out = torch.zeros_like(args[0])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(boys.BoysError, match="capture"):
        with torch.cuda.graph(g):
            boys.boys_weighted_sum(*args, out=out)
    torch.cuda.synchronize()
    assert not out.any()  # nothing ran
    check(bt, boys.boys_weighted_sum(*args, out=out).cpu().numpy())  # ordinary calls still work


def test_tuner_picks_a_valid_config():
    bt = small_batches(seed=3)
    args = to_dev(bt)
    cfg, ms, name = boys.boys_tune_weighted_sum(*args)
    assert 0 <= cfg < boys.weighted_sum_num_configs() and ms > 0 and name != "invalid"
    assert boys.weighted_sum_get_config() == cfg
    out = boys.boys_weighted_sum(*args).cpu().numpy()
    check(bt, out)
    boys.weighted_sum_set_config(-1)


def test_tuning_cache_file(tmp_path, monkeypatch):
    """BOYS_TUNE_CACHE: a missing file, garbage, another architecture, another
    table set or bucket, and an unknown configuration name all leave the
    default; a matching line selects its configuration, and the last
    matching line wins."""
    bt = small_batches(seed=11)
    args = to_dev(bt)
    nb = bt.batch_off.size
    bucket = int(np.floor(np.log2(nb)))
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    names = [boys.weighted_sum_config_name(c) for c in range(boys.weighted_sum_num_configs())]
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("BOYS_TUNE_CACHE", str(path))

    def chosen(text):
        if text is None:
            if path.exists():
                path.unlink()
        else:
            path.write_bytes(text if isinstance(text, bytes) else text.encode())
        boys.weighted_sum_set_config(-1)  # the next call consults the cache
        out = boys.boys_weighted_sum(*args).cpu().numpy()
        check(bt, out)
        return boys.weighted_sum_get_config()

    try:
        default = chosen(None)
        other = (default + 1) % len(names)
        assert chosen(b"\x00\xff garbage\n\nweighted_sum\n1 2 3\n") == default
        assert chosen(f"weighted_sum gfx942 0 {bucket} {names[other]}\n") == default
        assert chosen(f"weighted_sum {arch} 1 {bucket} {names[other]}\n") == default
        assert chosen(f"weighted_sum {arch} 0 {bucket + 1} {names[other]}\n") == default
        assert chosen(f"weighted_sum {arch} 0 {bucket} no-such-config\n") == default
        assert chosen(f"weighted_sum {arch} 0 {bucket} {names[other]}\n") == other
        assert chosen(f"weighted_sum {arch} 0 {bucket} {names[other]}\n"
                      f"weighted_sum {arch} 0 {bucket} {names[default]}\n") == default
        # The tuner appends its choice under the same key.
        path.unlink()
        cfg, ms, name = boys.boys_tune_weighted_sum(*args)
        lines = path.read_text().split("\n")
        assert lines[0].split() == ["weighted_sum", arch, "0", str(bucket), name]
    finally:
        boys.weighted_sum_set_config(-1)


def test_invalid_arguments_raise():
    bt = small_batches(seed=4)
    args = list(to_dev(bt))
    with pytest.raises(boys.BoysError):
        boys.boys_weighted_sum(args[0].float(), *args[1:])
    with pytest.raises(boys.BoysError):
        boys.boys_weighted_sum(args[0], args[1][:-1], *args[2:])


def test_full_batched_workload_sampled():
    """The full batched workload (8192 batches, lognormal sizes with mean 4096,
    orders uniform on 0..32): 400 sampled batches completely and the first
    argument of every batch against the oracle."""
    bt = workloads.batched_workload()
    args = to_dev(bt)
    out = boys.boys_weighted_sum(*args).cpu().numpy()
    rng = np.random.default_rng(8)
    sample = rng.choice(bt.batch_off.size, 400, replace=False)
    check(bt, out, batches=sample)
    firsts = bt.batch_off
    k = bt.batch_kmax
    F = oracle.boys(bt.x[firsts], 32)
    ref = np.array([(bt.w[bt.w_off[b]:bt.w_off[b] + k[b] + 1] * F[b, :k[b] + 1]).sum()
                    for b in range(firsts.size)])
    tol = np.array([EPS_TOL * np.abs(bt.w[bt.w_off[b]:bt.w_off[b] + k[b] + 1]).sum() * 1.01
                    for b in range(firsts.size)])
    assert np.all(np.abs(out[firsts] - ref) <= tol)


def test_graph_replays_with_eager_work_between():
    """The cached graph replayed five times, with unrelated eager work (fills,
    other library kernels) and synchronisations between the replays: every
    replay equals the first result bitwise."""
    bt = small_batches(seed=6)
    args = to_dev(bt)
    out = torch.zeros_like(args[0])
    boys.boys_weighted_sum(*args, out=out)
    torch.cuda.synchronize()
    first = out.cpu().numpy().copy()
    scratch = torch.empty(1 << 20, dtype=torch.float64, device=DEV)
    for r in range(5):
        out.fill_(float(r) - 7.0)
        scratch.uniform_()
        boys.boys_eval_f64(scratch[:4096].abs() * 40, 12)
        torch.cuda.synchronize()
        boys.boys_weighted_sum(*args, out=out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        mask = np.zeros(got.size, bool)
        for o, n in zip(bt.batch_off, bt.batch_n):
            mask[int(o):int(o) + max(int(n), 0)] = True
        assert np.array_equal(got[mask], first[mask]), f"replay {r} differs"


def test_side_stream():
    """Launches go to the caller's current stream: a non-default stream gives
    the same result."""
    bt = small_batches(seed=7)
    args = to_dev(bt)
    ref = boys.boys_weighted_sum(*args).cpu().numpy()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = boys.boys_weighted_sum(*args)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)


def test_more_batches_than_one_scan_round():
    """20011 batches (the cost scan takes the table in rounds of 8192, so
    this needs three, the last one ragged), sizes 1..60, every argument
    against the oracle."""
    rng = np.random.default_rng(11)
    nb = 20011
    n = rng.integers(0, 61, nb).astype(np.int32)
    off = np.concatenate([[0], np.cumsum(n[:-1])]).astype(np.int64)
    k = rng.integers(0, 33, nb).astype(np.int32)
    w_off = np.concatenate([[0], np.cumsum(k[:-1] + 1)]).astype(np.int64)
    w = rng.standard_normal(int((k + 1).sum()))
    x = workloads.gaussian_pair_arguments(int(n.sum()), seed=12)
    bt = workloads.Batches(x=x, batch_off=off, batch_n=n, batch_kmax=k, w=w, w_off=w_off)
    out = boys.boys_weighted_sum(*to_dev(bt)).cpu().numpy()
    check(bt, out)


@pytest.mark.parametrize("config", CONFIGS)
def test_partial_tiles_write_only_their_batch(config):
    """Batches separated by gaps in the argument and output arrays, with sizes
    around the tile lengths (1..1100: every partial-tile shape of tiles of 128,
    256 and 512): every argument of every batch matches the oracle, and the
    gaps keep the sentinel the output was filled with.  The last batch ends at
    the end of both arrays, so a load or store past a tile would leave them."""
    rng = np.random.default_rng(21)
    n = np.array([1, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 700, 1023, 1024, 1100, 5, 0, 3],
                 dtype=np.int32)
    gap = rng.integers(1, 40, n.size)
    off = np.zeros(n.size, np.int64)
    pos = 0
    for b in range(n.size):
        pos += int(gap[b])
        off[b] = pos
        pos += int(n[b])
    total = pos  # the last batch ends the arrays
    k = rng.integers(0, 33, n.size).astype(np.int32)
    w_off = np.concatenate([[0], np.cumsum(k[:-1] + 1)]).astype(np.int64)
    w = rng.standard_normal(int((k + 1).sum()))
    x = workloads.gaussian_pair_arguments(total, seed=22)
    bt = workloads.Batches(x=x, batch_off=off, batch_n=n, batch_kmax=k, w=w, w_off=w_off)
    sentinel = -12345.0
    out_dev = torch.full((total,), sentinel, dtype=torch.float64, device=DEV)
    boys.weighted_sum_set_config(config)
    try:
        out = boys.boys_weighted_sum(*to_dev(bt), out=out_dev).cpu().numpy()
    finally:
        boys.weighted_sum_set_config(-1)
    check(bt, out)
    inside = np.zeros(total, bool)
    for b in range(n.size):
        inside[off[b]:off[b] + n[b]] = True
    assert np.all(out[~inside] == sentinel)


@pytest.mark.parametrize("nb", [1, 8191, 8192, 8193, 16384])
def test_batch_counts_around_scan_rounds(nb):
    """The cost scan takes the batch table in rounds of 8192 entries: one
    batch, one short of a round, exactly one and two rounds, and one entry
    into a second round, with sizes 0..9 (empty batches included), every
    argument against the oracle."""
    rng = np.random.default_rng(31 + nb)
    n = rng.integers(0, 10, nb).astype(np.int32)
    if nb == 1:
        n[0] = 7
    off = np.concatenate([[0], np.cumsum(n[:-1])]).astype(np.int64)
    k = rng.integers(0, 33, nb).astype(np.int32)
    w_off = np.concatenate([[0], np.cumsum(k[:-1] + 1)]).astype(np.int64)
    w = rng.standard_normal(int((k + 1).sum()))
    x = workloads.gaussian_pair_arguments(int(n.sum()), seed=32)
    bt = workloads.Batches(x=x, batch_off=off, batch_n=n, batch_kmax=k, w=w, w_off=w_off)
    out = boys.boys_weighted_sum(*to_dev(bt)).cpu().numpy()
    check(bt, out)
