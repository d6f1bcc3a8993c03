"""boys_weighted_sum_noalloc (the entry point that allocates nothing) against
boys_weighted_sum on the GPU.

Both run the same kernels with the same configuration, so the results must
be equal bit for bit; the oracle bound of the batched consumer is checked as
well.  Two calls in a row share the per-device scratch array, the second with
a smaller batch table; a captured call is replayed with eager work and
synchronisations between the replays."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_10059_amd as boys
from paper_2512_10059_amd import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
MAX_BATCHES = 65536


def to_dev(bt):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return (t(bt.x), t(bt.batch_off), t(bt.batch_n), t(bt.batch_kmax), t(bt.w), t(bt.w_off))


def within_oracle_bound(bt, out):
    """|out - oracle| <= 5e-14 sum_l |w_l| + 4 (k+1) 2^-53 sum_l |w_l F_l| per argument."""
    ref = oracle.weighted_sum(bt.x, bt.batch_off, bt.batch_n, bt.batch_kmax, bt.w, bt.w_off)
    for b in range(bt.batch_off.size):
        o, n, k, wo = (int(bt.batch_off[b]), int(bt.batch_n[b]), int(bt.batch_kmax[b]),
                       int(bt.w_off[b]))
        if n <= 0:
            continue
        wl = bt.w[wo:wo + k + 1]
        F = oracle.boys(bt.x[o:o + n], k)
        tol = 5e-14 * np.abs(wl).sum() + 4 * (k + 1) * 2.0**-53 * (np.abs(wl) * F).sum(1)
        assert np.all(np.abs(out[o:o + n] - ref[o:o + n]) <= tol), b


def test_two_calls_match_the_allocating_entry_point():
    big = workloads.batched_workload(nbatch=3000, seed=61, mean_size=400.0, max_size=6000)
    small = workloads.batched_workload(nbatch=120, seed=62, mean_size=300.0, max_size=3000)
    small.batch_n[::17] = 0  # empty batches
    for bt in (big, small):  # the second call is smaller: stale scratch entries must not matter
        args = to_dev(bt)
        out = torch.full_like(args[0], -7.0)
        boys.boys_weighted_sum_noalloc(*args, out=out)
        ref = torch.full_like(args[0], -7.0)
        boys.boys_weighted_sum(*args, out=ref)
        got = out.cpu().numpy()
        assert np.array_equal(got, ref.cpu().numpy())
        within_oracle_bound(bt, got)


def test_limit_and_empty():
    bt = workloads.batched_workload(nbatch=4, seed=63, mean_size=50.0, max_size=100)
    args = to_dev(bt)
    out = torch.zeros_like(args[0])
    n = MAX_BATCHES + 1
    big = [torch.zeros(n, dtype=a.dtype, device=DEV) for a in args[1:4]]
    with pytest.raises(boys.BoysError):
        boys.boys_weighted_sum_noalloc(args[0], big[0], big[1], big[2], args[4],
                                       torch.zeros(n, dtype=torch.int64, device=DEV), out=out)
    empty = [a[:0] for a in args[1:4]]
    boys.boys_weighted_sum_noalloc(args[0], *empty, args[4], args[5][:0], out=out)
    torch.cuda.synchronize()
    assert not out.any()


def test_captured_call_replays():
    """The call captured into a graph and replayed three times, the arguments
    changed in place by eager work between the replays: each replay equals an
    eager call on the same inputs."""
    bt = workloads.batched_workload(nbatch=500, seed=64, mean_size=300.0, max_size=4000)
    args = list(to_dev(bt))
    out = torch.zeros_like(args[0])
    boys.boys_weighted_sum_noalloc(*args, out=out)  # first call on the device: outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        boys.boys_weighted_sum_noalloc(*args, out=out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(65)
    for r in range(3):
        args[0].mul_(float(rng.uniform(0.5, 1.5)))  # eager work on the inputs
        args[4].copy_(torch.from_numpy(rng.standard_normal(bt.w.size)).to(DEV))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = torch.zeros_like(args[0])
        boys.boys_weighted_sum(*args, out=ref)
        assert torch.equal(out, ref), r
