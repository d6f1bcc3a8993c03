#!/usr/bin/env python3
"""Benchmark of the Boys-function library on one MI355X.

Headline (one step = one write-out evaluation): F_0..F_32 in FP64 for 2^26
Gaussian-pair arguments x = ab/(a+b) R^2, written as a row-major 2^26 x 33
array (18.25 GB of algorithmic traffic per step).  The metric is Boys values
per second, N (kmax+1) / time, at max abs error <= 5e-14.

Beside the headline the same JSON line carries:
  roofline      achieved GB/s of the write-out kernel (algorithmic bytes /
                average launch time from HIP events) against 8 TB/s, and the
                HBM traffic measured by rocprofv3 counters when the committed
                counter summary matches the current kernel sources;
  cpu_baseline  the long-double CPU oracle on the first 2^25 arguments
                (all host cores), with the max abs error of the GPU rows there;
  legs          the small mixed-argument configuration (65 536 arguments,
                kmax=8; launch-bound), FP32 vs FP64 at kmax=16 on the same
                arguments, the batched
                fused consumer (8192 batches), the differentiation pass
                (2^24 arguments, kmax=16, forward + backward; backward also
                at kmax=30), the paper's
                own N^2 benchmark (n = 2^19, k = 12) beside its A100 time, and
                the screening table set (eps_tol = 1e-10) on the write-out
                and pair-sum workloads, the write-out at kmax = 40 (the
                high-order tables), and the variants of the 5e-14 tables
                (per-kmax regions, centre-of-anti-diagonal degrees) on the
                fused, write-out and pair-sum work.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3]
       [--only writeout,mixed,fp32,fused,backward,pairsum,screen,high,variants]
       [--no-cpu-baseline] [--copy-probe]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Boys values/s (x·(kmax+1)) at max abs err ≤5e-14 FP64; FP32 vs FP64 speedup"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
PMC_SUMMARY = os.path.join(ROOT, "profiles", "eval_f64_writeout_k32_n2e26_pmc.md")
KERNEL_SOURCES = ["paper_2512_10059_amd/csrc/boys_eval_f64.hip",
                  "paper_2512_10059_amd/csrc/boys_device_f64.hpp",
                  "paper_2512_10059_amd/csrc/boys_coeffs_f64.h",
                  "paper_2512_10059_amd/csrc/boys_coeffs_f64_perk.h",
                  "paper_2512_10059_amd/csrc/boys_coeffs_f64_centre.h",
                  "paper_2512_10059_amd/csrc/boys_common.hpp",
                  "paper_2512_10059_amd/build.py"]


FUSED_KT_SUMMARY = os.path.join(ROOT, "profiles", "weighted_sum_8192_batches_kernel_stats.md")
FUSED_PMC_SUMMARY = os.path.join(ROOT, "profiles", "weighted_sum_8192_batches_pmc.md")
FUSED_SOURCES = ["paper_2512_10059_amd/csrc/boys_weighted_sum.hip",
                 "paper_2512_10059_amd/csrc/boys_device_f64_batched.hpp",
                 "paper_2512_10059_amd/csrc/boys_device_f64.hpp",
                 "paper_2512_10059_amd/csrc/boys_coeffs_f64.h",
                 "paper_2512_10059_amd/csrc/boys_coeffs_f64_screen.h",
                 "paper_2512_10059_amd/csrc/boys_coeffs_f64_perk.h",
                 "paper_2512_10059_amd/csrc/boys_coeffs_f64_centre.h",
                 "paper_2512_10059_amd/csrc/boys_consumer_tables.h",
                 "paper_2512_10059_amd/build.py"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def summary_values(path, sources):
    """The '- key: value' lines of a committed profile summary, or None when
    it is missing or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    vals = dict(re.findall(r"^- (\w+): (\S+)\s*$", open(path).read(), re.M))
    return vals if vals.get("source_sha256") == kernel_source_hash(sources) else None


def pmc_traffic_bytes():
    """HBM bytes per write-out launch from the committed counter summary, or
    None when it is missing or was taken on other kernel sources."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    vals = dict(re.findall(r"^- (\w+): ([0-9.eE+-]+|[0-9a-f]+)\s*$", text, re.M))
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    try:
        fetch = float(vals["fetch_kib_per_dispatch"]) * float(vals["fetch_scale"])
        write = float(vals["write_kib_per_dispatch"]) * float(vals["write_scale"])
    except KeyError:
        return None
    return (fetch + write) * 1024.0


class Timer:
    """HIP events on the current (launch) stream around a region."""

    def __init__(self, torch):
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.t0 = time.perf_counter()
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self.torch.cuda.synchronize()
        self.wall = time.perf_counter() - self.t0
        self.ms = self.a.elapsed_time(self.b)


def leg_writeout(torch, boys, workloads, steps, warmup, dev):
    n, kmax = workloads.N_WRITEOUT, 32
    log(f"write-out: generating {n} arguments")
    x_host = workloads.gaussian_pair_arguments(n)
    x = torch.from_numpy(x_host).to(dev)
    out = torch.empty((n, kmax + 1), dtype=torch.float64, device=dev)
    for _ in range(warmup):
        boys.boys_eval_f64(x, kmax, out=out)
    with Timer(torch) as t:
        for _ in range(steps):
            boys.boys_eval_f64(x, kmax, out=out)
    ms = t.ms / steps
    alg_bytes = n * 8 * (kmax + 2)
    log(f"write-out: {ms:.3f} ms/step, {alg_bytes / ms / 1e6:.0f} GB/s")
    return dict(x_host=x_host, x=x, out=out, ms=ms, wall=t.wall, n=n, kmax=kmax,
                alg_bytes=alg_bytes)


def leg_mixed(torch, boys, workloads, dev, calls=500):
    """The small plain-FP64 configuration: 65 536 arguments in four equal
    quarters (U[0,1], U[1,30], log-uniform [30,1e4], exact zeros or U[0,1e-6]),
    kmax = 8.  At 5.2 MB per call it is bound by launch latency, not by HBM:
    timed as back-to-back calls on one stream and as replays of a captured
    graph of the same calls."""
    kmax = 8
    x = torch.from_numpy(workloads.mixed_arguments()).to(dev)
    n = x.numel()
    out = torch.empty((n, kmax + 1), dtype=torch.float64, device=dev)
    for _ in range(20):
        boys.boys_eval_f64(x, kmax, out=out)
    with Timer(torch) as t:
        for _ in range(calls):
            boys.boys_eval_f64(x, kmax, out=out)
    eager_us = t.ms * 1e3 / calls
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    per_graph = 50
    with torch.cuda.stream(side):
        boys.boys_eval_f64(x, kmax, out=out)
        torch.cuda.current_stream().synchronize()
        with torch.cuda.graph(g, stream=side):
            for _ in range(per_graph):
                boys.boys_eval_f64(x, kmax, out=out)
    torch.cuda.current_stream().wait_stream(side)
    g.replay()
    reps = max(1, calls // per_graph)
    with Timer(torch) as tg:
        for _ in range(reps):
            g.replay()
    graph_us = tg.ms * 1e3 / (reps * per_graph)
    values = n * (kmax + 1)
    log(f"mixed: {eager_us:.2f} us per call, {graph_us:.2f} us per call in a graph")
    return {"n": n, "kmax": kmax, "us_per_call": eager_us, "us_per_call_graph": graph_us,
            "values_per_s": values / (eager_us * 1e-6),
            "values_per_s_graph": values / (graph_us * 1e-6),
            "gbs_graph": n * 8 * (kmax + 2) / (graph_us * 1e3)}


def leg_fp32(torch, boys, workloads, steps, warmup, dev, x_host=None):
    n, kmax = workloads.N_WRITEOUT, 16
    if x_host is None:
        x_host = workloads.gaussian_pair_arguments(n)
    x32 = torch.from_numpy(x_host.astype(np.float32)).to(dev)
    x64 = x32.double()
    o32 = torch.empty((n, kmax + 1), dtype=torch.float32, device=dev)
    o64 = torch.empty((n, kmax + 1), dtype=torch.float64, device=dev)
    res = {}
    for name, fn, xx, oo in (("f32", boys.boys_eval_f32, x32, o32), ("f64", boys.boys_eval_f64, x64, o64)):
        for _ in range(warmup):
            fn(xx, kmax, out=oo)
        with Timer(torch) as t:
            for _ in range(steps):
                fn(xx, kmax, out=oo)
        res[name] = t.ms / steps
    b32, b64 = n * 4 * (kmax + 2), n * 8 * (kmax + 2)
    log(f"fp32: {res['f32']:.3f} ms vs fp64 {res['f64']:.3f} ms")
    return {"n": n, "kmax": kmax, "ms_f32": res["f32"], "ms_f64": res["f64"],
            "speedup_f32_vs_f64": res["f64"] / res["f32"],
            "values_per_s_f32": n * (kmax + 1) / (res["f32"] * 1e-3),
            "gbs_f32": b32 / (res["f32"] * 1e6), "gbs_f64": b64 / (res["f64"] * 1e6),
            "_x32": x32, "_o32": o32}


def algorithmic_flops(x, k, deg_nm):
    """Operation count of the method per argument (FMA = 2, exp, sqrt and
    division = 1 each): region A 2(n_k+m_k) + 2 + 3k, region B 25 + 3k,
    region C 2 + 2k; the fused consumer adds 2(k+1) for the weighted sum."""
    X0, X1 = 11.899848152108484, 28.98933773882074
    a = x < X0
    c = x > X1
    b = ~a & ~c
    nm = np.array([n + m for n, m in deg_nm])[k]
    return (a * (2 * nm + 2 + 3 * k) + b * (25 + 3 * k) + c * (2 + 2 * k) + 2 * (k + 1)).sum()


def leg_fused(torch, boys, workloads, steps, warmup, dev):
    bt = workloads.batched_workload()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    args = (t(bt.x), t(bt.batch_off), t(bt.batch_n), t(bt.batch_kmax), t(bt.w), t(bt.w_off))
    out = torch.zeros_like(args[0])
    cfg, tune_ms, name = boys.boys_tune_weighted_sum(*args, out=out)
    for _ in range(warmup):
        boys.boys_weighted_sum(*args, out=out)
    with Timer(torch) as tm:
        for _ in range(steps):
            boys.boys_weighted_sum(*args, out=out)
    ms = tm.ms / steps
    # The same calls with the screening tables (eps_tol = 1e-10), same
    # configuration.
    for _ in range(warmup):
        boys.boys_weighted_sum(*args, out=out, tol=1e-10)
    with Timer(torch) as ts:
        for _ in range(steps):
            boys.boys_weighted_sum(*args, out=out, tol=1e-10)
    ms_screen = ts.ms / steps
    kk = np.repeat(bt.batch_kmax.astype(np.int64), bt.batch_n.astype(np.int64))
    values = int((kk + 1).sum())
    from paper_2512_10059_amd.tables import f64_region_a_degrees
    flops = float(algorithmic_flops(bt.x, kk, f64_region_a_degrees()))
    nbytes = bt.x.size * 16 + bt.w.size * 8 + bt.batch_n.size * 24
    log(f"fused: {ms:.3f} ms, config {name}; screening tables {ms_screen:.3f} ms")
    res = {"nbatch": int(bt.batch_n.size), "arguments": int(bt.x.size), "values": values,
           "ms": ms, "config": name, "tune_ms": tune_ms, "ms_screen_1e-10": ms_screen,
           "values_per_s": values / (ms * 1e-3),
           "algorithmic_flop_per_call": flops,
           "algorithmic_tflops": flops / (ms * 1e-3) / 1e12,
           "fp64_peak_frac_algorithmic": flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
           "gbs": nbytes / (ms * 1e6)}
    # The persistent kernel alone (a call is the scan, this kernel and the
    # graph's launch gaps), from the committed rocprofv3 summaries when they
    # were taken on the current sources: its median duration, the
    # algorithmic and the issued FP64 rates against the 78.6 TFLOP/s peak.
    kt = summary_values(FUSED_KT_SUMMARY, FUSED_SOURCES)
    pmc = summary_values(FUSED_PMC_SUMMARY, FUSED_SOURCES)
    kernel = None
    if kt is not None:
        us = float(kt["main_kernel_median_us"])
        kernel = {"name": kt.get("main_kernel"), "median_us": us,
                  "algorithmic_tflops": flops / (us * 1e-6) / 1e12,
                  "fp64_peak_frac_algorithmic": flops / (us * 1e-6) / 1e12 / FP64_PEAK_TFLOPS,
                  "issued_fp64_flop": None, "fp64_peak_frac_issued": None,
                  "gbs": nbytes / (us * 1e3)}
        if pmc is not None:
            issued = float(pmc["issued_fp64_flop_per_dispatch"])
            kernel["issued_fp64_flop"] = issued
            kernel["fp64_peak_frac_issued"] = issued / (us * 1e-6) / 1e12 / FP64_PEAK_TFLOPS
    res["kernel_from_profiles"] = kernel
    return res


def leg_backward(torch, boys, workloads, steps, warmup, dev):
    n, kmax = workloads.N_BACKWARD, 16
    x_host, G_host = workloads.backward_workload(n=n, kmax=kmax)
    x = torch.from_numpy(x_host).to(dev)
    G = torch.from_numpy(G_host).to(dev)
    F = torch.empty((n, kmax + 1), dtype=torch.float64, device=dev)
    g = torch.empty_like(x)
    for _ in range(warmup):
        boys.boys_eval_f64(x, kmax, out=F)
        boys.boys_backward(x, G, kmax, out=g)
    with Timer(torch) as tf:
        for _ in range(steps):
            boys.boys_eval_f64(x, kmax, out=F)
    with Timer(torch) as tb:
        for _ in range(steps):
            boys.boys_backward(x, G, kmax, out=g)
    fms, bms = tf.ms / steps, tb.ms / steps
    del G, F
    # The same pass at kmax = 30, where the gradient rows reach LDS by
    # LDS-DMA loads during the evaluation.
    k_hi = 30
    _, G_hi = workloads.backward_workload(n=n, kmax=k_hi)
    G = torch.from_numpy(G_hi).to(dev)
    del G_hi
    for _ in range(warmup):
        boys.boys_backward(x, G, k_hi, out=g)
    with Timer(torch) as th:
        for _ in range(steps):
            boys.boys_backward(x, G, k_hi, out=g)
    hms = th.ms / steps
    del G
    log(f"backward: forward {fms:.3f} ms, backward {bms:.3f} ms, backward at kmax {k_hi} {hms:.3f} ms")
    return {"n": n, "kmax": kmax, "ms_forward": fms, "ms_backward": bms,
            "gbs_forward": n * 8 * (kmax + 2) / (fms * 1e6),
            "gbs_backward": n * 8 * (kmax + 3) / (bms * 1e6),
            "ms_backward_kmax30": hms, "gbs_backward_kmax30": n * 8 * (k_hi + 3) / (hms * 1e6)}


def leg_pairsum(torch, boys, workloads, steps, dev):
    """The paper's own benchmark configuration (Sec. III, Algorithm 2): n = 2^19
    arguments, k = 12, n^2 = 2^38 evaluations.  The paper reports 72 s for it
    on an NVIDIA A100 (OpenACC); quoted as context, not as a target."""
    n, kmax = 1 << 19, 12
    xh, yh, c = workloads.pair_workload(n=n, kmax=kmax)
    x = torch.from_numpy(xh).to(dev)
    y = torch.from_numpy(yh).to(dev)
    z = torch.empty_like(x)
    boys.boys_pairsum(x, y, c, out=z)  # warm-up (workspace, sort)
    reps = max(1, min(steps, 3))
    with Timer(torch) as t:
        for _ in range(reps):
            boys.boys_pairsum(x, y, c, out=z)
    s = t.ms / reps / 1e3
    pairs = float(n) * n
    # Region mix of x_i + x_j with x uniform on [0, 30] (triangular density).
    X0, X1 = 11.899848152108484, 28.98933773882074
    pa = X0 * X0 / 1800.0
    pc = 1.0 - X1 * X1 / 1800.0
    pb = 1.0 - pa - pc
    from paper_2512_10059_amd.tables import f64_region_a_degrees
    nm = sum(f64_region_a_degrees()[kmax])
    flops_pair = pa * (2 * nm + 2 + 3 * kmax) + pb * (25 + 3 * kmax) + pc * (2 + 2 * kmax) + 2 * (kmax + 1) + 2
    log(f"pairsum: {s:.3f} s per call (paper, A100: 72 s)")
    return {"n": n, "kmax": kmax, "seconds": s, "pairs_per_s": pairs / s,
            "values_per_s": pairs * (kmax + 1) / s,
            "algorithmic_tflops": pairs * flops_pair / s / 1e12,
            "fp64_peak_frac_algorithmic": pairs * flops_pair / s / 1e12 / FP64_PEAK_TFLOPS,
            "paper_a100_seconds": 72.0, "paper_xeon6338_seconds_at_n2e14": 40.4}


def leg_screen(torch, boys, workloads, steps, warmup, dev, wo=None):
    """The screening table set (eps_tol = 1e-10): the write-out launch of the
    headline workload and the pair sums of the paper's benchmark, each timed
    like its 5e-14 counterpart."""
    n, kmax, tol = workloads.N_WRITEOUT, 32, 1e-10
    x = wo["x"] if wo else torch.from_numpy(workloads.gaussian_pair_arguments(n)).to(dev)
    out = torch.empty((n, kmax + 1), dtype=torch.float64, device=dev)
    for _ in range(warmup):
        boys.boys_eval_f64_tol(x, kmax, tol, out=out)
    with Timer(torch) as t:
        for _ in range(steps):
            boys.boys_eval_f64_tol(x, kmax, tol, out=out)
    ms = t.ms / steps
    pn, pk = 1 << 19, 12
    xh, yh, c = workloads.pair_workload(n=pn, kmax=pk)
    px, py = torch.from_numpy(xh).to(dev), torch.from_numpy(yh).to(dev)
    z = torch.empty_like(px)
    boys.boys_pairsum(px, py, c, out=z, tol=tol)
    reps = max(1, min(steps, 3))
    with Timer(torch) as tp:
        for _ in range(reps):
            boys.boys_pairsum(px, py, c, out=z, tol=tol)
    ps = tp.ms / reps / 1e3
    log(f"screening set: write-out {ms:.3f} ms, pair sums {ps:.3f} s")
    return {"tol": tol, "writeout_ms": ms, "writeout_values_per_s": n * (kmax + 1) / (ms * 1e-3),
            "writeout_gbs": n * 8 * (kmax + 2) / (ms * 1e6), "pairsum_seconds": ps,
            "pairsum_pairs_per_s": float(pn) * pn / ps, "_out": out}


def leg_high(torch, boys, workloads, steps, warmup, dev, wo=None):
    """Orders up to 40 (the high-order tables, 5e-14): the headline write-out
    workload at kmax = 40, a 2^26 x 41 FP64 output (22.5 GB per launch)."""
    n, kmax = workloads.N_WRITEOUT, 40
    x = wo["x"] if wo else torch.from_numpy(workloads.gaussian_pair_arguments(n)).to(dev)
    out = torch.empty((n, kmax + 1), dtype=torch.float64, device=dev)
    for _ in range(warmup):
        boys.boys_eval_f64(x, kmax, out=out)
    with Timer(torch) as t:
        for _ in range(steps):
            boys.boys_eval_f64(x, kmax, out=out)
    ms = t.ms / steps
    log(f"high orders: write-out kmax=40 {ms:.3f} ms")
    res = {"kmax": kmax, "writeout_ms": ms, "writeout_values_per_s": n * (kmax + 1) / (ms * 1e-3),
           "writeout_gbs": n * 8 * (kmax + 2) / (ms * 1e6)}
    del out
    torch.cuda.empty_cache()
    return res


def leg_variants(torch, boys, workloads, steps, warmup, dev, wo=None):
    """The variants of the 5e-14 tables (boys_set_tables: the paper's, the
    per-kmax regions, the centre-of-anti-diagonal refit) on the same work:
    the batched consumer on the 8192-batch workload (the configuration
    already chosen), the write-out of the headline arguments at kmax = 4, 12
    and 24, and the pair sums at n = 2^17 for k = 5 (where the centre pick
    changes the degrees of r_{A,5} from (4, 13) to (8, 9)) and k = 12.
    The variants are timed in interleaved rounds (each round times every
    variant once, a few calls each) and each reports the median of its
    rounds: timed one after another, the first variant of a block ran up to
    10% slower or faster than the same kernel later in the run."""
    names = {"paper": boys.TABLES_PAPER, "per_kmax": boys.TABLES_PER_KMAX,
             "centre": boys.TABLES_CENTRE}
    rounds = 5

    def interleaved(call, calls_per_round):
        times = {name: [] for name in names}
        for name, v in names.items():  # warm-up (graphs, workspaces)
            with boys.table_variant(v):
                for _ in range(max(1, warmup)):
                    call()
        for _ in range(rounds):
            for name, v in names.items():
                with boys.table_variant(v):
                    with Timer(torch) as tm:
                        for _ in range(calls_per_round):
                            call()
                times[name].append(tm.ms / calls_per_round)
        return {name: float(np.median(t)) for name, t in times.items()}

    res = {"rounds": rounds}
    bt = workloads.batched_workload()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    args = (t(bt.x), t(bt.batch_off), t(bt.batch_n), t(bt.batch_kmax), t(bt.w), t(bt.w_off))
    out = torch.zeros_like(args[0])
    res["fused_config"] = boys.weighted_sum_config_name(boys.weighted_sum_get_config())
    res["fused_ms"] = interleaved(lambda: boys.boys_weighted_sum(*args, out=out), max(1, steps // 4))
    del args, out
    n = workloads.N_WRITEOUT
    x = wo["x"] if wo else torch.from_numpy(workloads.gaussian_pair_arguments(n)).to(dev)
    res["writeout_ms"] = {}
    for kmax in (4, 12, 24):
        o = torch.empty((n, kmax + 1), dtype=torch.float64, device=dev)
        res["writeout_ms"][f"kmax{kmax}"] = interleaved(lambda: boys.boys_eval_f64(x, kmax, out=o),
                                                        max(1, steps // 4))
        del o
    torch.cuda.empty_cache()
    res["pairsum_ms"] = {}
    for kmax in (5, 12):
        xh, yh, c = workloads.pair_workload(n=1 << 17, kmax=kmax)
        xp, yp = torch.from_numpy(xh).to(dev), torch.from_numpy(yh).to(dev)
        z = torch.empty_like(xp)
        res["pairsum_ms"][f"n2e17_k{kmax}"] = interleaved(lambda: boys.boys_pairsum(xp, yp, c, out=z), 1)
    log(f"variants: fused {res['fused_ms']}; write-out {res['writeout_ms']}; pairs {res['pairsum_ms']}")
    return res


def cpu_model() -> str:
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(torch, wo, fp32, screen=None):
    """The oracle on the first 2^25 write-out arguments (half the workload,
    about 20 thread-seconds of CPU work), all host cores; the GPU rows of the
    same arguments are compared with it on the way."""
    import oracle
    m = 1 << 25
    chunk = 1 << 21
    threads = oracle.max_threads()
    err = 0.0
    err_screen = 0.0
    t_cpu = 0.0
    for s in range(0, m, chunk):
        xs = wo["x_host"][s:s + chunk]
        t0 = time.perf_counter()
        ref = oracle.boys(xs, 32, threads=threads)
        t_cpu += time.perf_counter() - t0
        got = wo["out"][s:s + chunk].cpu().numpy()
        err = max(err, float(np.abs(got - ref).max()))
        if screen is not None:
            got = screen["_out"][s:s + chunk].cpu().numpy()
            err_screen = max(err_screen, float(np.abs(got - ref).max()))
    # The same oracle on one thread, over the first 2^20 of those arguments.
    m1 = 1 << 20
    t0 = time.perf_counter()
    oracle.boys(wo["x_host"][:m1], 32, threads=1)
    t_one = time.perf_counter() - t0
    res = {"value": m * 33 / t_cpu, "unit": "values/s", "cores": threads, "kind": "oracle",
           "sample": f"first 2^25 of the 2^26 write-out arguments, kmax=32, long-double oracle, "
                     f"{threads} threads, {t_cpu:.1f} s wall ({t_cpu * threads:.0f} thread-s)",
           "cpu_model": cpu_model(),
           "value_1_thread": m1 * 33 / t_one,
           "sample_1_thread": f"first 2^20 of the same arguments on one thread, {t_one:.1f} s",
           "gpu_max_abs_err_on_sample": err}
    if screen is not None:
        res["screen_max_abs_err_on_sample"] = err_screen
    if fp32 is not None:
        # FP32 path against the FP64 oracle at the FP32-rounded arguments.
        xs = fp32["_x32"][:1 << 20].cpu().numpy().astype(np.float64)
        ref = oracle.boys(xs, 16, threads=threads)
        got = fp32["_o32"][:1 << 20].cpu().numpy().astype(np.float64)
        row_err = np.abs(got - ref).max(axis=1)
        res["fp32_max_abs_err_on_2^20"] = float(row_err.max())
        from paper_2512_10059_amd.tables import f32_region_bounds
        x0f, x1f = f32_region_bounds()
        regions = {"A'": xs < x0f, "B'": (xs >= x0f) & (xs < x1f), "C'": xs >= x1f}
        res["fp32_max_abs_err_per_region"] = {
            name: float(row_err[m].max()) if m.any() else None for name, m in regions.items()}
    log(f"cpu baseline: {res['value']:.3e} values/s on {threads} threads "
        f"({res['value_1_thread']:.3e} on one); GPU max err {err:.2e}")
    return res


def copy_probe(torch, dev):
    """A plain elementwise copy of known size, for calibrating HBM counters."""
    n = 1 << 29  # 4 GiB in, 4 GiB out per op; torch splits it into two
    a = torch.ones(n, dtype=torch.float64, device=dev)  # launches of 2^28 doubles
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read_per_op": n * 8, "copy_probe_bytes_written_per_op": n * 8,
                      "ops": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--only", default="writeout,mixed,fp32,fused,backward,pairsum,screen,high,variants")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); every argument "
              "is independent, so the path would shard by contiguous slices, but no multi-GPU "
              "run is implemented here.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2512_10059_amd as boys
    from paper_2512_10059_amd import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        copy_probe(torch, dev)
        return
    legs = set(args.only.split(","))
    wo = None
    if "writeout" in legs:
        wo = leg_writeout(torch, boys, workloads, args.steps, args.warmup, dev)
    extra = {}
    fp32 = None
    if "fp32" in legs:
        try:
            fp32 = leg_fp32(torch, boys, workloads, args.steps, args.warmup, dev,
                            wo["x_host"] if wo else None)
            extra["fp32"] = {k: v for k, v in fp32.items() if not k.startswith("_")}
        except Exception as e:  # reported, not hidden
            extra["fp32"] = {"error": str(e)}
    if "mixed" in legs:
        try:
            extra["mixed"] = leg_mixed(torch, boys, workloads, dev)
        except Exception as e:
            extra["mixed"] = {"error": str(e)}
    if "fused" in legs:
        try:
            extra["fused"] = leg_fused(torch, boys, workloads, args.steps, args.warmup, dev)
        except Exception as e:
            extra["fused"] = {"error": str(e)}
    if "backward" in legs:
        try:
            extra["backward"] = leg_backward(torch, boys, workloads, args.steps, args.warmup, dev)
        except Exception as e:
            extra["backward"] = {"error": str(e)}
    if "pairsum" in legs:
        try:
            extra["pairsum"] = leg_pairsum(torch, boys, workloads, args.steps, dev)
        except Exception as e:
            extra["pairsum"] = {"error": str(e)}
    screen = None
    if "screen" in legs:
        try:
            screen = leg_screen(torch, boys, workloads, args.steps, args.warmup, dev, wo)
            extra["screen"] = {k: v for k, v in screen.items() if not k.startswith("_")}
        except Exception as e:
            extra["screen"] = {"error": str(e)}
    if "high" in legs:
        try:
            extra["high"] = leg_high(torch, boys, workloads, args.steps, args.warmup, dev, wo)
        except Exception as e:
            extra["high"] = {"error": str(e)}
    if "variants" in legs:
        try:
            extra["variants"] = leg_variants(torch, boys, workloads, args.steps, args.warmup, dev, wo)
        except Exception as e:
            extra["variants"] = {"error": str(e)}
    if wo is None:  # profiling runs of single legs
        print(json.dumps({"legs": extra}))
        return
    cpu = None if args.no_cpu_baseline else cpu_baseline_leg(torch, wo, fp32, screen)

    ms = wo["ms"]
    achieved = wo["alg_bytes"] / (ms * 1e-3) / 1e9
    traffic = pmc_traffic_bytes()
    line = {
        "metric": METRIC,
        "value": wo["n"] * (wo["kmax"] + 1) / (ms * 1e-3),
        "unit": "values/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "write-out F_0..F_32 of 2^26 Gaussian-pair arguments "
                               "x=ab/(a+b)R^2 (a,b log-uniform [0.05,1e4], R uniform [0,8]), "
                               "row-major 2^26 x 33 FP64",
                   "n": wo["n"], "kmax": wo["kmax"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "eval_f64_kernel<32, boys::PaperTables>",
                     "algorithmic_bytes_per_launch": wo["alg_bytes"]},
        "cpu_baseline": cpu,
        "legs": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
