#!/usr/bin/env python3
"""Generate the FP32-path coefficient header ``boys_coeffs_f32.h`` (offline).

Design of the FP32 variant of Algorithm 1 for orders 0..16 (all numbers are
derived here and written into the header and ``boys_coeffs_f32.json``):

* Region constants from the paper's two equations (Sec. II C) at kmax = 16:
  x0' = (prod_{n<16} (n+1/2))^(1/16) = 6.0139805..., the point from which
  upward recurrence to F_16 does not amplify errors; x1' solves
  Gamma(16.5, x1') / (2 x1'^16.5) = EPS_C, so that the asymptote is within
  EPS_C for every order <= 16 beyond it.  Both are rounded to float32, x0'
  to nearest and x1' upwards (the asymptote error decreases with x).
* A' = [0, x0'): r'_{A,k} from rational Remez with the paper's weight
  rho_{A,k} (so that the downward recurrence keeps every lower order within
  the target), evaluated in FP32 with FP32 coefficients, then FP32 downward
  recurrence.
* B' = [x0', x1'): r'_B for F_0 with weight 1, evaluated in FP64 with FP64
  coefficients, then FP64 upward recurrence (it subtracts nearly equal
  numbers near l ~ x, so it stays in FP64).
* C' = [x1', inf): the asymptote in FP32.
* Degrees: the Walsh-table walk of Sec. II D (first anti-diagonal with an
  entry meeting the target, smallest error on it), where an entry is only
  accepted if its coefficients, rounded to the working precision and run
  through an emulation of the kernel's arithmetic on a dense grid of FP32
  arguments, keep every order within the acceptance bound.

Usage: python gen_coeffs_f32.py [--jobs 8]   (writes next to this file)
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2512_10059_amd import remez  # noqa: E402

KMAX = 16
EPS_A = 5e-7       # Remez target on A' (weighted)
EPS_B = 5e-7       # Remez target on B'
EPS_C = 5e-7       # asymptote error at x1'
ACCEPT = 6.5e-7    # bound on the emulated end-to-end error of A' and B'
LD = np.longdouble
F32 = np.float32


def f32_boundaries():
    x0 = remez.region_x0(KMAX)
    x1 = remez.region_x1(KMAX, EPS_C, 13.0)
    x0f = F32(x0)
    x1f = F32(x1)
    if float(x1f) < x1:
        x1f = np.nextafter(x1f, F32(np.inf))
    return x0, x1, x0f, x1f


def fma32(a, b, c):
    """FP32 fused multiply-add: the FP32 product is exact in FP64."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def emulate_region_a(pf, qf, x, k):
    """Kernel arithmetic of A' in FP32: Horner (FMA), IEEE division, FP32
    exp, downward recurrence F_l = fma(2x, F_{l+1}, e) * (1/(2l+1))."""
    x = x.astype(F32)
    p = np.full(x.shape, pf[-1], dtype=F32)
    for c in pf[-2::-1]:
        p = fma32(p, x, np.full(x.shape, c, dtype=F32))
    q = (x + F32(qf[-2])).astype(F32)
    for c in qf[-3::-1]:
        q = fma32(q, x, np.full(x.shape, c, dtype=F32))
    F = np.empty(x.shape + (k + 1,), dtype=F32)
    F[:, k] = p / q
    e = np.exp(-x).astype(F32)
    two_x = (x + x).astype(F32)
    for l in range(k - 1, -1, -1):
        F[:, l] = (fma32(two_x, F[:, l + 1], e) * F32(1.0 / (2 * l + 1))).astype(F32)
    return F


def grid_f32(lo, hi, size):
    g = np.concatenate([np.linspace(float(lo), float(hi), size),
                        float(lo) + (float(hi) - float(lo)) * np.geomspace(1e-9, 1e-2, 300)])
    g = np.unique(g.astype(F32))
    g = g[(g >= lo) & (g < hi)]
    return np.unique(np.concatenate([g, [np.nextafter(F32(hi), F32(0))], [F32(lo)]]))


def fit_region_a(k, x0f):
    xg = grid_f32(F32(0), x0f, 12000)
    ref = remez.boys_series(xg.astype(LD), k)

    def accept(r):
        pf = np.array([float(c) for c in r.p], dtype=F32)
        qf = np.array([float(c) for c in r.q], dtype=F32)
        F = emulate_region_a(pf, qf, xg, k)
        err = float(np.max(np.abs(F.astype(LD) - ref)))
        return err <= ACCEPT, err

    r = remez.walsh_search(remez.boys_k(k), remez.rho_a(k), 0.0, float(x0f), EPS_A,
                           d_min=2, d_max=16, accept=accept, tol=1e-4, dps=30)
    ok, err = accept(r)
    return {"k": k, "n": r.n, "m": r.m, "E": r.E, "max_err_exact": r.max_err,
            "emulated_fp32_err": err, "nodes": r.nodes,
            "p": [mp.nstr(c, 30) for c in r.p], "q": [mp.nstr(c, 30) for c in r.q],
            "p_f32": [float(F32(float(c))) for c in r.p], "q_f32": [float(F32(float(c))) for c in r.q]}


def emulate_region_b(p, q, x):
    x = x.astype(np.float64)
    pv = np.full(x.shape, p[-1])
    for c in p[-2::-1]:
        pv = pv * x + c
    qv = x + q[-2]
    for c in q[-3::-1]:
        qv = qv * x + c
    F = np.empty(x.shape + (KMAX + 1,))
    F[:, 0] = pv / qv
    e = np.exp(-x)
    inv = 0.5 / x
    for l in range(KMAX):
        F[:, l + 1] = ((2 * l + 1) * F[:, l] - e) * inv
    return F.astype(F32)


def fit_region_b(x0f, x1f):
    xg = grid_f32(x0f, x1f, 12000)
    xg = np.concatenate([xg, [x1f]])  # x1' itself is evaluated in B'
    ref = remez.boys_series(xg.astype(LD), KMAX)

    def accept(r):
        F = emulate_region_b([float(c) for c in r.p], [float(c) for c in r.q], xg)
        err = float(np.max(np.abs(F.astype(LD) - ref)))
        return err <= ACCEPT, err

    r = remez.walsh_search(remez.boys_k(0), remez.rho_one, float(x0f), float(x1f), EPS_B,
                           d_min=2, d_max=14, accept=accept, tol=1e-4, dps=30)
    ok, err = accept(r)
    return {"n": r.n, "m": r.m, "E": r.E, "max_err_exact": r.max_err, "emulated_err": err,
            "nodes": r.nodes, "p": [mp.nstr(c, 30) for c in r.p],
            "q": [mp.nstr(c, 30) for c in r.q], "p_f64": [float(c) for c in r.p],
            "q_f64": [float(c) for c in r.q]}


def hexf(v: float) -> str:
    return float(v).hex() + "f"


def hexd(v: float) -> str:
    return repr(float(v))


def write_outputs(x0, x1, x0f, x1f, ra, rb):
    nmax = max(t["n"] for t in ra)
    mmax = max(t["m"] for t in ra)
    L = []
    w = L.append
    w("/* Generated by gen_coeffs_f32.py: coefficients of the FP32 variant of the")
    w(" * Boys-function method for orders 0..16 (own rational Remez; see the")
    w(" * generator for the design).  Do not edit by hand. */")
    w("#pragma once")
    w("")
    w(f"/* A' = [0, x0'), B' = [x0', x1'), C' = [x1', inf) as float32 values;")
    w(f" * x0' = {x0!r} (stability of upward recurrence to F_16),")
    w(f" * x1' = {x1!r} (asymptote error {EPS_C:g} for F_16), rounded up. */")
    w(f"#define BOYS_F32_KMAX {KMAX}")
    w(f"#define BOYS_F32_X0 {hexf(x0f)}")
    w(f"#define BOYS_F32_X1 {hexf(x1f)}")
    w(f"#define BOYS_F32_EPS_A {EPS_A!r}")
    w(f"#define BOYS_F32_EPS_B {EPS_B!r}")
    w(f"#define BOYS_F32_EPS_C {EPS_C!r}")
    w("")
    w(f"/* r'_B: F_0 on [x0', x1'], FP64, degrees ({rb['n']},{rb['m']}), minimax error {rb['E']:.3e}. */")
    w(f"#define BOYS_F32_RB_N {rb['n']}")
    w(f"#define BOYS_F32_RB_M {rb['m']}")
    w("#define BOYS_F32_RB_P_INIT { " + ", ".join(hexd(v) for v in rb["p_f64"]) + " }")
    w("#define BOYS_F32_RB_Q_INIT { " + ", ".join(hexd(v) for v in rb["q_f64"]) + " }")
    w("")
    w(f"/* r'_{{A,k}}: F_k on [0, x0'], FP32, k = 0..{KMAX}; padded with zeros to")
    w(f" * degrees ({nmax},{mmax}). */")
    w(f"#define BOYS_F32_RA_NMAX {nmax}")
    w(f"#define BOYS_F32_RA_MMAX {mmax}")
    w("#define BOYS_F32_RA_DEG_N_INIT { " + ", ".join(str(t["n"]) for t in ra) + " }")
    w("#define BOYS_F32_RA_DEG_M_INIT { " + ", ".join(str(t["m"]) for t in ra) + " }")
    w("#define BOYS_F32_RA_P_INIT { \\")
    for t in ra:
        v = t["p_f32"] + [0.0] * (nmax + 1 - len(t["p_f32"]))
        w(f"  /* k={t['k']:2d} ({t['n']},{t['m']}) E={t['E']:.2e} */ {{ " + ", ".join(hexf(c) for c in v)
          + " }" + ("," if t["k"] < KMAX else "") + " \\")
    w("}")
    w("#define BOYS_F32_RA_Q_INIT { \\")
    for t in ra:
        v = t["q_f32"] + [0.0] * (mmax + 1 - len(t["q_f32"]))
        w(f"  /* k={t['k']:2d} */ {{ " + ", ".join(hexf(c) for c in v) + " }"
          + ("," if t["k"] < KMAX else "") + " \\")
    w("}")
    with open(os.path.join(HERE, "boys_coeffs_f32.h"), "w") as f:
        f.write("\n".join(L) + "\n")
    rec = {"kmax": KMAX, "eps_a": EPS_A, "eps_b": EPS_B, "eps_c": EPS_C, "accept": ACCEPT,
           "x0": x0, "x1": x1, "x0_f32": float(x0f), "x1_f32": float(x1f),
           "region_a": ra, "region_b": rb}
    with open(os.path.join(HERE, "boys_coeffs_f32.json"), "w") as f:
        json.dump(rec, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    x0, x1, x0f, x1f = f32_boundaries()
    print(f"x0' = {x0!r} -> {float(x0f)!r}; x1' = {x1!r} -> {float(x1f)!r}", flush=True)
    with cf.ProcessPoolExecutor(max_workers=args.jobs) as ex:
        fut_b = ex.submit(fit_region_b, x0f, x1f)
        futs = [ex.submit(fit_region_a, k, x0f) for k in range(KMAX + 1)]
        ra = [f.result() for f in futs]
        rb = fut_b.result()
    for t in ra:
        print(f"r'_A,{t['k']:2d}: ({t['n']},{t['m']}) E={t['E']:.3e} emulated FP32 err={t['emulated_fp32_err']:.3e}")
    print(f"r'_B: ({rb['n']},{rb['m']}) E={rb['E']:.3e} emulated err={rb['emulated_err']:.3e}")
    write_outputs(x0, x1, x0f, x1f, ra, rb)


if __name__ == "__main__":
    main()
