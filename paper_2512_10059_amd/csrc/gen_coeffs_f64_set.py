#!/usr/bin/env python3
"""Generate an FP64 table set of the method for a given eps_tol and kmax
(offline; the outputs are committed):

    python gen_coeffs_f64_set.py --name screen --eps 1e-10 --kmax 32
        -> boys_coeffs_f64_screen.h/.json   ("screening" accuracy)
    python gen_coeffs_f64_set.py --name high --eps 5e-14 --kmax 40 --target 4.9e-14
        -> boys_coeffs_f64_high.h/.json     (orders up to 40 at the paper's accuracy)

The construction is the paper's, re-run (Sec. II C-D):

* x0 = (prod_{n<kmax} (n+1/2))^(1/kmax), from which the upward recurrence to
  F_kmax does not amplify errors.  For kmax = 32 it is the paper's printed
  x0 = 11.899848152108484 (kept verbatim); otherwise the double nearest the
  product formula.
* x1 solves Gamma(kmax + 1/2, x1) / (2 x1^(kmax + 1/2)) = eps (the asymptote's
  error for F_kmax, which bounds it for every lower order); the root is
  rounded up to a double, so C = (x1, inf) is within eps at every double
  beyond it.
* r_B approximates F_0 on [x0, x1] with weight 1; r_{A,k}, k = 0..kmax,
  approximates F_k on [0, x0] with the weight rho_{A,k} of Sec. II C, so that
  the downward recurrence keeps every lower order within the target.
* The record (.json) keeps every fit's extended-precision coefficients (30
  digits) beside the doubles, so the fit itself can be checked.
* Degrees: the Walsh-table walk of Sec. II D from n + m = d_min upwards
  (first anti-diagonal with an entry meeting the target, smallest error on
  it), where an entry counts only if its coefficients rounded to double still
  meet the target on a dense grid (evaluated in long double).  The target is
  eps, or a smaller --target that leaves room for the FP64 evaluation's own
  rounding (needed at 5e-14, where the paper's tables reach 4.95e-14).
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

PAPER_X0 = 11.899848152108484  # the paper's printed x0 (kmax = 32)
LD = np.longdouble


def region_x0(kmax: int) -> float:
    """The double nearest (prod_{n<kmax} (n+1/2))^(1/kmax); the paper's
    printed value for kmax = 32."""
    if kmax == 32:
        return PAPER_X0
    mp.mp.dps = 50
    v = mp.exp((mp.loggamma(kmax + mp.mpf(1) / 2) - mp.loggamma(mp.mpf(1) / 2)) / kmax)
    with mp.workprec(53):
        return float(+v)


def region_x1(eps: float, kmax: int) -> float:
    """Root of Gamma(kmax+1/2, x)/(2 x^(kmax+1/2)) = eps, rounded up to a
    double (solved on the logarithm, where Newton's method converges from a
    rough start)."""
    mp.mp.dps = 50
    s = kmax + mp.mpf(1) / 2
    g = lambda x: mp.log(mp.gammainc(s, x) / (2 * x ** s)) - mp.log(eps)
    root = mp.findroot(g, 20.0 + kmax / 4)
    x1 = float(root)
    if mp.mpf(x1) < root:
        x1 = float(np.nextafter(x1, np.inf))
    return x1


def double_error(f, rho, a, b, p, q):
    """max rho |f - p/q| with p, q rounded to double, evaluated in long
    double on a dense grid of [a, b]."""
    x = np.linspace(LD(a), LD(b), 20001, dtype=LD)
    pd = [LD(float(c)) for c in p]
    qd = [LD(float(c)) for c in q]
    pv = np.zeros_like(x)
    for c in reversed(pd):
        pv = pv * x + c
    qv = np.zeros_like(x)
    for c in reversed(qd):
        qv = qv * x + c
    return float(np.max(rho(x) * np.abs(f(x) - pv / qv)))


def fit(job):
    which, k, a, b, target, d_min = job
    f = remez.boys_k(0 if which == "B" else k)
    rho = remez.rho_one if which == "B" else remez.rho_a(k)

    def accept(r):
        e = double_error(f, rho, a, b, r.p, r.q)
        return e <= target, e

    r = remez.walsh_search(f, rho, a, b, target, d_min=d_min, d_max=26, accept=accept,
                           tol=1e-3, dps=40, max_iter=30)
    return dict(which=which, k=k, n=r.n, m=r.m, a=a, b=b, E=float(abs(r.E)),
                max_err=float(r.max_err), double_err=double_error(f, rho, a, b, r.p, r.q),
                p=[float(c) for c in r.p], q=[float(c) for c in r.q],
                p_ext=[mp.nstr(c, 30) for c in r.p], q_ext=[mp.nstr(c, 30) for c in r.q])


def hexd(v: float) -> str:
    return float(v).hex()


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", default="screen")
    ap.add_argument("--eps", type=float, default=1e-10)
    ap.add_argument("--kmax", type=int, default=32)
    ap.add_argument("--target", type=float, default=None)
    ap.add_argument("--d-min", type=int, default=2)
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    eps, kmax = args.eps, args.kmax
    target = args.target if args.target is not None else eps
    prefix = "BOYS_" + {"screen": "SCR", "high": "HIGH"}.get(args.name, args.name.upper())
    x0 = region_x0(kmax)
    x1 = region_x1(eps, kmax)
    jobs = [("B", 0, x0, x1, target, args.d_min)] + [("A", k, 0.0, x0, target, args.d_min)
                                                      for k in range(kmax + 1)]
    with cf.ProcessPoolExecutor(max_workers=args.jobs) as ex:
        res = list(ex.map(fit, jobs))
    rb = res[0]
    ra = sorted(res[1:], key=lambda t: t["k"])
    nmax = max(t["n"] for t in ra)
    mmax = max(t["m"] for t in ra)
    lines = [
        f"/* Generated by gen_coeffs_f64_set.py --name {args.name} -- do not edit.",
        f" * FP64 tables for eps_tol = {eps!r}, kmax = {kmax}, computed with the Remez tool",
        " * (weighted rational minimax, Walsh-table degree choice).  Hex-float literals",
        " * are the exact doubles; coefficients run from degree 0 upwards and the",
        " * denominators are monic. */",
        "#pragma once",
        f"#define {prefix}_EPS {eps!r}",
        f"#define {prefix}_KMAX {kmax}",
        f"#define {prefix}_X0 {hexd(x0)} /* {x0!r} */",
        f"#define {prefix}_X1 {hexd(x1)} /* {x1!r} */",
        f"#define {prefix}_RB_N {rb['n']}",
        f"#define {prefix}_RB_M {rb['m']}",
        f"#define {prefix}_RB_P_INIT {{ " + ", ".join(hexd(c) for c in rb["p"]) + " }",
        f"#define {prefix}_RB_Q_INIT {{ " + ", ".join(hexd(c) for c in rb["q"]) + " }",
        f"#define {prefix}_RA_NMAX {nmax}",
        f"#define {prefix}_RA_MMAX {mmax}",
        f"#define {prefix}_RA_DEG_N_INIT {{ " + ", ".join(str(t["n"]) for t in ra) + " }",
        f"#define {prefix}_RA_DEG_M_INIT {{ " + ", ".join(str(t["m"]) for t in ra) + " }",
        f"#define {prefix}_RA_P_INIT {{ \\",
    ]
    for t in ra:
        row = [hexd(c) for c in t["p"]] + ["0x0p+0"] * (nmax - t["n"])
        lines.append(f"  /* k={t['k']:2d} ({t['n']},{t['m']}) E={t['double_err']:.2e} */ {{ "
                     + ", ".join(row) + " }" + ("," if t["k"] < kmax else "") + " \\")
    lines.append("}")
    lines.append(f"#define {prefix}_RA_Q_INIT {{ \\")
    for t in ra:
        row = [hexd(c) for c in t["q"]] + ["0x0p+0"] * (mmax - t["m"])
        lines.append(f"  /* k={t['k']:2d} */ {{ " + ", ".join(row) + " }"
                     + ("," if t["k"] < kmax else "") + " \\")
    lines.append("}")
    stem = os.path.join(HERE, f"boys_coeffs_f64_{args.name}")
    with open(stem + ".h", "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(stem + ".json", "w") as fh:
        json.dump(dict(eps=eps, target=target, kmax=kmax, x0=x0, x1=x1, rb=rb, ra=ra), fh, indent=1)
    print(f"x0 = {x0!r}; x1 = {x1!r}; r_B ({rb['n']},{rb['m']}) err {rb['double_err']:.3e}")
    for t in ra:
        print(f"r_A,{t['k']}: ({t['n']},{t['m']}) err {t['double_err']:.3e}")


if __name__ == "__main__":
    main()
