#!/usr/bin/env python3
"""Re-run the paper's degree choice for its FP64 tables with our Remez (offline).

For r_B (F_0 on [x0, x1], weight 1) and every r_{A,k} (F_k on [0, x0],
weight rho_{A,k}), walk the Walsh table's anti-diagonals n + m = d (Sec. II D)
from one below the printed table's n + m, with target eps_tol = 5e-14, and
report the first feasible anti-diagonal and the entry of smallest error on
it.  The "centre" column is the alternative the paper mentions: the feasible
entry nearest the centre of that anti-diagonal (n close to m, more
instruction-level parallelism between numerator and denominator).

Usage: python walsh_fp64.py [--jobs 8] [--k 0,8,26]   (prints a Markdown table)
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2512_10059_amd import remez  # noqa: E402

EPS_TOL = 5e-14


def printed_degrees():
    import re
    text = open(os.path.join(HERE, "boys_coeffs_f64.h")).read().replace("\\\n", " ")
    get = lambda name: [int(v) for v in re.findall(r"-?\d+", re.search(
        r"#define " + name + r"\s+(.*)", text).group(1))]
    x0 = float(re.search(r"#define BOYS_F64_X0\s+(\S+)", text).group(1))
    x1 = float(re.search(r"#define BOYS_F64_X1\s+(\S+)", text).group(1))
    nb = int(re.search(r"#define BOYS_RB_N\s+(\d+)", text).group(1))
    mb = int(re.search(r"#define BOYS_RB_M\s+(\d+)", text).group(1))
    return x0, x1, list(zip(get("BOYS_RA_DEG_N_INIT"), get("BOYS_RA_DEG_M_INIT"))), (nb, mb)


def entry(args):
    which, k, n, m, a, b = args
    f = remez.boys_k(0 if which == "B" else k)
    rho = remez.rho_one if which == "B" else remez.rho_a(k)
    try:
        r = remez.remez(f, rho, a, b, n, m, tol=1e-3, target=EPS_TOL, dps=40, max_iter=30)
        return (which, k, n, m, r.E if r.max_err <= EPS_TOL * (1 + 1e-3) else None)
    except remez.RemezFailure:
        return (which, k, n, m, None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--k", default="all")
    args = ap.parse_args()
    x0, x1, ra, rb = printed_degrees()
    ks = list(range(33)) if args.k == "all" else [int(v) for v in args.k.split(",")]
    tables = [("B", 0, rb, x0, x1)] + [("A", k, ra[k], 0.0, x0) for k in ks]
    jobs = []
    for which, k, (n, m), a, b in tables:
        for d in (n + m - 1, n + m):
            jobs += [(which, k, d - mm, mm, a, b) for mm in range(d + 1)]
    with cf.ProcessPoolExecutor(args.jobs) as ex:
        res = list(ex.map(entry, jobs, chunksize=1))
    print("| table | printed (n,m) | first feasible n+m | smallest-error entry | its error | centre entry | feasible entries |")
    print("|---|---|---|---|---|---|---|")
    for which, k, (n, m), a, b in tables:
        name = "r_B" if which == "B" else f"r_A,{k}"
        mine = [r for r in res if r[0] == which and r[1] == k and r[4] is not None]
        first = min((r[2] + r[3] for r in mine), default=None)
        if first is None:
            print(f"| {name} | ({n},{m}) | none up to {n + m} | | | | |")
            continue
        on = [r for r in mine if r[2] + r[3] == first]
        best = min(on, key=lambda r: r[4])
        centre = min(on, key=lambda r: abs(r[2] - r[3]))
        feas = ", ".join(f"({r[2]},{r[3]})" for r in sorted(on, key=lambda r: r[3]))
        print(f"| {name} | ({n},{m}) | {first} | ({best[2]},{best[3]}) | {best[4]:.3e} | "
              f"({centre[2]},{centre[3]}) | {feas} |")


if __name__ == "__main__":
    main()
