#!/usr/bin/env python3
"""One approximant for F_0 on all of [x0, inf) (offline experiment).

The paper mentions rational minimax approximation on an infinite interval
(its appendix proves that one exists when n <= m) as a way to drop the
asymptotic region and the branch between B and C, and reports that the
attempt failed: the degrees it needed made the fit numerically unstable
(Sec. II A).  A rational in x must follow F_0 ~ (sqrt(pi)/2) x^(-1/2), which
no rational in x does.  This script takes that factor out and changes the
variable:

    s = x0 / x in (0, 1],   F_0(x) = sqrt(s / x0) g(s),
    g(s) = sqrt(x) F_0(x) = (sqrt(pi)/2) erf(sqrt(x0 / s)),

so g is smooth on [0, 1] and tends to sqrt(pi)/2 as s -> 0 with a correction
that is exponentially small there.  An absolute error eps on F_0 is a
weighted error on g with weight rho(s) = sqrt(s / x0).  The Walsh-table walk
of Sec. II D (first feasible anti-diagonal, smallest error; feasible = the
coefficients rounded to double still meet the target on a dense grid,
evaluated in long double) runs from n + m = 2 upwards with the library's
Remez tool, and the script prints every entry it tried.

The first feasible entry's fit is written to single_region_fp64.json (its
coefficients as doubles and to 30 digits), which tests/test_single_region.py
checks against the oracle.

Usage: python single_region_fp64.py [--target 4.9e-14] [--x0 11.899848152108484]
       [--d-min 2] [--d-max 24] [--jobs 8]
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

LD = np.longdouble
X0 = 11.899848152108484


def g_of_s(x0):
    def g(s):
        s = np.atleast_1d(np.asarray(s, dtype=LD))
        out = np.empty(s.shape, dtype=LD)
        with mp.workdps(40):
            half_sqrt_pi = mp.sqrt(mp.pi) / 2
            for i, v in enumerate(s.flat):
                v = remez._ld_to_mp(v)
                out.flat[i] = remez._to_ld(half_sqrt_pi if v == 0 else half_sqrt_pi * mp.erf(mp.sqrt(x0 / v)))
        return out
    return g


def rho_of_s(x0):
    def rho(s):
        s = np.atleast_1d(np.asarray(s, dtype=LD))
        # sqrt(s / x0), kept away from 0 so that the weight stays positive
        return np.sqrt(np.maximum(s, LD(1e-30)) / LD(x0))
    return rho


def double_error(g, rho, p, q, npts=20001):
    s = np.linspace(LD(0), LD(1), npts, dtype=LD)
    pv = remez.polyval_ld([LD(float(c)) for c in p], s)
    qv = remez.polyval_ld([LD(float(c)) for c in q], s)
    return float(np.max(rho(s) * np.abs(g(s) - pv / qv)))


def entry(job):
    """Remez fit of one Walsh-table entry and its error with double
    coefficients; the fit record travels along for the winner."""
    n, m, x0, target = job
    g, rho = g_of_s(x0), rho_of_s(x0)
    try:
        r = remez.remez(g, rho, 0.0, 1.0, n, m, tol=1e-3, target=target, dps=40, max_iter=40,
                        grid_size=4000)
    except remez.RemezFailure as e:
        return n, m, None, None, str(e)[:60], None
    fit = dict(n=n, m=m, x0=x0, target=target, E=float(r.E), max_err=float(r.max_err),
               p=[float(c) for c in r.p], q=[float(c) for c in r.q],
               p_ext=[mp.nstr(c, 30) for c in r.p], q_ext=[mp.nstr(c, 30) for c in r.q])
    return n, m, r.max_err, double_error(g, rho, r.p, r.q), "converged" if r.converged else "not converged", fit


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--target", type=float, default=4.9e-14)
    ap.add_argument("--x0", type=float, default=X0)
    ap.add_argument("--d-min", type=int, default=2)
    ap.add_argument("--d-max", type=int, default=24)
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    with cf.ProcessPoolExecutor(args.jobs) as ex:
        for d in range(args.d_min, args.d_max + 1):
            jobs = [(d - m, m, args.x0, args.target) for m in range(d + 1)]
            res = list(ex.map(entry, jobs, chunksize=1))
            ok = [r for r in res if r[3] is not None and r[3] <= args.target]
            for n, m, e, de, note, *_ in res:
                es = "-" if e is None else f"{e:.3e}"
                ds = "-" if de is None else f"{de:.3e}"
                print(f"d={d:2d} ({n:2d},{m:2d}) fit {es} with double coefficients {ds} {note}", flush=True)
            if ok:
                best = min(ok, key=lambda r: r[3])
                print(f"first feasible anti-diagonal n+m = {d}: ({best[0]},{best[1]}) {best[3]:.3e}")
                fit = dict(best[5], double_err=best[3],
                           feasible=[[r[0], r[1]] for r in ok], anti_diagonal=d)
                with open(os.path.join(HERE, "single_region_fp64.json"), "w") as fh:
                    json.dump(fit, fh, indent=1)
                return
    print(f"no entry up to n+m = {args.d_max} meets {args.target:g}")


if __name__ == "__main__":
    main()
