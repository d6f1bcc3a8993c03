#!/usr/bin/env python3
"""Generate two more FP64 table sets at the paper's eps_tol = 5e-14 with the
library's Remez tool (offline; the outputs are committed):

    python gen_coeffs_f64_perk.py --what perk
        -> boys_coeffs_f64_perk.h/.json     (regions of each kmax < 32)
    python gen_coeffs_f64_perk.py --what centre
        -> boys_coeffs_f64_centre.h/.json   (the paper's regions, centre picks)

Per-kmax regions (Sec. II C).  x0 and x1 depend on the highest order that a
call evaluates: x0 = max{1, (prod_{n<kmax} (n+1/2))^(1/kmax)} (the upward
recurrence to F_kmax does not amplify errors from there on) and x1 solves
Gamma(kmax+1/2, x1) / (2 x1^(kmax+1/2)) = eps_tol.  The paper prints one set
for kmax = 32; a call that stops at a lower order can use the smaller x0 and
x1 of its own kmax.  For each K = 0..31 this fits
    r_B^(K):    F_0 on [x0(K), x1(K)], weight 1,
    r_{A,K}^(K): F_K on [0, x0(K)], weight rho_{A,K},
which is all that an evaluation of F_0..F_K needs (r_{A,K} seeds the
downward recurrence; no other row of region A is used).  x0(K) is the double
nearest the product formula (1 for K <= 2).  x1(K) is the root of the
equation at the fitting target 4.9e-14 instead of eps_tol, rounded up to a
double: at low K the asymptote's F_K is large enough (about 1e-4 near x = 27
for K = 2) that the few roundings of its FP64 evaluation, added to a
truncation error of exactly eps_tol at the root, would exceed eps_tol by
about 1e-20 just beyond x1; the 1e-15 left covers them, as it does for the
fits.  Row 32 is the paper's own set and is not generated here.

Centre of the anti-diagonal (Sec. II D).  The paper picks, on the first
anti-diagonal n + m = d of the Walsh table with an entry that meets the
target, the entry of smallest error, and names an alternative: the feasible
entry nearest the centre of that anti-diagonal, where n and m are close, so
that numerator and denominator evaluate with more overlap.  The centre set
refits r_B and every r_{A,k}, k = 0..32, on the paper's x0 and x1 with that
choice (ties by smaller error).

An entry counts as feasible only if its coefficients rounded to double still
meet the fitting target on a dense grid, evaluated in long double; the
target is 4.9e-14, leaving room for the evaluation's own rounding in FP64.
The walk is level-synchronous: every table still searching submits all
entries of its current anti-diagonal to the process pool, so the pool stays
busy across tables.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys

import mpmath as mp

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

from paper_2512_10059_amd import remez  # noqa: E402
import gen_coeffs_f64_set as gen_set  # noqa: E402

EPS = 5e-14
TARGET = 4.9e-14
PAPER_X0 = 11.899848152108484
PAPER_X1 = 28.98933773882074
PERK_KMAX = 31


def perk_x0(K: int) -> float:
    """max{1, (prod_{n<K} (n+1/2))^(1/K)} as the nearest double."""
    if K <= 2:  # the product's K-th root is below 1 up to K = 2 (0.5, 0.866)
        return 1.0
    return gen_set.region_x0(K)


def entry(job):
    """One Walsh-table entry: Remez fit, then the double-rounding check."""
    key, which, k, a, b, n, m = job
    f = remez.boys_k(0 if which == "B" else k)
    rho = remez.rho_one if which == "B" else remez.rho_a(k)
    try:
        r = remez.remez(f, rho, a, b, n, m, tol=1e-3, target=TARGET, dps=40, max_iter=30)
    except remez.RemezFailure:
        return key, n, m, None
    if r.max_err > TARGET:
        return key, n, m, None
    derr = gen_set.double_error(f, rho, a, b, r.p, r.q)
    if derr > TARGET:
        return key, n, m, None
    return key, n, m, dict(which=which, k=k, n=n, m=m, a=a, b=b, E=float(abs(r.E)),
                           max_err=float(r.max_err), double_err=derr,
                           p=[float(c) for c in r.p], q=[float(c) for c in r.q],
                           p_ext=[mp.nstr(c, 30) for c in r.p], q_ext=[mp.nstr(c, 30) for c in r.q])


def walk(tables, pick, jobs, d_start):
    """tables: key -> (which, k, a, b).  Returns key -> chosen entry, with the
    feasible degrees of its anti-diagonal under 'feasible'."""
    d_start = dict(d_start)
    d = dict(d_start)
    done = {}
    with cf.ProcessPoolExecutor(max_workers=jobs) as ex:
        while len(done) < len(tables):
            batch = []
            for key, (which, k, a, b) in tables.items():
                if key in done:
                    continue
                batch += [(key, which, k, a, b, d[key] - m, m) for m in range(d[key] + 1)]
            found = {}
            for key, n, m, res in ex.map(entry, batch, chunksize=1):
                if res is not None:
                    found.setdefault(key, []).append(res)
            for key in tables:
                if key in done:
                    continue
                if key in found and d[key] == d_start[key] and d[key] > 1:
                    # Feasible at the starting anti-diagonal: it need not be
                    # the first; start lower.
                    d[key] = d_start[key] = max(1, d[key] - 3)
                elif key in found:
                    on = found[key]
                    best = pick(on)
                    best["feasible"] = sorted([e["n"], e["m"]] for e in on)
                    done[key] = best
                    print(f"{key}: d={d[key]} -> ({best['n']},{best['m']}) err {best['double_err']:.3e}",
                          flush=True)
                else:
                    d[key] += 1
                    if d[key] > 32:
                        raise RuntimeError(f"{key}: no entry up to n + m = 32")
    return done


def smallest_error(on):
    return min(on, key=lambda e: e["double_err"])


def centre(on):
    return min(on, key=lambda e: (abs(e["n"] - e["m"]), e["double_err"]))


def hexd(v: float) -> str:
    return float(v).hex()


def rows_init(name, rows, width, attr):
    lines = [f"#define {name} {{ \\"]
    for i, t in enumerate(rows):
        vals = [hexd(c) for c in t[attr]] + ["0x0p+0"] * (width + 1 - len(t[attr]))
        tail = "," if i < len(rows) - 1 else ""
        lines.append(f"  /* {t['key']} ({t['n']},{t['m']}) E={t['double_err']:.2e} */ {{ "
                     + ", ".join(vals) + " }" + tail + " \\")
    lines.append("}")
    return lines


def ints_init(name, vals):
    return f"#define {name} {{ " + ", ".join(str(v) for v in vals) + " }"


def paper_row32():
    """Row 32 of the per-kmax set: the paper's own x0, x1, r_B and r_{A,32},
    read from the appendix header."""
    import re
    text = open(os.path.join(HERE, "boys_coeffs_f64.h")).read().replace("\\\n", " ")
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    d = dict(re.findall(r"^#define\s+(\w+)\s+(.*)$", text, re.M))
    vec = lambda v: [float.fromhex(c.strip()) if "0x" in c else float(c) for c in v.strip()[1:-1].split(",")]
    rows = lambda v: [vec("{" + r + "}") for r in re.findall(r"\{([^{}]*)\}", v.strip()[1:-1])]
    n32 = int(vec(d["BOYS_RA_DEG_N_INIT"])[32])
    m32 = int(vec(d["BOYS_RA_DEG_M_INIT"])[32])
    x0, x1 = float(d["BOYS_F64_X0"]), float(d["BOYS_F64_X1"])
    rb = dict(n=int(d["BOYS_RB_N"]), m=int(d["BOYS_RB_M"]), p=vec(d["BOYS_RB_P_INIT"]),
              q=vec(d["BOYS_RB_Q_INIT"]), key="K=32 r_B (paper)", double_err=float("nan"))
    ra = dict(n=n32, m=m32, p=rows(d["BOYS_RA_P_INIT"])[32][:n32 + 1],
              q=rows(d["BOYS_RA_Q_INIT"])[32][:m32 + 1], key="K=32 r_A (paper)", double_err=float("nan"))
    return x0, x1, rb, ra


def rows_init_any(name, rows, width, attr):
    lines = [f"#define {name} {{ \\"]
    for i, t in enumerate(rows):
        vals = [hexd(c) for c in t[attr]] + ["0x0p+0"] * (width + 1 - len(t[attr]))
        tail = "," if i < len(rows) - 1 else ""
        err = "" if t["double_err"] != t["double_err"] else f" E={t['double_err']:.2e}"
        lines.append(f"  /* {t['key']} ({t['n']},{t['m']}){err} */ {{ "
                     + ", ".join(vals) + " }" + tail + " \\")
    lines.append("}")
    return lines


def emit_perk(record):
    """Header of the per-kmax set: rows K = 0..31 from the fits, row 32 the
    paper's set."""
    x0p, x1p, rbp, rap = paper_row32()
    x0s = record["x0"] + [x0p]
    x1s = record["x1"] + [x1p]
    rb = [dict(t, key=f"K={K:2d} r_B") for K, t in enumerate(record["rb"])] + [rbp]
    ra = [dict(t, key=f"K={t['k']:2d} r_A") for t in record["ra"]] + [rap]
    P = "BOYS_PK"
    nb, mb = max(t["n"] for t in rb), max(t["m"] for t in rb)
    na, ma = max(t["n"] for t in ra), max(t["m"] for t in ra)
    return [
        "/* Generated by gen_coeffs_f64_perk.py --what perk -- do not edit.",
        " * FP64 tables for eps_tol = 5e-14 with the regions of each kmax = 0..32",
        " * (row K: x0(K), x1(K), r_B on [x0(K), x1(K)] and r_{A,K} on [0, x0(K)];",
        " * x1(K) solves the asymptote-error equation at 4.9e-14, leaving room for",
        " * the FP64 evaluation's rounding),",
        " * rows 0..31 computed with the Remez tool and the Walsh-table degree choice",
        " * (first feasible anti-diagonal, smallest error), row 32 the paper's",
        " * appendix.  Hex-float literals are the exact doubles; coefficients run",
        " * from degree 0 upwards, denominators monic, rows padded with zeros. */",
        "#pragma once",
        f"#define {P}_EPS 5e-14",
        f"#define {P}_KMAX 32",
        f"#define {P}_X0_INIT {{ " + ", ".join(hexd(v) for v in x0s) + " }",
        f"#define {P}_X1_INIT {{ " + ", ".join(hexd(v) for v in x1s) + " }",
        f"#define {P}_RB_NMAX {nb}",
        f"#define {P}_RB_MMAX {mb}",
        ints_init(f"{P}_RB_N_INIT", [t["n"] for t in rb]),
        ints_init(f"{P}_RB_M_INIT", [t["m"] for t in rb]),
        *rows_init_any(f"{P}_RB_P_INIT", rb, nb, "p"),
        *rows_init_any(f"{P}_RB_Q_INIT", rb, mb, "q"),
        f"#define {P}_RA_NMAX {na}",
        f"#define {P}_RA_MMAX {ma}",
        ints_init(f"{P}_RA_N_INIT", [t["n"] for t in ra]),
        ints_init(f"{P}_RA_M_INIT", [t["m"] for t in ra]),
        *rows_init_any(f"{P}_RA_P_INIT", ra, na, "p"),
        *rows_init_any(f"{P}_RA_Q_INIT", ra, ma, "q"),
    ]


def emit_centre(record):
    rb = dict(record["rb"], key="r_B")
    ra = [dict(t, key=f"k={t['k']:2d}") for t in record["ra"]]
    P = "BOYS_CTR"
    na, ma = max(t["n"] for t in ra), max(t["m"] for t in ra)
    return [
        "/* Generated by gen_coeffs_f64_perk.py --what centre -- do not edit.",
        " * FP64 tables for eps_tol = 5e-14, kmax = 32 on the paper's x0 and x1, with",
        " * the Walsh-table entry nearest the centre of the first feasible",
        " * anti-diagonal (n close to m), computed with the Remez tool.  Hex-float",
        " * literals are the exact doubles; coefficients run from degree 0 upwards",
        " * and the denominators are monic. */",
        "#pragma once",
        f"#define {P}_EPS 5e-14",
        f"#define {P}_KMAX 32",
        f"#define {P}_X0 {hexd(PAPER_X0)} /* {PAPER_X0!r} */",
        f"#define {P}_X1 {hexd(PAPER_X1)} /* {PAPER_X1!r} */",
        f"#define {P}_RB_N {rb['n']}",
        f"#define {P}_RB_M {rb['m']}",
        f"#define {P}_RB_P_INIT {{ " + ", ".join(hexd(c) for c in rb["p"]) + " }",
        f"#define {P}_RB_Q_INIT {{ " + ", ".join(hexd(c) for c in rb["q"]) + " }",
        f"#define {P}_RA_NMAX {na}",
        f"#define {P}_RA_MMAX {ma}",
        ints_init(f"{P}_RA_DEG_N_INIT", [t["n"] for t in ra]),
        ints_init(f"{P}_RA_DEG_M_INIT", [t["m"] for t in ra]),
        *rows_init_any(f"{P}_RA_P_INIT", ra, na, "p"),
        *rows_init_any(f"{P}_RA_Q_INIT", ra, ma, "q"),
    ]


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--what", choices=["perk", "centre"], required=True)
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--emit-only", action="store_true",
                    help="rewrite the header from the committed record without refitting")
    args = ap.parse_args()
    stem = os.path.join(HERE, f"boys_coeffs_f64_{args.what}")
    if args.emit_only:
        record = json.load(open(stem + ".json"))
    elif args.what == "perk":
        tables, d0 = {}, {}
        x0s, x1s = [], []
        for K in range(PERK_KMAX + 1):
            x0, x1 = perk_x0(K), gen_set.region_x1(TARGET, K)
            x0s.append(x0)
            x1s.append(x1)
            tables[f"B{K}"] = ("B", 0, x0, x1)
            tables[f"A{K}"] = ("A", K, 0.0, x0)
            d0[f"B{K}"], d0[f"A{K}"] = 10, (4 if K < 8 else 9)
        res = walk(tables, smallest_error, args.jobs, d0)
        rb = [res[f"B{K}"] for K in range(PERK_KMAX + 1)]
        ra = [res[f"A{K}"] for K in range(PERK_KMAX + 1)]
        record = dict(eps=EPS, target=TARGET, kmax=PERK_KMAX, x0=x0s, x1=x1s, rb=rb, ra=ra)
    else:
        tables = {"B": ("B", 0, PAPER_X0, PAPER_X1)}
        d0 = {"B": 8}
        for k in range(33):
            tables[f"A{k}"] = ("A", k, 0.0, PAPER_X0)
            d0[f"A{k}"] = 8
        res = walk(tables, centre, args.jobs, d0)
        record = dict(eps=EPS, target=TARGET, kmax=32, x0=PAPER_X0, x1=PAPER_X1, rb=res["B"],
                      ra=[res[f"A{k}"] for k in range(33)])
    if not args.emit_only:
        with open(stem + ".json", "w") as fh:
            json.dump(record, fh, indent=1)
    lines = emit_perk(record) if args.what == "perk" else emit_centre(record)
    with open(stem + ".h", "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
