"""The two table sets of csrc/gen_coeffs_f64_perk.py, pinned against the
long-double oracle, mpmath and the paper's definitions (Sec. II C-D):

* "perk": the regions of each kmax K = 0..31 at eps_tol = 5e-14 (x0(K),
  x1(K), r_B on [x0(K), x1(K)], r_{A,K} on [0, x0(K)]); row 32 is the
  paper's appendix set;
* "centre": the paper's x0 and x1 with r_B and every r_{A,k} refitted at the
  Walsh-table entry nearest the centre of the first feasible anti-diagonal.

For the per-kmax set:
* x0(K) = max{1, (prod_{n<K} (n+1/2))^(1/K)}, checked through an exact
  rational product (1 for K <= 2);
* x1(K) lies between the root of Gamma(K+1/2, x)/(2 x^(K+1/2)) = 4.9e-14 (the
  fitting target, which leaves room for the evaluation's rounding) and the
  next double (mpmath, the equation evaluated directly), so the asymptote is
  within 4.9e-14 for F_K beyond it; checked against the oracle for every
  order up to K at x1(K);
* row 32 is the paper's printed set, entry for entry.
For both sets:
* the header repeats the record, with monic denominators;
* every rational, with its coefficients rounded to double, meets the fitting
  target against the oracle on a dense grid (weight rho_{A,K} on A, 1 on B),
  and the fit itself equioscillates on n+m+2 points;
* an emulation of the evaluator's arithmetic in float64 keeps every order
  0..K within 5e-14 of the oracle on all three regions (the per-kmax set at
  every K, the centre set at a spread of K);
* the choice on the Walsh table: for a sample of rows the anti-diagonal below
  the chosen one has no entry meeting the target (the chosen one is the
  first feasible), and the centre set's chosen entry is the one nearest the
  centre among the feasible entries the record lists, of which the
  entries nearer the centre are re-checked infeasible for one row;
* the checks fail for a perturbed coefficient."""
import json
import math
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle
from tests.coeff_header import CSRC, _defines, load_f64
from tests.test_coeff_tables_sets import (LD, alternations, assert_fit_equioscillates, emulate,
                                          horner_ld, rho_a, weighted_error)

EPS = 5e-14
PAPER = load_f64()


def _num(c):
    c = c.strip()
    return float.fromhex(c) if "0x" in c else float(c)


def _nested(v):
    """A brace initialiser of hex-float or decimal numbers: a list, or a list
    of rows."""
    import re
    v = v.strip()
    if v[1:].lstrip().startswith("{"):
        return [[_num(c) for c in r.split(",") if c.strip()] for r in re.findall(r"\{([^{}]*)\}", v[1:-1])]
    return [_num(c) for c in v[1:-1].split(",") if c.strip()]


def _ints(v):
    return [int(c) for c in _nested(v)]


def load_perk():
    d = _defines(os.path.join(CSRC, "boys_coeffs_f64_perk.h"))
    rec = json.load(open(os.path.join(CSRC, "boys_coeffs_f64_perk.json")))
    x0 = [float(c) for c in _nested(d["BOYS_PK_X0_INIT"])]
    x1 = [float(c) for c in _nested(d["BOYS_PK_X1_INIT"])]
    bn, bm = _ints(d["BOYS_PK_RB_N_INIT"]), _ints(d["BOYS_PK_RB_M_INIT"])
    an, am = _ints(d["BOYS_PK_RA_N_INIT"]), _ints(d["BOYS_PK_RA_M_INIT"])
    BP, BQ = _nested(d["BOYS_PK_RB_P_INIT"]), _nested(d["BOYS_PK_RB_Q_INIT"])
    AP, AQ = _nested(d["BOYS_PK_RA_P_INIT"]), _nested(d["BOYS_PK_RA_Q_INIT"])
    rows = []
    for K in range(33):
        rows.append(dict(K=K, x0=x0[K], x1=x1[K], rb=(BP[K][:bn[K] + 1], BQ[K][:bm[K] + 1]),
                         ra=(AP[K][:an[K] + 1], AQ[K][:am[K] + 1]), rb_deg=(bn[K], bm[K]),
                         ra_deg=(an[K], am[K]), rb_full=(BP[K], BQ[K]), ra_full=(AP[K], AQ[K])))
    return rows, rec, int(d["BOYS_PK_KMAX"]), float(d["BOYS_PK_EPS"])


def load_centre():
    d = _defines(os.path.join(CSRC, "boys_coeffs_f64_centre.h"))
    rec = json.load(open(os.path.join(CSRC, "boys_coeffs_f64_centre.json")))
    degn, degm = _ints(d["BOYS_CTR_RA_DEG_N_INIT"]), _ints(d["BOYS_CTR_RA_DEG_M_INIT"])
    P, Q = _nested(d["BOYS_CTR_RA_P_INIT"]), _nested(d["BOYS_CTR_RA_Q_INIT"])
    ra = [(P[k][:degn[k] + 1], Q[k][:degm[k] + 1]) for k in range(33)]
    rb = (_nested(d["BOYS_CTR_RB_P_INIT"]), _nested(d["BOYS_CTR_RB_Q_INIT"]))
    return dict(x0=_num(d["BOYS_CTR_X0"]), x1=_num(d["BOYS_CTR_X1"]), ra=ra, rb=rb,
                degn=degn, degm=degm, rb_deg=(int(d["BOYS_CTR_RB_N"]), int(d["BOYS_CTR_RB_M"])),
                P_full=P, Q_full=Q, rec=rec, target=rec["target"], eps=float(d["BOYS_CTR_EPS"]))


PK, PK_REC, PK_KMAX, PK_EPS = load_perk()
CT = load_centre()
TARGET = PK_REC["target"]


def as_set(row):
    """A per-kmax row in the layout emulate() reads (only row K of ra is used)."""
    K = row["K"]
    return dict(x0=row["x0"], x1=row["x1"], rb=row["rb"], ra=[None] * K + [row["ra"]])


# --------------------------------------------------------------------------
# Per-kmax regions.

def test_per_kmax_header_basics():
    assert PK_KMAX == 32 and PK_EPS == EPS and len(PK) == 33
    assert PK_REC["eps"] == EPS and PK_REC["target"] <= EPS and PK_REC["kmax"] == 31


@pytest.mark.parametrize("K", range(33))
def test_per_kmax_x0_is_the_product_formula(K):
    mp.mp.dps = 50
    x0 = PK[K]["x0"]
    if K == 32:
        assert x0 == 11.899848152108484  # the paper's printed value
        return
    prod = Fraction(1)
    for n in range(K):
        prod *= Fraction(2 * n + 1, 2)
    exact = mp.root(mp.mpf(prod.numerator) / mp.mpf(prod.denominator), K) if K else mp.mpf(0)
    exact = max(exact, mp.mpf(1))
    assert abs(mp.mpf(x0) - exact) <= mp.mpf(math.ulp(x0)) / 2 * (1 + mp.mpf(10) ** -20)
    assert (x0 == 1.0) == (K <= 2)


@pytest.mark.parametrize("K", range(32))
def test_per_kmax_x1_brackets_the_root(K):
    mp.mp.dps = 50
    s = K + mp.mpf(1) / 2
    err = lambda x: mp.gammainc(s, mp.mpf(x)) / (2 * mp.mpf(x) ** s)
    x1 = PK[K]["x1"]
    assert err(x1) <= TARGET < err(np.nextafter(x1, 0.0))
    assert PK[K]["x0"] < x1 <= PK[32]["x1"] + 1e-9


@pytest.mark.parametrize("K", [0, 1, 2, 3, 7, 12, 20, 31])
def test_per_kmax_asymptote_within_eps_at_x1(K):
    x1 = PK[K]["x1"]
    F = oracle.boys_ld(np.array([x1], dtype=LD), K)[0]
    asym = LD(math.sqrt(math.pi)) / 2 / np.sqrt(LD(x1))
    for k in range(K + 1):
        assert abs(F[k] - asym) <= TARGET, k
        asym = asym * (LD(k) + LD(0.5)) / LD(x1)


def test_per_kmax_row_32_is_the_papers_set():
    r = PK[32]
    assert r["x0"] == PAPER["x0"] and r["x1"] == PAPER["x1"]
    assert list(r["rb"][0]) == list(PAPER["rb"][0]) and list(r["rb"][1]) == list(PAPER["rb"][1])
    assert list(r["ra"][0]) == list(PAPER["ra"][32][0]) and list(r["ra"][1]) == list(PAPER["ra"][32][1])


@pytest.mark.parametrize("K", range(32))
def test_per_kmax_header_matches_record(K):
    r = PK[K]
    tb, ta = PK_REC["rb"][K], PK_REC["ra"][K]
    assert PK_REC["x0"][K] == r["x0"] and PK_REC["x1"][K] == r["x1"]
    assert (tb["n"], tb["m"]) == r["rb_deg"] and (ta["n"], ta["m"]) == r["ra_deg"]
    assert tb["p"] == list(r["rb"][0]) and tb["q"] == list(r["rb"][1])
    assert ta["p"] == list(r["ra"][0]) and ta["q"] == list(r["ra"][1])
    assert ta["k"] == K and ta["a"] == 0.0 and ta["b"] == r["x0"]
    assert tb["a"] == r["x0"] and tb["b"] == r["x1"]
    for (p, q), (pf, qf), (n, m) in ((r["rb"], r["rb_full"], r["rb_deg"]), (r["ra"], r["ra_full"], r["ra_deg"])):
        assert q[-1] == 1.0  # monic
        assert all(v == 0.0 for v in list(pf[n + 1:]) + list(qf[m + 1:]))


@pytest.mark.parametrize("K", range(32))
def test_per_kmax_rationals_meet_target_and_equioscillate(K):
    r = PK[K]
    x, e = weighted_error(*r["ra"], K, 0.0, r["x0"], lambda x: rho_a(K, x))
    assert float(np.max(np.abs(e))) <= TARGET * (1 + 1e-9), f"r_A,{K}"
    assert_fit_equioscillates(PK_REC["ra"][K], K, 0.0, r["x0"], lambda x: rho_a(K, x), sum(r["ra_deg"]) + 2)
    x, e = weighted_error(*r["rb"], 0, r["x0"], r["x1"], lambda x: np.ones_like(x))
    assert float(np.max(np.abs(e))) <= TARGET * (1 + 1e-9), f"r_B ({K})"
    assert_fit_equioscillates(PK_REC["rb"][K], 0, r["x0"], r["x1"], lambda x: np.ones_like(x),
                              sum(r["rb_deg"]) + 2)


def region_grid(x0, x1):
    pts = [np.linspace(0.0, x0, 1501), np.linspace(x0, x1, 2001), np.linspace(x1, 60.0, 501)]
    edge = []
    for b in (x0, x1):
        v = b
        for _ in range(3):
            v = np.nextafter(v, 0.0)
        for _ in range(7):
            edge.append(v)
            v = np.nextafter(v, np.inf)
    return np.concatenate(pts + [np.array(edge)])


@pytest.mark.parametrize("K", range(33))
def test_per_kmax_emulated_evaluator_within_eps(K):
    r = PK[K]
    x = region_grid(r["x0"], r["x1"])
    err = np.abs(emulate(as_set(r), x, K) - oracle.boys(x, K))
    assert err.max() <= EPS, f"K={K}: {err.max():.3e}"


def feasible(which, k, a, b, n, m, target=TARGET):
    """Does the Remez fit of this Walsh-table entry meet the target with its
    coefficients rounded to double (the generators' acceptance rule)?"""
    from paper_2512_10059_amd import remez
    f = remez.boys_k(0 if which == "B" else k)
    rho = remez.rho_one if which == "B" else remez.rho_a(k)
    try:
        res = remez.remez(f, rho, a, b, n, m, tol=1e-3, target=target, dps=30, max_iter=30)
    except remez.RemezFailure:
        return False
    if res.max_err > target:
        return False
    x, e = weighted_error([float(c) for c in res.p], [float(c) for c in res.q], 0 if which == "B" else k,
                          a, b, lambda t: rho(t))
    return float(np.max(np.abs(e))) <= target


@pytest.mark.parametrize("which,K", [("A", 5), ("B", 24), ("B", 31)])
def test_per_kmax_degree_is_the_first_feasible_antidiagonal(which, K):
    r = PK[K]
    n, m = r["ra_deg"] if which == "A" else r["rb_deg"]
    a, b = (0.0, r["x0"]) if which == "A" else (r["x0"], r["x1"])
    for mm in range(n + m):
        assert not feasible(which, K, a, b, n + m - 1 - mm, mm), (n + m - 1 - mm, mm)


def test_per_kmax_checks_detect_a_perturbed_coefficient():
    r = PK[9]
    p, q = list(r["ra"][0]), r["ra"][1]
    p[0] *= 1 + 1e-8
    x, e = weighted_error(p, q, 9, 0.0, r["x0"], lambda x: rho_a(9, x))
    assert np.max(np.abs(e)) > TARGET
    bp, bq = list(r["rb"][0]), r["rb"][1]
    bp[1] *= 1 + 1e-8
    x, e = weighted_error(bp, bq, 0, r["x0"], r["x1"], lambda x: np.ones_like(x))
    assert np.max(np.abs(e)) > TARGET
    broken = dict(as_set(r), x1=np.nextafter(r["x1"], 0.0) - 0.05)  # asymptote too early
    x = region_grid(r["x0"], r["x1"])
    assert np.abs(emulate(broken, x, 9) - oracle.boys(x, 9)).max() > EPS


# --------------------------------------------------------------------------
# Centre of the anti-diagonal.

def test_centre_regions_are_the_papers():
    assert CT["x0"] == PAPER["x0"] and CT["x1"] == PAPER["x1"] and CT["eps"] == EPS
    assert CT["rec"]["x0"] == CT["x0"] and CT["rec"]["x1"] == CT["x1"]


def test_centre_header_matches_record():
    rec = CT["rec"]
    assert (rec["rb"]["n"], rec["rb"]["m"]) == CT["rb_deg"]
    assert rec["rb"]["p"] == list(CT["rb"][0]) and rec["rb"]["q"] == list(CT["rb"][1])
    for k in range(33):
        t = rec["ra"][k]
        assert t["k"] == k and (t["n"], t["m"]) == (CT["degn"][k], CT["degm"][k])
        assert t["p"] == list(CT["ra"][k][0]) and t["q"] == list(CT["ra"][k][1])
        assert CT["ra"][k][1][-1] == 1.0
        assert all(v == 0.0 for v in list(CT["P_full"][k][t["n"] + 1:]) + list(CT["Q_full"][k][t["m"] + 1:]))


@pytest.mark.parametrize("k", [None] + list(range(33)))
def test_centre_pick_is_nearest_the_centre_of_its_antidiagonal(k):
    """Among the feasible entries the generator found on the chosen
    anti-diagonal (all on the same n + m), none is nearer the centre."""
    t = CT["rec"]["rb"] if k is None else CT["rec"]["ra"][k]
    feas = t["feasible"]
    assert [t["n"], t["m"]] in feas
    assert len({n + m for n, m in feas}) == 1
    assert abs(t["n"] - t["m"]) == min(abs(n - m) for n, m in feas)


def test_centre_entries_nearer_the_centre_are_infeasible():
    """Row 3's pick (4, 12) is far from the centre of n + m = 16: every entry
    between it and the centre fails the target (re-run here)."""
    n, m = CT["degn"][3], CT["degm"][3]
    assert (n, m) == (4, 12)
    for nn in range(5, 9):
        assert not feasible("A", 3, 0.0, CT["x0"], nn, 16 - nn), (nn, 16 - nn)


@pytest.mark.parametrize("k", [None, 0, 1, 2, 3, 5, 7, 9, 10, 12, 20, 26, 32])
def test_centre_rationals_meet_target_and_equioscillate(k):
    if k is None:
        x, e = weighted_error(*CT["rb"], 0, CT["x0"], CT["x1"], lambda x: np.ones_like(x))
        assert float(np.max(np.abs(e))) <= CT["target"] * (1 + 1e-9)
        assert_fit_equioscillates(CT["rec"]["rb"], 0, CT["x0"], CT["x1"], lambda x: np.ones_like(x),
                                  sum(CT["rb_deg"]) + 2)
        return
    x, e = weighted_error(*CT["ra"][k], k, 0.0, CT["x0"], lambda x: rho_a(k, x))
    assert float(np.max(np.abs(e))) <= CT["target"] * (1 + 1e-9), f"r_A,{k}"
    assert_fit_equioscillates(CT["rec"]["ra"][k], k, 0.0, CT["x0"], lambda x: rho_a(k, x),
                              CT["degn"][k] + CT["degm"][k] + 2)


@pytest.mark.parametrize("kmax", [0, 1, 2, 3, 5, 7, 9, 12, 16, 20, 26, 32])
def test_centre_emulated_evaluator_within_eps(kmax):
    x = region_grid(CT["x0"], CT["x1"])
    err = np.abs(emulate(CT, x, kmax) - oracle.boys(x, kmax))
    assert err.max() <= EPS, f"kmax={kmax}: {err.max():.3e}"
