"""The FP64 table set for eps_tol = 1e-10 ("screening"), generated with the
library's Remez tool by csrc/gen_coeffs_f64_screen.py, pinned against the
long-double oracle and the paper's definitions (Sec. II C-D):

* x0 is the paper's (it depends only on kmax) and equals
  (prod_{n<32} (n+1/2))^(1/32);
* the asymptote-error equation Gamma(32.5, x)/(2 x^32.5) = 1e-10 has its root
  between the previous double and x1 (evaluated directly, not in the
  generator's logarithmic form), and at x1 the asymptote is within 1e-10 of
  the oracle for every order 0..32;
* every r_{A,k} (weighted by rho_{A,k}) and r_B meets 1e-10 against the
  oracle on a dense grid and equioscillates on n+m+2 points;
* an emulation of the kernel's arithmetic (rational, exp, recurrences,
  asymptote) in float64 keeps every order 0..32 within 1e-10 of the oracle
  on all three regions;
* r_B's degree is minimal: the anti-diagonal below it has no entry meeting
  1e-10;
* the checks fail for a perturbed coefficient."""
import json
import math
import os
import re

import mpmath as mp
import numpy as np
import pytest

import oracle
from tests.coeff_header import CSRC

EPS = 1e-10
LD = np.longdouble
HEADER = os.path.join(CSRC, "boys_coeffs_f64_screen.h")
RECORD = os.path.join(CSRC, "boys_coeffs_f64_screen.json")


def load_header():
    text = open(HEADER).read().replace("\\\n", " ")
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    d = dict(re.findall(r"^#define\s+(\w+)\s+(.*)$", text, re.M))
    num = lambda v: float.fromhex(v.strip())
    rows = lambda v: [[num(c) for c in r.split(",")] for r in re.findall(r"\{([^{}]*)\}", v.strip()[1:-1])]
    vec = lambda v: [num(c) for c in v.strip()[1:-1].split(",")]
    ints = lambda v: [int(c) for c in v.strip()[1:-1].split(",")]
    degn, degm = ints(d["BOYS_SCR_RA_DEG_N_INIT"]), ints(d["BOYS_SCR_RA_DEG_M_INIT"])
    P, Q = rows(d["BOYS_SCR_RA_P_INIT"]), rows(d["BOYS_SCR_RA_Q_INIT"])
    ra = [(P[k][:degn[k] + 1], Q[k][:degm[k] + 1]) for k in range(33)]
    rb = (vec(d["BOYS_SCR_RB_P_INIT"]), vec(d["BOYS_SCR_RB_Q_INIT"]))
    return dict(x0=num(d["BOYS_SCR_X0"]), x1=num(d["BOYS_SCR_X1"]), ra=ra, rb=rb,
                rb_deg=(int(d["BOYS_SCR_RB_N"]), int(d["BOYS_SCR_RB_M"])),
                P_full=P, Q_full=Q, degn=degn, degm=degm)


H = load_header()


def rho_a(k, x):
    """Weight of region A: the largest amplification of an error in F_k by
    the downward recurrence, max_l prod_{n=l}^{k-1} x/(n+1/2)."""
    x = np.asarray(x, dtype=LD)
    best = np.ones_like(x)
    prod = np.ones_like(x)
    for n in range(k - 1, -1, -1):
        prod = prod * x / (LD(n) + LD(0.5))
        best = np.maximum(best, prod)
    return best


def horner_ld(c, x):
    v = np.zeros_like(x)
    for a in reversed(c):
        v = v * x + LD(a)
    return v


def weighted_error(p, q, k, a, b, weight, npts=8001):
    x = np.linspace(LD(a), LD(b), npts, dtype=LD)
    f = oracle.boys_ld(x, k)[:, k]
    w = weight(x)
    return x, w * (f - horner_ld(p, x) / horner_ld(q, x))


def test_x0_is_the_papers_and_the_product_formula():
    assert H["x0"] == 11.899848152108484
    x0 = math.exp((math.lgamma(32.5) - math.lgamma(0.5)) / 32)  # prod_{n<32}(n+1/2) = G(32.5)/G(0.5)
    assert abs(H["x0"] - x0) <= 2e-15 * x0


def test_x1_brackets_the_root_of_the_asymptote_error_equation():
    mp.mp.dps = 50
    s = mp.mpf(65) / 2
    err = lambda x: mp.gammainc(s, mp.mpf(x)) / (2 * mp.mpf(x) ** s)
    x1 = H["x1"]
    assert err(x1) <= EPS < err(np.nextafter(x1, 0.0))
    assert abs(x1 - 23.149988540679747) < 1e-13


def test_asymptote_within_eps_at_x1_for_every_order():
    x1 = H["x1"]
    F = oracle.boys_ld(np.array([x1], dtype=LD), 32)[0]
    asym = LD(math.sqrt(math.pi)) / 2 / np.sqrt(LD(x1))
    for k in range(33):
        assert abs(F[k] - asym) <= EPS, k
        asym = asym * (LD(k) + LD(0.5)) / LD(x1)


def test_header_matches_record():
    rec = json.load(open(RECORD))
    assert rec["x1"] == H["x1"] and rec["x0"] == H["x0"] and rec["eps"] == EPS
    assert (rec["rb"]["n"], rec["rb"]["m"]) == H["rb_deg"]
    assert rec["rb"]["p"] == H["rb"][0] and rec["rb"]["q"] == H["rb"][1]
    for k in range(33):
        t = rec["ra"][k]
        assert t["k"] == k and (t["n"], t["m"]) == (H["degn"][k], H["degm"][k])
        assert t["p"] == H["ra"][k][0] and t["q"] == H["ra"][k][1]
        assert H["ra"][k][1][-1] == 1.0  # monic
        assert all(v == 0.0 for v in H["P_full"][k][t["n"] + 1:] + H["Q_full"][k][t["m"] + 1:])


def alternations(e, level):
    """Number of sign alternations among the extrema of e with |e| >= level."""
    signs = []
    i, n = 0, len(e)
    while i < n:
        if abs(e[i]) >= level:
            j = i
            while j + 1 < n and abs(e[j + 1]) >= level and np.sign(e[j + 1]) == np.sign(e[i]):
                j += 1
            s = int(np.sign(e[i]))
            if not signs or signs[-1] != s:
                signs.append(s)
            i = j + 1
        else:
            i += 1
    return len(signs)


@pytest.mark.parametrize("k", list(range(0, 33, 4)) + [1, 2, 3, 26, 31])
def test_region_a_rational_meets_eps_and_equioscillates(k):
    p, q = H["ra"][k]
    x, e = weighted_error(p, q, k, 0.0, H["x0"], lambda x: rho_a(k, x))
    E = float(np.max(np.abs(e)))
    assert E <= EPS * (1 + 1e-9), f"r_A,{k}: {E:.3e}"
    n, m = H["degn"][k], H["degm"][k]
    assert alternations(e.astype(float), 0.97 * E) >= n + m + 2


def test_region_b_rational_meets_eps_and_equioscillates():
    p, q = H["rb"]
    x, e = weighted_error(p, q, 0, H["x0"], H["x1"], lambda x: np.ones_like(x))
    E = float(np.max(np.abs(e)))
    assert E <= EPS * (1 + 1e-9)
    n, m = H["rb_deg"]
    assert alternations(e.astype(float), 0.97 * E) >= n + m + 2


def emulate(x, kmax):
    """The evaluator's steps in float64: region A: r_{A,kmax} then the
    downward recurrence; B: r_B then the upward recurrence; C: the
    asymptote.  (FMA roundings differ from the device's by ~1e-16, far
    below 1e-10.)"""
    x = np.asarray(x, dtype=np.float64)
    F = np.empty((x.size, kmax + 1))
    e = np.exp(-x)
    A = x < H["x0"]
    C = x > H["x1"]
    B = ~A & ~C
    horner = lambda c, t: np.polyval(np.asarray(c, dtype=np.float64)[::-1], t)
    p, q = H["ra"][kmax]
    xa = x[A]
    G = horner(p, xa) / horner(q, xa)
    F[A, kmax] = G
    for l in range(kmax - 1, -1, -1):
        G = (2 * xa * G + e[A]) / (2 * l + 1)
        F[A, l] = G
    p, q = H["rb"]
    xb = x[B]
    G = horner(p, xb) / horner(q, xb)
    F[B, 0] = G
    for l in range(kmax):
        G = ((2 * l + 1) * G - e[B]) / (2 * xb)
        F[B, l + 1] = G
    xc = x[C]
    G = math.sqrt(math.pi) / 2 / np.sqrt(xc)
    F[C, 0] = G
    for l in range(kmax):
        G = G * (l + 0.5) / xc
        F[C, l + 1] = G
    return F


def grid():
    x0, x1 = H["x0"], H["x1"]
    pts = [np.linspace(0.0, x0, 3001), np.linspace(x0, x1, 2001), np.linspace(x1, 60.0, 1001),
           np.array([np.nextafter(x0, 0), x0, np.nextafter(x1, 0), x1, np.nextafter(x1, 99)])]
    return np.concatenate(pts)


@pytest.mark.parametrize("kmax", [0, 1, 2, 5, 8, 12, 16, 20, 24, 26, 29, 32])
def test_emulated_evaluator_within_eps_for_every_order(kmax):
    x = grid()
    err = np.abs(emulate(x, kmax) - oracle.boys(x, kmax))
    assert err.max() <= EPS * (1 + 1e-4), f"kmax={kmax}: {err.max():.3e}"


def test_region_b_degree_is_minimal():
    from paper_2512_10059_amd import remez
    n, m = H["rb_deg"]
    for mm in range(0, n + m):
        nn = n + m - 1 - mm
        try:
            r = remez.remez(remez.boys_k(0), remez.rho_one, H["x0"], H["x1"], nn, mm, tol=1e-3,
                            target=EPS, dps=30, max_iter=30)
        except remez.RemezFailure:
            continue
        assert r.max_err > EPS, f"({nn},{mm}) below the chosen anti-diagonal meets eps"


def test_checks_detect_a_perturbed_coefficient():
    p, q = H["ra"][16]
    p = list(p)
    p[0] *= 1 + 1e-8
    x, e = weighted_error(p, q, 16, 0.0, H["x0"], lambda x: rho_a(16, x))
    assert np.max(np.abs(e)) > EPS
