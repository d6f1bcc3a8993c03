"""Constants of the VALU-bound consumer kernels (batched weighted sums, pair
sums): the table-driven e^{-x} and the region-C coefficients.

Pins, none of which reuses the generator's arithmetic:
* every table entry T_i is the double nearest 2^(i/128), checked in exact
  integer arithmetic: 2^i lies between (T_i - ulp/2)^128 and (T_i + ulp/2)^128;
* ln2/128 = L_HI + L_LO to 1e-32 relative, checked through exp, not log;
* the kernel's sequence of roundings (fused multiply-adds emulated exactly
  with rationals) stays within 2^-52 relative of e^{-x} on [0, 32), the
  bound of the method (table rounding plus one final rounding);
* a_l = Gamma(l + 1/2)/2 is the double nearest (sqrt(pi)/2) prod_{m<l} (m + 1/2),
  the product taken exactly in rationals (the generator uses the gamma
  function), and a_l x^(-l-1/2) reproduces the upward asymptote recurrence."""
import math
import os
import re
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from tests.coeff_header import CSRC

HEADER = os.path.join(CSRC, "boys_consumer_tables.h")


def load():
    text = open(HEADER).read().replace("\\\n", " ")
    d = dict(re.findall(r"^#define\s+(\w+)\s+(.*)$", text, re.M))
    vec = lambda name: [float.fromhex(v.strip()) for v in d[name].strip()[1:-1].split(",")]
    return dict(bits=int(d["BOYS_EXP_TABLE_BITS"]), inv_l=float.fromhex(d["BOYS_EXP_INV_L"]),
                l_hi=float.fromhex(d["BOYS_EXP_L_HI"]), l_lo=float.fromhex(d["BOYS_EXP_L_LO"]),
                tab=vec("BOYS_EXP_TABLE_INIT"), asym=vec("BOYS_ASYM_COEF_INIT"),
                asym_orders=int(d["BOYS_ASYM_ORDERS"]))


C = load()


def fma(a, b, c):
    """Correctly rounded a*b + c (Fraction arithmetic is exact; float() of a
    Fraction rounds once, to nearest even)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def exp_neg_emulated(x):
    """The device routine's operations in its order, each rounded as the
    hardware rounds it."""
    nd = float(round(x * C["inv_l"]))          # v_rndne_f64 of the rounded product
    r = fma(-nd, C["l_hi"], x)
    r = fma(-nd, C["l_lo"], r)
    N = -int(nd)
    T = C["tab"][N & ((1 << C["bits"]) - 1)]
    v = r - 5.0
    v = fma(v, r, 20.0)
    v = fma(v, r, -60.0)
    v = fma(v, r, 120.0)
    q = (r * (-1.0 / 120.0)) * v
    return math.ldexp(fma(T, q, T), N >> C["bits"])


def test_table_is_correctly_rounded():
    n = 1 << C["bits"]
    assert len(C["tab"]) == n
    for i, t in enumerate(C["tab"]):
        assert 1.0 <= t < 2.0
        half_ulp = Fraction(math.ulp(t)) / 2
        lo, hi = Fraction(t) - half_ulp, Fraction(t) + half_ulp
        target = Fraction(2) ** i
        assert lo ** n <= target <= hi ** n, f"entry {i} is not the nearest double to 2^({i}/{n})"


def test_split_of_ln2_over_table_length():
    mp.mp.dps = 50
    n = 1 << C["bits"]
    s = mp.mpf(C["l_hi"]) + mp.mpf(C["l_lo"])
    assert abs(mp.exp(n * s) / 2 - 1) < mp.mpf("1e-32")
    assert abs(C["l_lo"]) <= math.ulp(C["l_hi"])       # a genuine two-part split
    assert abs(C["inv_l"] * C["l_hi"] - 1.0) < 1e-15


def arguments():
    rng = np.random.default_rng(42)
    pts = list(rng.uniform(0.0, 32.0, 3000)) + list(np.exp(rng.uniform(np.log(1e-300), np.log(1.0), 500)))
    L = math.log(2) / (1 << C["bits"])
    for m in (1, 2, 63, 64, 127, 128, 129, 1000, 5000, 5900):   # reduction interval edges
        c = (m + 0.5) * L
        pts += [np.nextafter(c, 0.0), c, np.nextafter(c, 99.0), m * L]
    pts += [0.0, 5e-324, 1e-17, 11.899848152108484, 28.98933773882074, 31.999]
    return pts


def test_emulated_routine_within_two_ulps_relative():
    mp.mp.dps = 40
    worst = 0.0
    for x in arguments():
        got = exp_neg_emulated(float(x))
        ref = mp.exp(-mp.mpf(float(x)))
        rel = float(abs((mp.mpf(got) - ref) / ref))
        worst = max(worst, rel)
    assert worst <= 2.0 ** -52, f"worst relative error {worst:.3e}"


@pytest.mark.parametrize("mutation", ["index", "sign", "lo", "coef"])
def test_emulation_detects_planted_mistakes(mutation):
    """The accuracy check above fails for plausible mistakes in the routine."""
    saved = dict(C)
    try:
        if mutation == "index":
            C["tab"] = C["tab"][1:] + C["tab"][:1]
        elif mutation == "sign":
            C["l_hi"] = -C["l_hi"]
        elif mutation == "lo":
            C["l_lo"] = 0.0
        elif mutation == "coef":
            C["inv_l"] = C["inv_l"] * 0.5   # picks the wrong N: |r| leaves the polynomial's range
        with pytest.raises(AssertionError):
            test_emulated_routine_within_two_ulps_relative()
    finally:
        C.clear()
        C.update(saved)


def test_asymptote_coefficients_correctly_rounded():
    mp.mp.dps = 50
    assert C["asym_orders"] == 33 and len(C["asym"]) == 33
    half_sqrt_pi = mp.sqrt(mp.pi) / 2
    prod = Fraction(1)
    for l, a in enumerate(C["asym"]):
        exact = half_sqrt_pi * mp.mpf(prod.numerator) / mp.mpf(prod.denominator)
        half_ulp = mp.mpf(math.ulp(a)) / 2
        assert abs(mp.mpf(a) - exact) <= half_ulp, f"a_{l} is not the nearest double"
        prod *= Fraction(2 * l + 1, 2)


def test_asymptote_coefficients_reproduce_the_recurrence():
    """a_l x^(-l-1/2) equals the region-C recurrence F_0 = (sqrt(pi)/2) x^(-1/2),
    F_{l+1} = F_l (l + 1/2)/x, here run in 50-digit arithmetic."""
    mp.mp.dps = 50
    for x in (28.98933773882074, 30.0, 57.5, 1e3):
        F = mp.sqrt(mp.pi) / 2 / mp.sqrt(x)
        for l, a in enumerate(C["asym"]):
            assert abs(mp.mpf(a) * mp.mpf(x) ** (-l - mp.mpf(1) / 2) / F - 1) < mp.mpf(2.0 ** -52)
            F = F * (l + mp.mpf(1) / 2) / x


def region_b_polys(c):
    """P and Q of the pair kernel's region-B closed form, built by the same
    rules as the library's host code: A_l = (2l-1)!! g^l, B_0 = 0,
    B_{l+1} = g ((2l+1) B_l + 1); P = sum c_l A_l, Q = sum c_l B_l."""
    K = len(c) - 1
    a, b = mp.mpf(1), [mp.mpf(0)] * (K + 2)
    p, q = [mp.mpf(0)] * (K + 1), [mp.mpf(0)] * (K + 1)
    for l in range(K + 1):
        p[l] = c[l] * a
        for j in range(1, l + 1):
            q[j] += c[l] * b[j]
        for j in range(l + 1, 1, -1):
            b[j] = (2 * l + 1) * b[j - 1]
        b[1] = mp.mpf(1)
        a *= 2 * l + 1
    return p, q


@pytest.mark.parametrize("K", [0, 1, 5, 12, 32])
def test_region_b_closed_form_equals_the_upward_recurrence(K):
    """sum_l c_l F_l with F_{l+1} = ((2l+1) F_l - e^-x)/(2x) from any F_0 equals
    F_0 P(g) - e^-x Q(g), g = 1/(2x) (identity of the recurrence, checked in
    50-digit arithmetic for arbitrary F_0 and weights)."""
    mp.mp.dps = 50
    rng = np.random.default_rng(K)
    c = [mp.mpf(float(v)) for v in rng.standard_normal(K + 1)]
    p, q = region_b_polys(c)
    for x in (11.9, 15.0, 23.0, 28.98):
        x = mp.mpf(x)
        e = mp.exp(-x)
        F = mp.mpf(float(rng.uniform(0.1, 1.0)))  # any starting value
        g = 1 / (2 * x)
        closed = F * mp.polyval(p[::-1], g) - e * mp.polyval(q[::-1], g)
        s = c[0] * F
        for l in range(K):
            F = ((2 * l + 1) * F - e) / (2 * x)
            s += c[l + 1] * F
        assert abs(closed - s) <= mp.mpf(10) ** -40 * (1 + abs(s))


def test_region_b_closed_form_check_detects_a_wrong_shift():
    """A mutant of the construction (B_{l+1} without the shift by g) fails."""
    mp.mp.dps = 50
    c = [mp.mpf(v) for v in (0.3, -1.2, 0.7, 2.0)]
    p, q = region_b_polys(c)
    q_bad = q[1:] + [mp.mpf(0)]
    x = mp.mpf(13.0)
    e, g, F = mp.exp(-x), 1 / (2 * mp.mpf(13.0)), mp.mpf(0.5)
    s = c[0] * F
    for l in range(3):
        F = ((2 * l + 1) * F - e) / (2 * x)
        s += c[l + 1] * F
    bad = mp.mpf(0.5) * mp.polyval(p[::-1], g) - e * mp.polyval(q_bad[::-1], g)
    assert abs(bad - s) > mp.mpf(10) ** -10
