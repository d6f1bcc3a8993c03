"""Constants of the VALU-bound consumer kernels (batched weighted sums, pair
sums): the table-free e^{-x} and the region-C coefficients.

Pins, none of which reuses the generator's arithmetic:
* every Taylor coefficient c_j is the double nearest 1/j!, checked in exact
  integer arithmetic: |c_j j! - 1| <= j! ulp(c_j)/2;
* ln2 = LN2_HI + LN2_LO to 1e-32 relative, checked through exp, not log,
  and 1/ln2 through its product with LN2_HI;
* the kernel's sequence of roundings (fused multiply-adds emulated exactly
  with rationals) stays within 2^-52 relative of e^{-x} on [0, 32), the
  bound stated for the routine (one rounding in the reduction, Horner's
  roundings damped by |r| <= ln2/2, truncation below 1e-17);
* a_l = Gamma(l + 1/2)/2 is the double nearest (sqrt(pi)/2) prod_{m<l} (m + 1/2),
  the product taken exactly in rationals (the generator uses the gamma
  function), and a_l x^(-l-1/2) reproduces the upward asymptote recurrence;
* (2l-1)!! and 1/(2l-1)!! are the doubles nearest the exact integers and
  rationals;
* the batched consumer's weight sweeps (the kernel's table entries, padding
  and operation order, emulated in FP64 with exact fused multiply-adds) give
  sum_l w_l F_l to within their rounding bound for every order 0..32, with the
  exact F_l from mpmath's incomplete gamma and the exact seed and e^-x, so a
  mistake in the algebra shows as an O(1) error; planted mistakes fail; and
  the kernel's power-of-two-scaled, first-step-peeled form gives the same
  doubles as the plain recurrence."""
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
    return dict(inv_ln2=float.fromhex(d["BOYS_EXP_INV_LN2"]), ln2_hi=float.fromhex(d["BOYS_EXP_LN2_HI"]),
                ln2_lo=float.fromhex(d["BOYS_EXP_LN2_LO"]), degree=int(d["BOYS_EXP_DEGREE"]),
                taylor=vec("BOYS_EXP_TAYLOR_INIT"), asym=vec("BOYS_ASYM_COEF_INIT"),
                asym_orders=int(d["BOYS_ASYM_ORDERS"]), poly_orders=int(d["BOYS_POLY_ORDERS"]),
                dfact=vec("BOYS_DFACT_INIT"), inv_dfact=vec("BOYS_INV_DFACT_INIT"))


C = load()


def fma(a, b, c):
    """Correctly rounded a*b + c (Fraction arithmetic is exact; float() of a
    Fraction rounds once, to nearest even)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def exp_neg_emulated(x):
    """The device routine's operations in its order, each rounded as the
    hardware rounds it."""
    nd = float(round(x * C["inv_ln2"]))        # v_rndne_f64 of the rounded product
    r = fma(nd, C["ln2_hi"], -x)
    r = fma(nd, C["ln2_lo"], r)
    c = C["taylor"]
    p = float(Fraction(r) * Fraction(c[-1]))   # top term: product, then sum
    p = float(Fraction(p) + Fraction(c[-2]))
    for j in range(len(c) - 3, -1, -1):
        p = fma(p, r, c[j])
    return math.ldexp(p, -int(nd))


def test_taylor_coefficients_are_correctly_rounded():
    assert C["degree"] == 13 and len(C["taylor"]) == C["degree"] + 1
    for j, cj in enumerate(C["taylor"]):
        fact = math.factorial(j)
        assert abs(Fraction(cj) * fact - 1) <= Fraction(math.ulp(cj)) / 2 * fact, f"c_{j} is not the nearest double to 1/{j}!"


def test_taylor_truncation_bound():
    """The first omitted term at |r| = ln2/2 bounds the truncation: below 1e-17
    relative (Lagrange remainder e^xi r^14/14!, |xi| <= |r|, over e^r)."""
    r = math.log(2) / 2 * (1 + 1e-12)
    d = C["degree"] + 1
    assert r ** d / math.factorial(d) * math.exp(r) / math.exp(-r) < 1e-17


def test_split_of_ln2():
    mp.mp.dps = 50
    s = mp.mpf(C["ln2_hi"]) + mp.mpf(C["ln2_lo"])
    assert abs(mp.exp(s) / 2 - 1) < mp.mpf("1e-32")
    assert abs(C["ln2_lo"]) <= math.ulp(C["ln2_hi"])   # a genuine two-part split
    assert abs(C["inv_ln2"] * C["ln2_hi"] - 1.0) < 1e-15


def test_reduction_first_step_is_exact():
    """n LN2_HI - x needs no rounding for the n that rint(x/ln2) picks on the
    kernels' domain (checked exactly in rationals)."""
    rng = np.random.default_rng(7)
    for x in list(rng.uniform(0.0, 1024.0, 2000)) + list(rng.uniform(0.0, 1.0, 500)):
        x = float(x)
        nd = float(round(x * C["inv_ln2"]))
        exact = Fraction(nd) * Fraction(C["ln2_hi"]) - Fraction(x)
        assert Fraction(fma(nd, C["ln2_hi"], -x)) == exact


def arguments():
    rng = np.random.default_rng(42)
    pts = list(rng.uniform(0.0, 32.0, 3000)) + list(np.exp(rng.uniform(np.log(1e-300), np.log(1.0), 500)))
    L = math.log(2)
    for m in range(0, 47):                        # reduction interval edges
        c = (m + 0.5) * L
        pts += [np.nextafter(c, 0.0), c, np.nextafter(c, 99.0), m * L]
    pts += [0.0, 5e-324, 1e-17, 11.899848152108484, 14.842842360917231, 23.149988540679747,
            28.98933773882074, 30.455574446774907, 31.999]
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


@pytest.mark.parametrize("mutation", ["order", "sign", "lo", "pick", "degree"])
def test_emulation_detects_planted_mistakes(mutation):
    """The accuracy check above fails for plausible mistakes in the routine."""
    saved = dict(C)
    try:
        if mutation == "order":
            t = list(C["taylor"])
            t[3], t[4] = t[4], t[3]
            C["taylor"] = t
        elif mutation == "sign":
            C["ln2_hi"] = -C["ln2_hi"]
        elif mutation == "lo":
            C["ln2_lo"] = 0.0
        elif mutation == "pick":
            C["inv_ln2"] = C["inv_ln2"] * 0.5   # picks the wrong n: |r| leaves the polynomial's range
        elif mutation == "degree":
            C["taylor"] = C["taylor"][:-2]      # degree 11: truncation 6e-15 at |r| = ln2/2
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


def region_a_polys(c):
    """U and V of the pair kernel's region-A closed form, by the library's
    host rule: u_j = c_{K-j} (2K-2j-1)!!/(2K-1)!!,
    v_j = sum_{l=0}^{K-1-j} c_l (2l-1)!!/(2l+2j+1)!!."""
    K = len(c) - 1
    df = [mp.mpf(1)]
    for l in range(1, K + 2):
        df.append(df[-1] * (2 * l - 1))
    u = [c[K - j] * df[K - j] / df[K] for j in range(K + 1)]
    v = [sum((c[l] * df[l] / df[l + j + 1] for l in range(K - j)), mp.mpf(0)) for j in range(K + 1)]
    return u, v


@pytest.mark.parametrize("K", [0, 1, 5, 12, 32])
def test_region_a_closed_form_equals_the_downward_recurrence(K):
    """sum_l c_l F_l with F_l = (2x F_{l+1} + e^-x)/(2l+1) from any F_K equals
    F_K U(2x) + e^-x V(2x) (identity of the recurrence, 50-digit arithmetic,
    arbitrary F_K and weights)."""
    mp.mp.dps = 50
    rng = np.random.default_rng(100 + K)
    c = [mp.mpf(float(v)) for v in rng.standard_normal(K + 1)]
    u, v = region_a_polys(c)
    for x in (0.0, 0.3, 4.0, 11.89):
        x = mp.mpf(x)
        e = mp.exp(-x)
        F = mp.mpf(float(rng.uniform(0.01, 1.0)))  # any starting value
        t = 2 * x
        closed = F * mp.polyval(u[::-1], t) + e * mp.polyval(v[::-1], t)
        s = c[K] * F
        for l in range(K - 1, -1, -1):
            F = (2 * x * F + e) / (2 * l + 1)
            s += c[l] * F
        assert abs(closed - s) <= mp.mpf(10) ** -40 * (1 + abs(s))


def test_region_a_closed_form_check_detects_planted_mistakes():
    """Mutants of the construction (the double factorial one place off in V,
    U's coefficients in reverse order) fail the identity."""
    mp.mp.dps = 50
    c = [mp.mpf(v) for v in (0.3, -1.2, 0.7, 2.0, -0.4)]
    K = len(c) - 1
    u, v = region_a_polys(c)
    df = [mp.mpf(1)]
    for l in range(1, K + 3):
        df.append(df[-1] * (2 * l - 1))
    v_bad = [sum((c[l] * df[l] / df[l + j + 2] for l in range(K - j)), mp.mpf(0)) for j in range(K + 1)]
    x = mp.mpf(5.0)
    e, t, F = mp.exp(-x), 2 * mp.mpf(5.0), mp.mpf(0.02)
    s = c[K] * F
    for l in range(K - 1, -1, -1):
        F = (2 * x * F + e) / (2 * l + 1)
        s += c[l] * F
    for uu, vv in ((u, v_bad), (u[::-1], v)):
        bad = mp.mpf(0.02) * mp.polyval(uu[::-1], t) + e * mp.polyval(vv[::-1], t)
        assert abs(bad - s) > mp.mpf(10) ** -10


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


# ---------------------------------------------------------------------------
# The batched consumer's weight sweeps.

X0, X1 = 11.899848152108484, 28.98933773882074


def odd_dfact(l):
    v = 1
    for i in range(1, 2 * l, 2):
        v *= i
    return v


def test_double_factorial_tables_correctly_rounded():
    assert C["poly_orders"] == 33 and len(C["dfact"]) == 33 and len(C["inv_dfact"]) == 33
    for l in range(33):
        d = odd_dfact(l)
        assert abs(Fraction(C["dfact"][l]) - d) <= Fraction(math.ulp(C["dfact"][l])) / 2, l
        inv = Fraction(1, d)
        assert abs(Fraction(C["inv_dfact"][l]) - inv) <= Fraction(math.ulp(C["inv_dfact"][l])) / 2, l


def rnd(q):
    """The double nearest the rational q."""
    return float(q)


def sweep_entries_a(x, w, CH, mistake=None):
    """Region A's table entries (w_s D_s/D_k, D_k/D_s), (w_0/D_k, 0) at s = 0,
    zeros below, in the order the sweep takes them (upwards, padded below to
    whole chunks)."""
    k = len(w) - 1
    D, ID = C["dfact"], C["inv_dfact"]
    dk, idk = D[k], ID[k]
    out = []
    steps = (k + CH) & ~(CH - 1)
    for s in range(k + 1 - steps, k + 1):
        if s < 0:
            out.append((s, 0.0, 0.0))
            continue
        a = rnd(Fraction(w[s]) * Fraction(rnd(Fraction(D[s]) * Fraction(idk))))
        b = rnd(Fraction(ID[s]) * Fraction(dk)) if s >= 1 else 0.0
        if mistake == "no_scale":
            a = rnd(Fraction(w[s]) * Fraction(D[s]))
        out.append((s, a, b))
    return out


def sweep_entries_b(w, CH, mistake=None):
    """Region B's entries i = l-1: (w_i D_i, -1/D_{i+1}) for i < k,
    (w_k D_k, 0) at i = k, zeros above, in the sweep's order (downwards from
    the top of the padded range)."""
    k = len(w) - 1
    D, ID = C["dfact"], C["inv_dfact"]
    top = (k + CH) & ~(CH - 1)
    out = []
    for l in range(top, 0, -1):
        a = rnd(Fraction(w[l - 1]) * Fraction(D[l - 1])) if l - 1 <= k else 0.0
        b = -ID[l] if l <= k else 0.0
        if mistake == "sign":
            b = -b
        if mistake == "shift":
            a = rnd(Fraction(w[l]) * Fraction(D[l])) if 1 <= l <= k else 0.0
        out.append((l - 1, a, b))
    return out


def sweep_plain(mult, entries, mistake=None):
    """The sweeps' recurrence from z = v = 0: z <- mult z + a, v <- v + z_prev b."""
    z = v = 0.0
    for _, a, b in entries:
        if mistake == "new_z":
            z = fma(mult, z, a)
            v = fma(z, b, v)
        else:
            z, v = fma(mult, z, a), fma(z, b, v)
    return z, v


def sweep_kernel(mult, entries, mistake=None):
    """As the kernel runs it: the first step leaves z = a_0 (v stays 0), the
    second forms v by a multiply, the rest are fused multiply-adds."""
    (_, a0, _), (_, a1, b1) = entries[0], entries[1]
    z = a0
    v = z * b1
    z = fma(mult, z, a1)
    for _, a, b in entries[2:]:
        if mistake == "new_z":
            z = fma(mult, z, a)
            v = fma(z, b, v)
        else:
            z, v = fma(mult, z, a), fma(z, b, v)
    return z, v


def sweep_a(x, w, S, e, CH=4, mistake=None, kernel=True):
    """Region A, sum = z S + v e.  The kernel's tables hold entry s as
    (2^(k-s) a_s, 2^(s-k-1) b_s) and it sweeps in x; kernel=False runs the
    unscaled entries in 2x from z = v = 0."""
    k = len(w) - 1
    ent = sweep_entries_a(x, w, CH, mistake)
    if kernel:
        scaled = [(s, math.ldexp(a, k - s), math.ldexp(b, s - k - 1)) for s, a, b in ent]
        z, v = sweep_kernel(x, scaled, mistake)
    else:
        z, v = sweep_plain(x + x, ent, mistake)
    return fma(z, S, rnd(Fraction(v) * Fraction(e)))


def sweep_b(x, w, S, e, CH=4, mistake=None, kernel=True):
    """Region B, sum = z S + (g v) e with g = 1/(2x).  The kernel's tables hold
    entry i as (2^-i a_i, 2^i b_i) and it sweeps in h = 1/x, ending with
    (h v) e; kernel=False runs the unscaled entries in g from z = v = 0."""
    ent = sweep_entries_b(w, CH, mistake)
    if kernel:
        h = rnd(Fraction(1) / Fraction(x))
        scaled = [(i, math.ldexp(a, -i), math.ldexp(b, i)) for i, a, b in ent]
        z, v = sweep_kernel(h, scaled, mistake)
        m = h
    else:
        g = rnd(Fraction(1) / (2 * Fraction(x)))
        z, v = sweep_plain(g, ent, mistake)
        m = g
    return fma(z, S, rnd(Fraction(rnd(Fraction(m) * Fraction(v))) * Fraction(e)))


def exact_F(x, K):
    """F_0..F_K(x) from mpmath's incomplete gamma (50 digits)."""
    mp.mp.dps = 50
    xm = mp.mpf(x)
    return [mp.gammainc(l + mp.mpf(1) / 2, 0, xm) / (2 * xm ** (l + mp.mpf(1) / 2)) for l in range(K + 1)]


def sweep_cases():
    rng = np.random.default_rng(2024)
    cases = []
    for K in range(33):
        cases.append((K, float(rng.uniform(0.05, X0)), "A"))
        cases.append((K, float(rng.uniform(X0, X1)), "B"))
    cases += [(32, float(np.nextafter(X0, 0)), "A"), (32, X0, "B"), (32, X1, "B"), (5, 1e-3, "A")]
    return cases


def check_sweeps(mistake=None, CH=4):
    rng = np.random.default_rng(7)
    u = 2.0 ** -53
    for K, x, region in sweep_cases():
        w = [float(v) for v in rng.standard_normal(K + 1)]
        F = exact_F(x, K)
        exact = sum(mp.mpf(wl) * Fl for wl, Fl in zip(w, F))
        e = mp.exp(-mp.mpf(x))
        if region == "A":
            got = sweep_a(x, w, float(F[K]), float(e), CH, mistake)
            scale = sum(abs(wl) * Fl for wl, Fl in zip(w, F))
        else:
            got = sweep_b(x, w, float(F[0]), float(e), CH, mistake)
            scale = F[0] * sum(abs(wl) for wl in w)
        bound = 4 * (K + 2) * u * scale
        assert abs(mp.mpf(got) - exact) <= bound, (K, x, region, float(abs(mp.mpf(got) - exact) / scale))


@pytest.mark.parametrize("CH", [4, 8])
def test_weight_sweeps_reproduce_the_weighted_sum(CH):
    check_sweeps(CH=CH)


@pytest.mark.parametrize("mistake", ["no_scale", "new_z", "sign", "shift"])
def test_weight_sweep_check_detects_planted_mistakes(mistake):
    with pytest.raises(AssertionError):
        check_sweeps(mistake=mistake)


@pytest.mark.parametrize("CH", [4, 8])
def test_scaled_peeled_sweeps_round_like_the_plain_recurrence(CH):
    """The kernel's form (power-of-two-scaled entries swept in x or 1/x, the
    first step taken as z = a_0 and the second's v formed by a multiply)
    gives the same double as the plain sweep in 2x or 1/(2x) from z = v = 0,
    for every case and order: scaling by a power of two commutes with
    rounding, and the first steps are exact."""
    rng = np.random.default_rng(8)
    for K, x, region in sweep_cases():
        w = [float(v) for v in rng.standard_normal(K + 1)]
        S, e = float(rng.uniform(0.1, 1.0)), float(rng.uniform(1e-13, 1.0))
        f = sweep_a if region == "A" else sweep_b
        assert f(x, w, S, e, CH) == f(x, w, S, e, CH, kernel=False), (K, x, region)
