"""Pins that tie the CPU oracle to facts fixed outside it.

Each check takes an :class:`oracle.OracleLib` and raises AssertionError when
the oracle disagrees with the fact it pins.  The facts are independent of the
oracle's own arithmetic:

* mpmath's incomplete gamma function at 40 digits, through
  F_k(x) = gamma(k+1/2, x) / (2 x^(k+1/2)) (the asymptotic form of Sec. II C
  and its exact error are this identity split in two);
* mpmath's erf through F_0(x) = 1/2 sqrt(pi/x) erf(sqrt x);
* numerical quadrature of the defining integral (Sec. I, eq. 3);
* F_k(0) = 1/(2k+1), read off eq. 3;
* the asymptote Gamma(k+1/2)/(2x^(k+1/2)) and its exact error (Sec. II C);
* the two recurrences (Sec. II C) between values the oracle computes along
  different routes (series at another order, the other branch);
* dF_k/dx = -F_{k+1} and monotonicity in x and in k, both from eq. 3.

``tests/test_oracle_pins.py`` runs them on the oracle; ``tests/
test_oracle_mutants.py`` runs them on deliberately broken builds of it and
requires each break to be caught.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

mp.mp.dps = 40
HALF = mp.mpf(1) / 2

# Arguments chosen to cover the oracle's two branches (series up to 30, erf
# plus upward recurrence above), the method's region boundaries and the tails.
X_GRID = [1e-12, 1e-6, 1e-3, 0.05, 0.5, 1.0, 2.5, 5.0, 8.0, 11.899848152108484, 15.0,
          20.0, 25.0, 28.98933773882074, 29.5, 30.0, 30.5, 35.0, 50.0, 100.0, 1e3, 1e4, 3e5]
K_GRID = [0, 1, 2, 3, 5, 8, 13, 16, 17, 26, 32, 33, 40]
KMAX = 40


def ld_to_mp(v) -> mp.mpf:
    """Exact value of a long double as an mpmath number."""
    m, e = np.frexp(np.longdouble(v))
    return mp.ldexp(mp.mpf(int(np.longdouble(m) * np.longdouble(2.0) ** 64)), int(e) - 64)


def boys_mp(k: int, x: float) -> mp.mpf:
    """F_k(x) from mpmath's lower incomplete gamma function."""
    x = mp.mpf(x)
    if x == 0:
        return mp.mpf(1) / (2 * k + 1)
    a = k + HALF
    return mp.gammainc(a, 0, x) / (2 * x ** a)


def _rel(a, b):
    b = mp.mpf(b)
    return abs(mp.mpf(a) - b) / abs(b) if b != 0 else abs(mp.mpf(a))


def check_gammainc(o, tol=2e-17):
    """Every F_k on the grid, both from the order-KMAX evaluation (downward or
    upward recurrence) and from the evaluation at order k itself."""
    x = np.array(X_GRID)
    Fall = o.boys_ld(x, KMAX)
    for k in K_GRID:
        Fk = o.boys_ld(x, k)
        for i, xv in enumerate(X_GRID):
            ref = boys_mp(k, xv)
            for src, val in (("kmax=40", Fall[i, k]), (f"kmax={k}", Fk[i, k])):
                err = _rel(ld_to_mp(val), ref)
                assert err <= tol, f"F_{k}({xv}) [{src}] rel err {mp.nstr(err, 3)}"


def check_erf_closed_form(o, tol=2e-18):
    xs = [1e-9, 0.1, 1.0, 3.0, 10.0, 29.999, 30.001, 60.0, 1e4]
    for kmax in (0, 17, KMAX):
        F = o.boys_ld(np.array(xs), kmax)
        for i, xv in enumerate(xs):
            xm = mp.mpf(xv)
            ref = HALF * mp.sqrt(mp.pi / xm) * mp.erf(mp.sqrt(xm))
            err = _rel(ld_to_mp(F[i, 0]), ref)
            assert err <= tol, f"F_0({xv}) at kmax={kmax}: rel err {mp.nstr(err, 3)}"


def check_value_at_zero(o):
    F = o.boys_ld(np.array([0.0, -0.0]), KMAX)
    for k in range(KMAX + 1):
        for row in F:
            err = _rel(ld_to_mp(row[k]), mp.mpf(1) / (2 * k + 1))
            assert err <= 2e-19, f"F_{k}(0) rel err {mp.nstr(err, 3)}"


def check_quadrature(o, tol=2e-17):
    """Numerical quadrature (mpmath, tanh-sinh, 40 digits) of the defining
    integral t^(2k) exp(-x t^2) over [0, 1]."""
    xs = [0.0, 1e-4, 0.3, 1.7, 6.0, 11.9, 19.0, 29.0, 31.0, 45.0, 60.0]
    F = o.boys_ld(np.array(xs), KMAX)
    for k in range(0, KMAX + 1, 3):
        for i, xv in enumerate(xs):
            xm = mp.mpf(xv)
            q = mp.quad(lambda t: t ** (2 * k) * mp.exp(-xm * t * t), [0, 1])
            err = _rel(ld_to_mp(F[i, k]), q)
            assert err <= tol, f"F_{k}({xv}) quadrature rel err {mp.nstr(err, 3)}"


def check_recurrences(o):
    """Values computed along different routes satisfy both recurrences:
    F_K from the series at order K equals F_K recurred down from order KMAX
    (x <= 30), and the erf-plus-upward values (x > 30) satisfy the downward
    recurrence F_k = (2x F_{k+1} + e^-x)/(2k+1)."""
    xs = np.array([1e-8, 0.25, 3.0, 9.0, 17.0, 24.0, 29.99])
    Fall = o.boys_ld(xs, KMAX)
    for K in (0, 1, 7, 20, 33):
        FK = o.boys_ld(xs, K)
        for i in range(xs.size):
            err = _rel(ld_to_mp(FK[i, K]), ld_to_mp(Fall[i, K]))
            assert err <= 1e-17, f"x={xs[i]} F_{K}: series vs recurred rel {mp.nstr(err, 3)}"
    xs = np.array([30.01, 33.0, 41.0, 77.0, 500.0])
    F = o.boys_ld(xs, KMAX)
    for i, xv in enumerate(xs):
        xm = mp.mpf(xv)
        e = mp.exp(-xm)
        for k in range(KMAX):
            lhs = ld_to_mp(F[i, k])
            rhs = (2 * xm * ld_to_mp(F[i, k + 1]) + e) / (2 * k + 1)
            assert _rel(rhs, lhs) <= 1e-17, f"downward identity x={xv} k={k}"


def check_asymptote(o):
    """For large x, Gamma(k+1/2)/(2 x^(k+1/2)) - F_k(x) equals the upper
    incomplete gamma Gamma(k+1/2, x)/(2 x^(k+1/2)) and is positive."""
    xs = [28.98933773882074, 30.0, 35.0, 50.0, 100.0, 1e3]
    F = o.boys_ld(np.array(xs), 32)
    for k in (0, 8, 16, 32):
        a = k + HALF
        prev = None
        for i, xv in enumerate(xs):
            xm = mp.mpf(xv)
            asym = mp.gamma(a) / (2 * xm ** a)
            gap = asym - ld_to_mp(F[i, k])
            exact = mp.gammainc(a, xm) / (2 * xm ** a)
            assert abs(gap - exact) <= 2e-17 * asym, \
                f"asymptote error F_{k}({xv}): {mp.nstr(gap, 5)} vs {mp.nstr(exact, 5)}"
            if exact > 1e-15 * asym:      # gap resolvable in long double
                assert gap > 0, f"asymptote below F_{k}({xv})"
                assert prev is None or gap < prev
                prev = gap


def check_monotone_and_bounds(o):
    xs = np.unique(np.concatenate([np.geomspace(1e-8, 1e5, 220), np.linspace(0.0, 40.0, 161)]))
    F = o.boys_ld(xs, KMAX)
    assert np.all(np.diff(F, axis=0) < 0), "F_k not decreasing in x"
    assert np.all(np.diff(F, axis=1) < 0), "F_k not decreasing in k"
    k = np.arange(KMAX + 1, dtype=np.longdouble)
    xl = xs.astype(np.longdouble)[:, None]
    lower = np.exp(-xl) / (2 * k + 1)
    upper = 1 / (2 * k + 1)
    assert np.all(F >= lower * (1 - 1e-18)), "F_k below exp(-x)/(2k+1)"
    assert np.all(F <= upper * (1 + 1e-18) + 0 * xl), "F_k above 1/(2k+1)"


def check_derivative(o, rel_step=1e-7):
    """Central difference of F_k in long double against -F_{k+1}."""
    xs = np.array([1e-3, 0.7, 4.0, 11.9, 22.0, 29.9, 30.1, 64.0], dtype=np.longdouble)
    K = 20
    h = np.longdouble(rel_step) * np.maximum(np.longdouble(1), xs)
    Fp = o.boys_ld(xs + h, K + 1)
    Fm = o.boys_ld(xs - h, K + 1)
    F0 = o.boys_ld(xs, K + 1)
    d = (Fp - Fm) / (2 * h)[:, None]
    err = np.abs(d[:, :K + 1] + F0[:, 1:]) / F0[:, 1:]
    assert float(err.max()) <= 1e-9, f"dF/dx vs -F_(k+1): max rel {float(err.max())}"


def check_branch_continuity(o):
    """The series (x <= 30) and erf-plus-upward (x > 30) branches meet."""
    x0 = np.longdouble(30.0)
    xs = np.array([x0, np.nextafter(x0, np.longdouble(np.inf))])
    F = o.boys_ld(xs, KMAX)
    rel = np.abs(F[1] - F[0]) / F[0]
    assert float(rel.max()) <= 1e-17, f"branch jump at 30: {float(rel.max())}"


def _at_40_digits(check):
    """Runs a check with mpmath at 40 digits, whatever precision other code in
    the process left set."""
    @functools.wraps(check)
    def run(o, *args, **kwargs):
        with mp.workdps(40):
            return check(o, *args, **kwargs)
    return run


ALL_CHECKS = [_at_40_digits(c) for c in (
    check_value_at_zero, check_erf_closed_form, check_gammainc, check_quadrature,
    check_recurrences, check_asymptote, check_monotone_and_bounds, check_derivative,
    check_branch_continuity)]
