"""The FP64 coefficient tables of the GPU library against the paper and the
mathematics (CPU only).

The tables are the paper's appendix (eps_tol = 5e-14, kmax = 32).  These
tests check them three ways: a few printed entries and the printed degrees;
the region constants against their defining equations (Sec. II C: x0 from the
stability of upward recurrence, x1 from the asymptote's error); and the
approximants themselves, evaluated in float64 the way Algorithm 1 does,
against the oracle on dense grids, to the guaranteed 5e-14.
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from tests.coeff_header import load_f64

EPS_TOL = 5e-14
T = load_f64()
X0, X1 = T["x0"], T["x1"]


def horner(c, x):
    r = np.zeros_like(x) + c[-1]
    for a in c[-2::-1]:
        r = r * x + a
    return r


def test_printed_entries_and_degrees():
    # Degrees (numerator, denominator) as printed in the appendix tables.
    printed = {0: (6, 9), 1: (6, 10), 2: (6, 10), 3: (4, 12), 4: (8, 9), 5: (4, 13), 6: (8, 9),
               7: (4, 13), 18: (8, 8), 19: (8, 8), 20: (7, 9), 25: (8, 8), 26: (7, 8), 32: (7, 8)}
    printed.update({k: (8, 9) for k in range(8, 18)})
    for k, (n, m) in printed.items():
        p, q = T["ra"][k]
        assert (len(p) - 1, len(q) - 1) == (n, m), k
        assert q[-1] == 1.0
    assert (len(T["rb"][0]) - 1, len(T["rb"][1]) - 1) == (5, 6)
    # A few entries copied from the tables for r_B, r_{A,0} and r_{A,32}.
    assert T["rb"][0][0] == 5.74537531702047552E+07
    assert T["rb"][1][2] == -1.66693114610725015E+06
    assert T["ra"][0][1][0] == 4.59649054199579770E+11
    assert T["ra"][32][1][7] == 3.14246148951811622E+01
    assert T["ra"][32][0][7] == -1.07813149210223792E-03


def test_x0_from_its_equation():
    """x0 = max{1, (prod_{n<kmax} (n+1/2))^(1/kmax)} with kmax = 32 (Sec. II C)."""
    mp.mp.dps = 40
    p = mp.mpf(1)
    for n in range(32):
        p *= n + mp.mpf(1) / 2
    assert float(max(mp.mpf(1), p ** (mp.mpf(1) / 32))) == X0


def test_x1_from_its_equation():
    """x1 solves Gamma(kmax+1/2, x1) / (2 x1^(kmax+1/2)) = eps_tol (Sec. II C).

    The printed x1 is the double nearest the root but just below it, so at
    that double the asymptote misses eps_tol for F_32 by 8e-30; the next
    double meets it.  The GPU kernels therefore start region C just above the
    printed x1 (x > x1) and evaluate x = x1 itself in region B."""
    mp.mp.dps = 40
    a = 32 + mp.mpf(1) / 2
    err = lambda x: mp.gammainc(a, mp.mpf(x)) / (2 * mp.mpf(x) ** a)
    root = mp.findroot(lambda x: err(x) - mp.mpf(EPS_TOL), 29)
    assert float(root) == X1
    assert err(X1) > EPS_TOL
    assert err(np.nextafter(X1, 100.0)) <= EPS_TOL


def _grid(lo, hi, n):
    g = np.concatenate([np.linspace(lo, hi, n), lo + (hi - lo) * np.geomspace(1e-12, 1e-2, 200)])
    g = np.concatenate([g, [np.nextafter(hi, -1.0)]])
    return np.unique(g[(g >= lo) & (g <= hi)])


@pytest.fixture(scope="module")
def grid_A():
    x = _grid(0.0, X0, 4000)
    x = x[x < X0]
    return x, oracle.boys(x, 32)


@pytest.mark.parametrize("k", range(33))
def test_region_A_table(k, grid_A):
    """r_{A,k} then downward recurrence in float64 meets 5e-14 for every l <= k on [0, x0)."""
    x, F = grid_A
    p, q = T["ra"][k]
    y = np.empty((x.size, k + 1))
    y[:, k] = horner(p, x) / horner(q, x)
    e = np.exp(-x)
    for l in range(k - 1, -1, -1):
        y[:, l] = (2 * x * y[:, l + 1] + e) / (2 * l + 1)
    err = np.abs(y - F[:, :k + 1]).max()
    assert err <= EPS_TOL, f"k={k}: max abs error {err:.3e}"


def test_region_B_table():
    """r_B then upward recurrence to F_32 meets 5e-14 on [x0, x1]."""
    x = _grid(X0, X1, 6000)
    F = oracle.boys(x, 32)
    p, q = T["rb"]
    y = np.empty((x.size, 33))
    y[:, 0] = horner(p, x) / horner(q, x)
    e = np.exp(-x)
    for l in range(32):
        y[:, l + 1] = ((2 * l + 1) * y[:, l] - e) / (2 * x)
    err = np.abs(y - F).max()
    assert err <= EPS_TOL, f"max abs error {err:.3e}"


def test_region_C_asymptote():
    """The asymptote F_0 = sqrt(pi)/(2 sqrt x), F_{l+1} = (l+1/2)/x F_l meets
    5e-14 for every l <= 32 on (x1, inf)."""
    x = np.unique(np.concatenate([np.nextafter(X1, 100.0) + np.arange(50) * 4e-15,
                                  np.geomspace(np.nextafter(X1, 100.0), 1e6, 3000)]))
    F = oracle.boys(x, 32)
    y = np.empty((x.size, 33))
    y[:, 0] = np.sqrt(np.pi) / 2 / np.sqrt(x)
    for l in range(32):
        y[:, l + 1] = y[:, l] * (l + 0.5) / x
    err = np.abs(y - F).max()
    assert err <= EPS_TOL, f"max abs error {err:.3e}"
