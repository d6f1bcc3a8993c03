"""The single approximant for F_0 on [x0, inf) found by
csrc/single_region_fp64.py (the branch-free alternative of Sec. II A, with
the x^(-1/2) factor taken out and s = x0/x), pinned against the oracle:

* F_0(x) = x^(-1/2) p(s)/q(s) with its coefficients rounded to double is
  within the fitting target 4.9e-14 of the oracle from x0 to 1e15 (dense
  and logarithmic grids, and both ends);
* the fit itself (its 30-digit coefficients) equioscillates on n+m+2 points
  of the weighted error in s, at the level it reports;
* q has no zero on [0, 1];
* evaluated in float64 (rsqrt-free: 1/sqrt(x), Horner, one division), the
  approximant stays within 5e-14;
* the checks fail for a perturbed coefficient."""
import json
import os

import numpy as np

import oracle
from tests.coeff_header import CSRC
from tests.test_coeff_tables_sets import LD, alternations, horner_ld

REC = json.load(open(os.path.join(CSRC, "single_region_fp64.json")))
X0 = REC["x0"]


def grid():
    return np.unique(np.concatenate([np.linspace(X0, 60.0, 6001), np.geomspace(60.0, 1e15, 3001),
                                     [X0, np.nextafter(X0, np.inf), 1e15]]))


def approx_ld(p, q, x):
    x = np.asarray(x, dtype=LD)
    s = LD(X0) / x
    return horner_ld(p, s) / horner_ld(q, s) / np.sqrt(x)


def test_record_is_the_first_feasible_entry():
    assert (REC["n"], REC["m"]) == (11, 2) and REC["anti_diagonal"] == 13
    assert [REC["n"], REC["m"]] in REC["feasible"]
    assert REC["double_err"] <= REC["target"] == 4.9e-14
    assert REC["q"][-1] == 1.0


def test_within_target_against_the_oracle():
    x = grid()
    err = np.abs(approx_ld(REC["p"], REC["q"], x) - oracle.boys_ld(x.astype(LD), 0)[:, 0])
    assert float(err.max()) <= REC["target"], float(err.max())


def test_fit_equioscillates():
    p = [LD(c) for c in REC["p_ext"]]
    q = [LD(c) for c in REC["q_ext"]]
    s = np.linspace(LD(1e-6), LD(1), 20001, dtype=LD)
    x = LD(X0) / s
    e = np.sqrt(s / LD(X0)) * (oracle.boys_ld(x, 0)[:, 0] * np.sqrt(x) - horner_ld(p, s) / horner_ld(q, s))
    E = float(np.max(np.abs(e)))
    assert E <= 1.01 * REC["E"]
    assert alternations(e.astype(float), 0.97 * E) >= REC["n"] + REC["m"] + 2


def test_denominator_has_no_zero_on_the_interval():
    q = np.array(REC["q"][::-1])
    roots = np.roots(q)
    real = roots[np.abs(roots.imag) < 1e-12].real
    assert not np.any((real >= 0.0) & (real <= 1.0)), roots


def test_float64_evaluation_within_eps():
    x = grid()
    s = X0 / x
    r = np.polyval(np.array(REC["p"])[::-1], s) / np.polyval(np.array(REC["q"])[::-1], s)
    F0 = r / np.sqrt(x)
    assert np.abs(F0 - oracle.boys(x, 0)[:, 0]).max() <= 5e-14


def test_checks_detect_a_perturbed_coefficient():
    p = list(REC["p"])
    p[2] *= 1 + 1e-9
    x = grid()
    err = np.abs(approx_ld(p, REC["q"], x) - oracle.boys_ld(x.astype(LD), 0)[:, 0])
    assert float(err.max()) > REC["target"]
