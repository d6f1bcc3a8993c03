"""The offline Remez tool against the paper's own tables and known facts (CPU).

* Run on the paper's setting for r_B (F_0 on [x0, x1], weight 1, degrees
  (5,6)), it lands within 1e-16 of the printed r_B everywhere on the
  interval (the printed table's own error is 9.44e-15), i.e. it reproduces
  the appendix approximant in function space.
* Run for r_{A,26} with the paper's weight rho_{A,26}, it finds a weighted
  error no larger than the printed table's (the paper's Remez stops once
  below eps_tol, so its tables need not be the exact minimax).
* The result equioscillates: n+m+2 alternating extrema of equal size.
* Region constants: x0(32) and x1(32, 5e-14) reproduce the printed values.
* The tool's reference values agree with the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2512_10059_amd import remez
from tests.coeff_header import load_f64

T = load_f64()
LD = np.longdouble


def polyval(c, x):
    return remez.polyval_ld([LD(v) for v in c], x)


def test_reproduces_printed_rB():
    r = remez.remez(remez.boys_k(0), remez.rho_one, T["x0"], T["x1"], 5, 6, tol=1e-5)
    assert r.converged
    x = np.linspace(T["x0"], T["x1"], 20001).astype(LD)
    paper = polyval(T["rb"][0], x) / polyval(T["rb"][1], x)
    assert float(np.max(np.abs(r(x) - paper))) <= 1e-16
    assert abs(r.E - 9.43e-15) <= 0.01e-15


def test_rA26_not_worse_than_printed():
    k = 26
    n, m = len(T["ra"][k][0]) - 1, len(T["ra"][k][1]) - 1
    r = remez.remez(remez.boys_k(k), remez.rho_a(k), 0.0, T["x0"], n, m, tol=1e-4)
    x = np.linspace(0, T["x0"], 20001).astype(LD)
    w = remez.rho_a(k)(x)
    f = remez.boys_k(k)(x)
    paper = float(np.max(w * np.abs(f - polyval(T["ra"][k][0], x) / polyval(T["ra"][k][1], x))))
    ours = float(np.max(w * np.abs(f - r(x))))
    assert ours <= paper <= 5e-14
    # de la Vallee-Poussin: the printed approximant's error at our nodes
    # alternates, so its smallest node error bounds the minimax error below.
    nodes = np.array(r.nodes, dtype=LD)
    e_p = remez.rho_a(k)(nodes) * (remez.boys_k(k)(nodes) - polyval(T["ra"][k][0], nodes) /
                                   polyval(T["ra"][k][1], nodes))
    assert float(np.min(np.abs(e_p))) <= r.E * 1.001


def test_equioscillation_of_result():
    r = remez.remez(remez.boys_k(3), remez.rho_a(3), 0.0, 6.0, 3, 3, tol=1e-6)
    nodes = np.array(r.nodes, dtype=LD)
    e = remez.rho_a(3)(nodes) * (remez.boys_k(3)(nodes) - r(nodes))
    assert nodes.size == 8
    assert np.all(np.sign(e[1:]) == -np.sign(e[:-1]))
    assert np.allclose(np.abs(e).astype(float), r.E, rtol=1e-4)


def test_early_abort_when_target_unreachable():
    with pytest.raises(remez.RemezFailure):
        remez.remez(remez.boys_k(0), remez.rho_one, T["x0"], T["x1"], 1, 1, target=1e-12)


def test_region_constants_reproduce_paper():
    assert remez.region_x0(32) == pytest.approx(T["x0"], rel=1e-15)
    assert remez.region_x1(32, 5e-14, 29.0) == pytest.approx(T["x1"], rel=1e-15)
    assert remez.region_x0(0) == 1.0 and remez.region_x0(1) == 1.0


def test_reference_values_match_oracle():
    x = np.concatenate([[0.0], np.geomspace(1e-9, 40.0, 300)])
    F = remez.boys_series(x.astype(LD), 20)
    ref = oracle.boys_ld(x, 20)
    assert float(np.max(np.abs(F - ref) / ref)) <= 1e-17


def test_weight_matches_definition():
    """rho_{A,k}(x) = max_l prod_{n=l}^{k-1} x/(n+1/2), 1 for the empty product."""
    x = np.array([0.0, 0.3, 2.0, 7.5, 11.0], dtype=LD)
    k = 6
    direct = []
    for xv in x:
        vals = [1.0]
        for l in range(k):
            vals.append(float(np.prod([xv / (n + 0.5) for n in range(l, k)])))
        direct.append(max(vals))
    assert np.allclose(remez.rho_a(k)(x).astype(float), direct, rtol=1e-15)


@pytest.mark.parametrize("which,k", [("B", 0), ("A", 26)])
def test_walsh_walk_reproduces_printed_degrees(which, k):
    """The degree choice of Sec. II D (first anti-diagonal n+m with an entry
    meeting 5e-14, smallest error on it), run with this Remez, lands on the
    degrees the appendix prints: (5,6) for r_B, (7,8) for r_{A,26}."""
    f = remez.boys_k(0 if which == "B" else k)
    rho = remez.rho_one if which == "B" else remez.rho_a(k)
    a, b = (T["x0"], T["x1"]) if which == "B" else (0.0, T["x0"])
    p, q = T["rb"] if which == "B" else T["ra"][k]
    printed = (len(p) - 1, len(q) - 1)
    r = remez.walsh_search(f, rho, a, b, 5e-14, d_min=sum(printed) - 1, d_max=sum(printed),
                           tol=1e-3, dps=40, max_iter=30)
    assert (r.n, r.m) == printed
