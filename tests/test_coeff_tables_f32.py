"""The FP32 coefficient tables (own rational Remez) against the mathematics (CPU).

Checks: the region constants against the paper's two region equations at
kmax = 16; each stored approximant equioscillates (N = n+m+2 alternating
extrema of equal weighted error, the characterisation of Sec. II A) and is
within its levelled error everywhere; the header holds the stored values;
the degree choice is the first feasible anti-diagonal of the Walsh table
(spot check); and an emulation of the kernel's FP32/FP64 arithmetic stays
within 1e-6 of the oracle on dense grids of FP32 arguments in every region.
"""
import json
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
from tests.coeff_header import CSRC, _defines, _nested

REC = json.load(open(os.path.join(CSRC, "boys_coeffs_f32.json")))
D = _defines(os.path.join(CSRC, "boys_coeffs_f32.h"))
F32 = np.float32
TOL = 1e-6
KMAX = 16
X0F = F32(float.fromhex(D["BOYS_F32_X0"].rstrip("f")))
X1F = F32(float.fromhex(D["BOYS_F32_X1"].rstrip("f")))


def hexlist(s):
    s = s.strip().strip("{}")
    return [float.fromhex(v.strip().rstrip("f")) if "0x" in v else float(v)
            for v in s.split(",") if v.strip()]


def header_tables():
    text = D["BOYS_F32_RA_P_INIT"]
    import re
    rowsP = [hexlist(r) for r in re.findall(r"\{([^{}]*)\}", text.strip()[1:-1])]
    rowsQ = [hexlist(r) for r in re.findall(r"\{([^{}]*)\}", D["BOYS_F32_RA_Q_INIT"].strip()[1:-1])]
    degn = [int(v) for v in _nested(D["BOYS_F32_RA_DEG_N_INIT"])]
    degm = [int(v) for v in _nested(D["BOYS_F32_RA_DEG_M_INIT"])]
    ra = [(np.array(rowsP[k][:degn[k] + 1], F32), np.array(rowsQ[k][:degm[k] + 1], F32))
          for k in range(KMAX + 1)]
    rb = (hexlist(D["BOYS_F32_RB_P_INIT"]), hexlist(D["BOYS_F32_RB_Q_INIT"]))
    return ra, rb


RA, RB = header_tables()


def rho_a(k, x):
    x = np.asarray(x, dtype=np.longdouble)
    best = np.ones_like(x)
    prod = np.ones_like(x)
    for n in range(k - 1, -1, -1):
        prod = prod * x / (n + 0.5)
        best = np.maximum(best, prod)
    return best


def test_region_constants():
    mp.mp.dps = 40
    p = mp.mpf(1)
    for n in range(KMAX):
        p *= n + mp.mpf(1) / 2
    x0 = p ** (mp.mpf(1) / KMAX)
    assert X0F == F32(float(x0))
    s = KMAX + mp.mpf(1) / 2
    err = lambda x: mp.gammainc(s, mp.mpf(float(x))) / (2 * mp.mpf(float(x)) ** s)
    eps_c = REC["eps_c"]
    assert err(X1F) <= eps_c < err(np.nextafter(X1F, F32(0)))


def test_header_matches_record():
    for k in range(KMAX + 1):
        t = REC["region_a"][k]
        assert list(RA[k][0].astype(float)) == t["p_f32"] and list(RA[k][1].astype(float)) == t["q_f32"]
    assert RB[0] == REC["region_b"]["p_f64"] and RB[1] == REC["region_b"]["q_f64"]


def _mp_eval(c, x):
    return mp.polyval([mp.mpf(v) for v in c][::-1], x)


@pytest.mark.parametrize("k", list(range(KMAX + 1)) + ["B"])
def test_equioscillation(k):
    """Exact coefficients: the weighted error takes alternating signs and equal
    magnitude E (to 1%) at the N = n+m+2 stored nodes, and |weighted error|
    <= 1.001 E on a dense grid (so r is the minimax approximation)."""
    mp.mp.dps = 40
    t = REC["region_b"] if k == "B" else REC["region_a"][k]
    order = 0 if k == "B" else k
    lo, hi = (REC["x0_f32"], REC["x1_f32"]) if k == "B" else (0.0, REC["x0_f32"])
    nodes = np.array(t["nodes"])
    assert nodes.size == t["n"] + t["m"] + 2
    F = oracle.boys_ld(nodes, order)[:, order]
    w = np.ones(nodes.size) if k == "B" else rho_a(order, nodes)
    e = [float(mp.mpf(float(w[i])) * (mp.mpf(np.format_float_scientific(F[i], 25)) -
                                      _mp_eval(t["p"], mp.mpf(nodes[i])) / _mp_eval(t["q"], mp.mpf(nodes[i]))))
         for i in range(nodes.size)]
    e = np.array(e)
    assert np.all(np.sign(e[1:]) == -np.sign(e[:-1])), "no alternation"
    assert np.allclose(np.abs(e), t["E"], rtol=1e-2), (np.abs(e) / t["E"])
    xs = np.linspace(lo, hi, 4001)
    Fx = oracle.boys_ld(xs, order)[:, order]
    wx = np.ones(xs.size) if k == "B" else rho_a(order, xs)
    pv = np.polynomial.polynomial.polyval(xs, [float(v) for v in t["p"]])
    qv = np.polynomial.polynomial.polyval(xs, [float(v) for v in t["q"]])
    assert np.max(np.abs(wx * (Fx - pv / qv))) <= t["E"] * 1.001 + 1e-15


def test_walsh_choice_is_first_feasible_antidiagonal():
    """For r'_{A,16} and r'_B no entry of the previous anti-diagonal meets the
    target (spot check of the degree choice of Sec. II D)."""
    from paper_2512_10059_amd import remez
    for f, rho, a, b, t, target in (
            (remez.boys_k(16), remez.rho_a(16), 0.0, REC["x0_f32"], REC["region_a"][16], REC["eps_a"]),
            (remez.boys_k(0), remez.rho_one, REC["x0_f32"], REC["x1_f32"], REC["region_b"], REC["eps_b"])):
        d = t["n"] + t["m"] - 1
        for m in range(d + 1):
            try:
                r = remez.remez(f, rho, a, b, d - m, m, tol=1e-4, dps=30)
            except remez.RemezFailure:
                continue
            assert r.E > target, f"({d - m},{m}) already meets {target}"


# ---------------------------------------------------------------------------
# Emulation of the kernel arithmetic.

def fma32(a, b, c):
    return (np.float64(a) * np.float64(b) + np.float64(c)).astype(F32)


def emulate(x, K):
    """The FP32 kernel's arithmetic on FP32 arguments x (all in the domain)."""
    x = x.astype(F32)
    out = np.empty((x.size, K + 1), F32)
    A = x < X0F
    C = x >= X1F
    B = ~A & ~C
    if A.any():
        xa = x[A]
        p_, q_ = RA[K]
        p = np.full(xa.shape, p_[-1], F32)
        for c in p_[-2::-1]:
            p = fma32(p, xa, c)
        q = (xa + q_[-2]).astype(F32)
        for c in q_[-3::-1]:
            q = fma32(q, xa, c)
        Fa = np.empty((xa.size, K + 1), F32)
        Fa[:, K] = p / q
        e = np.exp(-xa).astype(F32)
        tx = (xa + xa).astype(F32)
        for l in range(K - 1, -1, -1):
            Fa[:, l] = (fma32(tx, Fa[:, l + 1], e) * F32(1.0 / (2 * l + 1))).astype(F32)
        out[A] = Fa
    if B.any():
        xb = x[B].astype(np.float64)
        p = np.polynomial.polynomial.polyval(xb, RB[0])
        q = np.polynomial.polynomial.polyval(xb, RB[1])
        f = p / q
        e = np.exp(-xb)
        inv = 0.5 / xb
        Fb = np.empty((xb.size, K + 1), F32)
        Fb[:, 0] = f
        for l in range(K):
            f = ((2 * l + 1) * f - e) * inv
            Fb[:, l + 1] = f
        out[B] = Fb
    if C.any():
        xc = x[C]
        inv = (F32(0.5) / xc).astype(F32)
        f = (F32(0.886226925452758) / np.sqrt(xc)).astype(F32)
        Fc = np.empty((xc.size, K + 1), F32)
        Fc[:, 0] = f
        for l in range(K):
            f = ((F32(2 * l + 1) * f).astype(F32) * inv).astype(F32)
            Fc[:, l + 1] = f
        out[C] = Fc
    return out


def dense_f32(lo, hi, n):
    g = np.unique(np.linspace(lo, hi, n).astype(F32))
    return g[(g >= F32(lo)) & (g < F32(hi))]


@pytest.mark.parametrize("K", [0, 1, 2, 5, 8, 12, 15, 16])
def test_emulated_fp32_path_within_1e6(K):
    xs = np.concatenate([dense_f32(0, float(X0F), 6000), [np.nextafter(X0F, F32(0))],
                         dense_f32(float(X0F), float(X1F), 6000), [X0F, X1F],
                         np.geomspace(float(X1F), 1e5, 3000).astype(F32)])
    got = emulate(xs, K).astype(np.float64)
    ref = oracle.boys(xs.astype(np.float64), K)
    err = np.abs(got - ref)
    assert err.max() <= TOL, f"K={K}: {err.max():.3e}"


def test_package_reads_the_fp32_region_bounds():
    """The host helper that splits reported errors by region reads the same
    x0' and x1' as the kernels compile in."""
    from paper_2512_10059_amd.tables import f32_region_bounds
    x0, x1 = f32_region_bounds()
    assert F32(x0) == X0F and F32(x1) == X1F and x0 == float(X0F) and x1 == float(X1F)
