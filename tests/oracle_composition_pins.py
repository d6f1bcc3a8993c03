"""Pins for the quantities the oracle composes from F_k (oracle/__init__.py).

``oracle.weighted_sum``, ``oracle.backward`` / ``backward_ld``,
``oracle.central_difference`` and ``oracle.pairsum`` are checked here against
values built independently of them:

* every F_l(x) comes from mpmath's lower incomplete gamma function at 30
  digits, F_l(x) = gamma(l+1/2, x) / (2 x^(l+1/2)) (Sec. I, eq. 3), never
  from the oracle's own F;
* the weighted sum of Sec. III, Algorithm 2's consumer is then formed in
  mpmath over a hand-made batch table with gaps between batches, an empty
  batch, batches listed out of storage order, weight ranges with unused
  weights between them, and orders 0 and 32;
* the derivative dL/dx = -sum_k G_k F_{k+1} (eq. 3 differentiated under the
  integral sign) is formed in mpmath for the backward pass and for the
  central difference, which must reach it within its O(h^2) truncation;
* the pair sums z_i = sum_l c_l sum_j F_l(x_i + x_j) y_j (Sec. III,
  Algorithm 2) are formed in mpmath for a subset of rows given out of order,
  with pair arguments that land on both sides of x0 and x1;
* identities that need no mpmath: unit weights pick one column of F, the
  backward pass equals the central difference, and pairsum with one weight
  and unit y is a plain row sum of F.

``tests/test_oracle_compositions.py`` runs the checks on the oracle and on
deliberately broken copies of ``oracle/__init__.py`` (a shifted weight
offset, k weights instead of k+1, the wrong column of F, x_i*x_j for
x_i+x_j, ...), and requires every break to be caught.  Each check takes the
oracle module (or a broken copy of it) and raises AssertionError.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

from tests.oracle_pins import ld_to_mp

DPS = 30
HALF = mp.mpf(1) / 2


@functools.lru_cache(maxsize=None)
def _f_mp(k: int, x: float) -> mp.mpf:
    """F_k(x) from mpmath's incomplete gamma function (x as the exact double)."""
    with mp.workdps(DPS):
        xm = mp.mpf(x)
        if xm == 0:
            return mp.mpf(1) / (2 * k + 1)
        a = k + HALF
        return mp.gammainc(a, 0, xm) / (2 * xm ** a)


def _rel_ok(got: float, ref: mp.mpf, scale: mp.mpf, rel: float, what: str):
    """|got - ref| <= rel * scale + one rounding of ref to double."""
    with mp.workdps(DPS):
        err = abs(mp.mpf(float(got)) - ref)
        bound = mp.mpf(rel) * scale + abs(ref) * mp.mpf(2) ** -53
        assert err <= bound, f"{what}: got {got!r}, mpmath {mp.nstr(ref, 20)}, err {mp.nstr(err, 3)}"


# ---------------------------------------------------------------------------
# Weighted sums over a batch table.

# Arguments on both sides of x0 = 11.9 and x1 = 28.99, zero and the tails.
WS_X = np.array([0.0, 1e-9, 0.3, 2.9, 3.1, 6.0, 11.8, 11.899848152108484, 12.0, 20.0,
                 28.9, 28.98933773882074, 29.1, 45.0, 300.0, 1e4, 0.75, 7.5, 17.0, 33.0,
                 1.25, 9.0, 26.0, 60.0])
# Batches (offset, size, order, weight offset), deliberately out of storage
# order: arguments 4-5, 14-15 and 22-23 belong to no batch, batch 3 is empty,
# and the weight ranges leave unused weights between them.
WS_BATCHES = [(16, 6, 1, 3), (0, 4, 0, 0), (6, 5, 32, 6), (4, 0, 5, 41), (11, 3, 7, 48)]
WS_NW = 60


def ws_table():
    rng = np.random.default_rng(2024)
    w = rng.standard_normal(WS_NW)
    off = np.array([b[0] for b in WS_BATCHES], dtype=np.int64)
    n = np.array([b[1] for b in WS_BATCHES], dtype=np.int32)
    k = np.array([b[2] for b in WS_BATCHES], dtype=np.int32)
    wo = np.array([b[3] for b in WS_BATCHES], dtype=np.int64)
    return WS_X.copy(), off, n, k, w, wo


def ws_reference(x, off, n, k, w, wo):
    """(expected value, scale sum_l |w_l F_l|) per argument, in mpmath."""
    ref = [mp.mpf(0)] * x.size
    scale = [mp.mpf(0)] * x.size
    with mp.workdps(DPS):
        for ob, nb, kb, wb in zip(off, n, k, wo):
            for i in range(int(ob), int(ob) + int(nb)):
                terms = [mp.mpf(float(w[int(wb) + l])) * _f_mp(l, float(x[i])) for l in range(int(kb) + 1)]
                ref[i] = mp.fsum(terms)
                scale[i] = mp.fsum(abs(t) for t in terms)
    return ref, scale


def check_weighted_sum_mpmath(o):
    x, off, n, k, w, wo = ws_table()
    got = o.weighted_sum(x, off, n, k, w, wo)
    assert got.shape == x.shape and got.dtype == np.float64
    ref, scale = ws_reference(x, off, n, k, w, wo)
    covered = np.zeros(x.size, bool)
    for ob, nb in zip(off, n):
        covered[int(ob):int(ob) + int(nb)] = True
    for i in range(x.size):
        if covered[i]:
            _rel_ok(got[i], ref[i], scale[i], 1e-17, f"weighted_sum[{i}] (x={x[i]})")
        else:
            assert got[i] == 0.0, f"weighted_sum wrote {got[i]} at argument {i}, outside every batch"


def check_weighted_sum_unit_weights(o):
    """A weight vector e_l selects column l of F (and all-ones weights sum
    the columns), for a single batch of order 32 over every argument."""
    x = WS_X
    K = 32
    F = o.boys(x, K)
    off = np.array([0], np.int64)
    n = np.array([x.size], np.int32)
    k = np.array([K], np.int32)
    wo = np.array([0], np.int64)
    for l in (0, 1, 16, 31, 32):
        w = np.zeros(K + 1)
        w[l] = 1.0
        got = o.weighted_sum(x, off, n, k, w, wo)
        assert np.array_equal(got, F[:, l]), f"unit weight e_{l} does not select column {l}"
    got = o.weighted_sum(x, off, n, k, np.ones(K + 1), wo)
    Fld = o.boys_ld(x, K)
    assert np.allclose(got, Fld.sum(axis=1).astype(np.float64), rtol=4e-16, atol=0), "all-ones weights"


# ---------------------------------------------------------------------------
# Backward pass and central difference.

BW_X = np.array([0.0, 2e-7, 0.4, 3.0, 9.5, 11.899848152108484, 17.25, 28.98933773882074,
                 29.5, 42.0, 250.0, 5e3])


def bw_inputs(K: int):
    rng = np.random.default_rng(100 + K)
    return BW_X.copy(), rng.standard_normal((BW_X.size, K + 1))


def bw_reference(x, G):
    """-sum_k G_k F_{k+1}(x) and sum_k |G_k| F_{k+1}(x), per argument, in mpmath."""
    K = G.shape[1] - 1
    ref, scale = [], []
    with mp.workdps(DPS):
        for i in range(x.size):
            t = [mp.mpf(float(G[i, kk])) * _f_mp(kk + 1, float(x[i])) for kk in range(K + 1)]
            ref.append(-mp.fsum(t))
            scale.append(mp.fsum(abs(v) for v in t))
    return ref, scale


def check_backward_mpmath(o):
    for K in (0, 5, 16):
        x, G = bw_inputs(K)
        ref, scale = bw_reference(x, G)
        got = o.backward(x, G)
        got_ld = o.backward_ld(x, G)
        assert got.shape == (x.size,)
        for i in range(x.size):
            _rel_ok(got[i], ref[i], scale[i], 1e-17, f"backward K={K} x={x[i]}")
            with mp.workdps(DPS):
                err = abs(ld_to_mp(got_ld[i]) - ref[i])
                assert err <= mp.mpf(1e-17) * scale[i], f"backward_ld K={K} x={x[i]} err {mp.nstr(err, 3)}"


def check_central_difference_mpmath(o):
    """The long-double central difference with h = 1e-6 max(1, x) reaches the
    exact derivative within its truncation, h^2/6 |L'''| <= h^2/6 sum |G_k|
    F_{k+3} (F_k decreases in k, so that is below h^2/6 of the scale), plus
    the rounding of the difference, about 1e-19/h of the scale."""
    for K in (0, 5, 16):
        x, G = bw_inputs(K)
        ref, scale = bw_reference(x, G)
        got = o.central_difference(x, G)
        for i in range(x.size):
            h = 1e-6 * max(1.0, float(x[i]))
            rel = h * h / 6 + 1e-18 / h + 1e-15
            _rel_ok(got[i], ref[i], scale[i], rel, f"central_difference K={K} x={x[i]}")


def check_backward_is_central_difference(o):
    """The derivative rule and the difference quotient agree (a relation
    between two oracle functions that share no formula)."""
    rng = np.random.default_rng(7)
    x = np.concatenate([np.geomspace(1e-6, 3e3, 40), [0.0, 11.9, 29.0]])
    G = rng.standard_normal((x.size, 10))
    a = o.backward(x, G)
    b = o.central_difference(x, G)
    F = o.boys(x, 10)
    scale = (np.abs(G) * F[:, 1:]).sum(axis=1)
    assert np.all(np.abs(a - b) <= 1e-9 * scale), "backward and central_difference disagree"


# ---------------------------------------------------------------------------
# Pair sums.

PS_X = np.array([0.0, 0.5, 3.0, 5.95, 6.0, 11.0, 14.5, 15.0, 25.0])
PS_ROWS = [4, 0, 8, 6]


def ps_inputs(K: int):
    rng = np.random.default_rng(300 + K)
    return PS_X.copy(), rng.standard_normal(PS_X.size), rng.standard_normal(K + 1)


def check_pairsum_mpmath(o):
    for K in (0, 12, 32):
        x, y, c = ps_inputs(K)
        z, sc = o.pairsum(x, y, c, PS_ROWS)
        assert len(z) == len(PS_ROWS) and len(sc) == len(PS_ROWS)
        with mp.workdps(DPS):
            for r, i in enumerate(PS_ROWS):
                terms, aterms = [], []
                for j in range(x.size):
                    s = float(x[i] + x[j])  # the pair argument is formed in double
                    for l in range(K + 1):
                        t = mp.mpf(float(c[l])) * _f_mp(l, s)
                        terms.append(t * mp.mpf(float(y[j])))
                        aterms.append(abs(t) * abs(mp.mpf(float(y[j]))))
                ref, scale = mp.fsum(terms), mp.fsum(aterms)
                _rel_ok(z[r], ref, scale, 1e-17, f"pairsum K={K} row {i}")
                _rel_ok(sc[r], scale, scale, 1e-17, f"pairsum scale K={K} row {i}")


def check_pairsum_row_sums(o):
    """With c = e_l and y = 1, z_i is the row sum of F_l over the pair
    arguments x_i + x_j; every row, in the default order."""
    x = PS_X
    for l in (0, 3):
        c = np.zeros(l + 1)
        c[l] = 1.0
        z, _ = o.pairsum(x, np.ones(x.size), c)
        assert len(z) == x.size
        for i in range(x.size):
            col = o.boys_ld(x[i] + x, l)[:, l]
            assert abs(float(z[i]) - float(col.sum())) <= 4e-16 * float(col.sum()), \
                f"pairsum row sum l={l} row {i}"


ALL_CHECKS = [check_weighted_sum_mpmath, check_weighted_sum_unit_weights, check_backward_mpmath,
              check_central_difference_mpmath, check_backward_is_central_difference,
              check_pairsum_mpmath, check_pairsum_row_sums]

# Which check pins which oracle function (every composition has at least one
# check built from mpmath, not from the oracle's own F).
PINS = {
    "weighted_sum": ["check_weighted_sum_mpmath", "check_weighted_sum_unit_weights"],
    "backward": ["check_backward_mpmath", "check_backward_is_central_difference"],
    "backward_ld": ["check_backward_mpmath"],
    "central_difference": ["check_central_difference_mpmath", "check_backward_is_central_difference"],
    "pairsum": ["check_pairsum_mpmath", "check_pairsum_row_sums"],
}
