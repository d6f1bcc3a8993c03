"""Rational minimax approximation by Remez' algorithm in extended precision.

Offline coefficient generation for the library (run once; its output headers
are committed).  It follows the six steps of the paper's Sec. II B:

1. initial equioscillation nodes (Chebyshev extrema of the interval; random
   ones when no pole-free solution exists);
2. solve rho(x_i) (f(x_i) - p(x_i)/q(x_i)) = (-1)^i E at the fixed nodes.  The
   divided differences of order n+1 of g_i = (f_i - (-1)^i E / rho_i) q(x_i)
   must vanish (g interpolates the degree-n polynomial p), which eliminates p
   and leaves an (m+1)x(m+1) eigenproblem for (E, q); p then follows by
   least squares;
3. keep the eigen-solution whose denominator has no zero on the interval;
4. stop when max |rho (f - r)| - |E| is small relative to |E|;
5. move the nodes to alternating local extrema of rho (f - r) found on a fine
   grid and refined by golden-section search, keeping the global maximum;
6. abort early when the smallest error at the new nodes already exceeds the
   target (de la Vallee-Poussin: no rational of this degree can meet it).

Linear algebra runs in mpmath (40 digits by default); function values come
from the Boys reference below in numpy long double (x87, 64-bit mantissa),
i.e. to about 1e-18 relative, which is far below the 5e-14 and 1e-6 targets.

The Boys reference values here are the series the paper uses for its own
reference values (Sec. II E, after Shavitt) followed by downward recurrence;
this module is product tooling and shares no code with the test oracle.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import mpmath as mp
import numpy as np

LD = np.longdouble


# ---------------------------------------------------------------------------
# Boys reference values (long double).

def boys_series(x, kmax: int) -> np.ndarray:
    """F_0..F_kmax at x (0 <= x <= 60), shape (len(x), kmax+1), long double.

    F_K(x) = e^-x / 2 sum_l x^l / prod_{j=0..l} (K + j + 1/2) with K = kmax,
    then F_k = (2x F_{k+1} + e^-x) / (2k+1)."""
    x = np.atleast_1d(np.asarray(x, dtype=LD))
    K = LD(kmax)
    term = np.full(x.shape, 1 / (K + LD(0.5)), dtype=LD)
    s = term.copy()
    l = 1
    while True:
        term = term * x / (K + LD(l) + LD(0.5))
        s += term
        r = x / (K + LD(l) + LD(1.5))
        if np.all(r < 1) and np.all(term * r / (1 - r) <= s * LD(2.0) ** -70):
            break
        l += 1
        if l > 10000:
            raise RuntimeError("series did not converge")
    e = np.exp(-x)
    F = np.empty(x.shape + (kmax + 1,), dtype=LD)
    F[..., kmax] = LD(0.5) * e * s
    for k in range(kmax - 1, -1, -1):
        F[..., k] = (2 * x * F[..., k + 1] + e) / (2 * k + 1)
    return F


def boys_k(k: int):
    """f(x) = F_k(x) as a vectorised long-double function."""
    return lambda x: boys_series(x, k)[..., k]


def rho_a(k: int):
    """Weight of region A (Sec. II C): rho_{A,k}(x) = max_l prod_{n=l}^{k-1} x/(n+1/2)."""
    def rho(x):
        x = np.atleast_1d(np.asarray(x, dtype=LD))
        best = np.ones(x.shape, dtype=LD)
        prod = np.ones(x.shape, dtype=LD)
        for n in range(k - 1, -1, -1):  # l = n: product over n..k-1
            prod = prod * x / (LD(n) + LD(0.5))
            best = np.maximum(best, prod)
        return best
    return rho


def rho_one(x):
    return np.ones(np.shape(np.atleast_1d(x)), dtype=LD)


# ---------------------------------------------------------------------------
# Helpers between mpmath and long double.

def _to_ld(v) -> LD:
    v = mp.mpf(v)
    if v == 0:
        return LD(0)
    m, e = mp.frexp(v)  # v = m 2^e, 0.5 <= |m| < 1
    mi = int(mp.nint(mp.ldexp(m, 64)))
    return np.ldexp(LD(mi), int(e) - 64)


def _ld_to_mp(v) -> mp.mpf:
    m, e = np.frexp(LD(v))
    return mp.ldexp(mp.mpf(int(m * LD(2.0) ** 64)), int(e) - 64)


def polyval_ld(c, x):
    """Horner in long double; c low -> high."""
    r = np.zeros_like(x) + c[-1]
    for a in c[-2::-1]:
        r = r * x + a
    return r


@dataclass
class RemezResult:
    n: int
    m: int
    a: float
    b: float
    p: list          # mp numbers, degree 0 upwards
    q: list          # mp numbers, degree 0 upwards, monic (q[m] = 1)
    E: float         # levelled error |E| of the last solve
    max_err: float   # max |rho (f - r)| on the final grid
    nodes: list = field(default_factory=list)
    iterations: int = 0
    converged: bool = False

    def p_ld(self):
        return [_to_ld(c) for c in self.p]

    def q_ld(self):
        return [_to_ld(c) for c in self.q]

    def __call__(self, x):
        x = np.asarray(x, dtype=LD)
        return polyval_ld(self.p_ld(), x) / polyval_ld(self.q_ld(), x)


class RemezFailure(RuntimeError):
    pass


def _divided_difference_rows(x, order: int):
    """Rows i = 0..N-order-1: weights of the divided difference over nodes
    x_i..x_{i+order} (annihilates every polynomial of degree < order)."""
    N = len(x)
    rows = []
    for i in range(N - order):
        row = [mp.mpf(0)] * N
        idx = list(range(i, i + order + 1))
        for j in idx:
            d = mp.mpf(1)
            for l in idx:
                if l != j:
                    d *= (x[j] - x[l])
            row[j] = 1 / d
        rows.append(row)
    return mp.matrix(rows)


def _solve_fixed_nodes(x, fx, rx, n, m, a, b):
    """Step 2 and 3: all (E, q) solutions, then the pole-free one."""
    N = n + m + 2
    D = _divided_difference_rows(x, n + 1)              # (m+1) x N
    V = mp.matrix(N, m + 1)
    for i in range(N):
        v = mp.mpf(1)
        for j in range(m + 1):
            V[i, j] = v
            v *= x[i]
    Fm = mp.diag(fx)
    S = mp.diag([(-1) ** i / rx[i] for i in range(N)])
    A = D * Fm * V
    B = D * S * V
    try:
        M = mp.inverse(B) * A
    except ZeroDivisionError as e:
        raise RemezFailure("singular system") from e
    evals, evecs = mp.eig(M)
    candidates = []
    for idx, E in enumerate(evals):
        if abs(mp.im(E)) > mp.mpf(10) ** (-mp.mp.dps // 2) * (1 + abs(E)):
            continue
        E = mp.re(E)
        q = [mp.re(evecs[j, idx]) for j in range(m + 1)]
        if q[m] == 0:
            continue
        q = [c / q[m] for c in q]  # monic
        if _has_pole(q, a, b):
            continue
        # p from V_n p = (f - E s) q at all nodes (least squares; consistent).
        Vn = mp.matrix(N, n + 1)
        rhs = mp.matrix(N, 1)
        for i in range(N):
            v = mp.mpf(1)
            for j in range(n + 1):
                Vn[i, j] = v
                v *= x[i]
            qi = mp.polyval(q[::-1], x[i])
            rhs[i] = (fx[i] - E * (-1) ** i / rx[i]) * qi
        p, _res = mp.qr_solve(Vn, rhs)
        candidates.append((abs(E), E, [p[j] for j in range(n + 1)], q))
    if not candidates:
        raise RemezFailure("no pole-free solution")
    candidates.sort(key=lambda c: c[0])
    return candidates[0][1:]


def _has_pole(q, a, b) -> bool:
    """Step 3: does q vanish on [a, b]?  Sign check on a fine grid plus the
    real roots of q."""
    a_, b_ = mp.mpf(a), mp.mpf(b)
    qa, qb = mp.polyval(q[::-1], a_), mp.polyval(q[::-1], b_)
    if qa == 0 or qb == 0 or (qa > 0) != (qb > 0):
        return True
    grid = np.linspace(float(a), float(b), 2001).astype(LD)
    vals = polyval_ld([_to_ld(c) for c in q], grid)
    if np.any(np.sign(vals) != np.sign(vals[0])):
        return True
    if len(q) > 1:
        try:
            roots = mp.polyroots(q[::-1], maxsteps=200, extraprec=60)
        except mp.NoConvergence:
            return False
        for r in roots:
            if abs(mp.im(r)) < mp.mpf(10) ** -20 and a_ <= mp.re(r) <= b_:
                return True
    return False


def _fine_grid(a, b, size):
    """Grid clustered towards both ends (Chebyshev-like) plus a uniform part."""
    t = np.linspace(0.0, np.pi, size // 2)
    cheb = 0.5 * (a + b) - 0.5 * (b - a) * np.cos(t)
    uni = np.linspace(a, b, size - size // 2)
    g = np.unique(np.concatenate([cheb, uni, [a, b]]))
    return g.astype(LD)


def _alternating_extrema(y, e, N):
    """Indices of N alternating extrema of e on the grid y, including the
    global maximum of |e|; None when fewer than N sign runs exist."""
    s = np.sign(e)
    s[s == 0] = 1
    runs = []
    start = 0
    for i in range(1, len(y) + 1):
        if i == len(y) or s[i] != s[start]:
            seg = slice(start, i)
            j = start + int(np.argmax(np.abs(e[seg])))
            runs.append(j)
            start = i
    if len(runs) < N:
        return None
    gmax = int(np.argmax(np.abs(e)))
    while len(runs) > N:
        # Drop an end run (keeps alternation); never the global maximum.
        if runs[0] == gmax:
            runs.pop()
        elif runs[-1] == gmax:
            runs.pop(0)
        elif abs(e[runs[0]]) < abs(e[runs[-1]]):
            runs.pop(0)
        else:
            runs.pop()
    return runs


def _golden_refine(err_fn, lo, hi, sign, iters=40):
    """Maximise sign * err over [lo, hi], elementwise over arrays of intervals."""
    gr = (np.sqrt(LD(5)) - 1) / 2
    a, b = lo.copy(), hi.copy()
    c = b - gr * (b - a)
    d = a + gr * (b - a)
    fc = sign * err_fn(c)
    fd = sign * err_fn(d)
    for _ in range(iters):
        left = fc > fd  # maximum in [a, d]: drop (d, b]; else drop [a, c)
        a, b, keep, fkeep = (np.where(left, a, c), np.where(left, d, b),
                             np.where(left, c, d), np.where(left, fc, fd))
        new = np.where(left, b - gr * (b - a), a + gr * (b - a))
        fnew = sign * err_fn(new)
        c, fc, d, fd = (np.where(left, new, keep), np.where(left, fnew, fkeep),
                        np.where(left, keep, new), np.where(left, fkeep, fnew))
    return (a + b) / 2


def remez(f, rho, a: float, b: float, n: int, m: int, tol: float = 1e-6, max_iter: int = 40,
          grid_size: int = 6000, dps: int = 40, seed: int = 0, target: float | None = None,
          verbose: bool = False) -> RemezResult:
    """Weighted rational minimax approximation of f on [a, b] in R_{n,m}.

    f and rho are vectorised long-double functions.  Returns the pole-free
    equioscillating r = p/q with monic q.  ``target``: abort early (step 6)
    when the levelled error cannot reach it.  Raises RemezFailure.  mpmath
    runs at ``dps`` digits inside the call; the caller's precision is left
    as it was."""
    with mp.workdps(dps):
        return _remez(f, rho, a, b, n, m, tol, max_iter, grid_size, seed, target, verbose)


def _remez(f, rho, a, b, n, m, tol, max_iter, grid_size, seed, target, verbose) -> RemezResult:
    N = n + m + 2
    rng = np.random.default_rng(seed)
    y = _fine_grid(a, b, grid_size)
    fy = f(y)
    ry = rho(y)

    def err_fn(x):
        return rho(x) * (f(x) - polyval_ld(p_ld, x) / polyval_ld(q_ld, x))

    # Step 1: Chebyshev extrema as the first guess.
    k = np.arange(N)
    nodes = (0.5 * (a + b) - 0.5 * (b - a) * np.cos(np.pi * k / (N - 1))).astype(LD)
    last = None
    for it in range(1, max_iter + 1):
        xs = [_ld_to_mp(v) for v in nodes]
        fx = [_ld_to_mp(v) for v in f(nodes)]
        rx = [_ld_to_mp(v) for v in rho(nodes)]
        try:
            E, p, q = _solve_fixed_nodes(xs, fx, rx, n, m, a, b)
        except RemezFailure:
            if last is not None and it > 3:
                raise
            # Step 1 again: a random guess.
            nodes = np.sort(rng.uniform(a, b, N)).astype(LD)
            nodes[0], nodes[-1] = LD(a), LD(b)
            continue
        p_ld = [_to_ld(c) for c in p]
        q_ld = [_to_ld(c) for c in q]
        e = ry * (fy - polyval_ld(p_ld, y) / polyval_ld(q_ld, y))
        idx = _alternating_extrema(y, e, N)
        if idx is None:
            raise RemezFailure(f"error curve has fewer than {N} alternations")
        # Step 5: refine every extremum by golden-section search.
        lo = np.array([y[max(i - 1, 0)] for i in idx], dtype=LD)
        hi = np.array([y[min(i + 1, len(y) - 1)] for i in idx], dtype=LD)
        sgn = np.sign(e[idx]).astype(LD)
        new = _golden_refine(err_fn, lo, hi, sgn)
        # Keep grid points that the refinement could not beat (end points).
        better = sgn * err_fn(new) >= sgn * e[idx]
        new = np.where(better, new, y[idx])
        err_new = np.abs(err_fn(new))
        max_err = float(max(np.max(np.abs(e)), np.max(err_new)))
        last = RemezResult(n, m, a, b, p, q, float(abs(E)), max_err, [float(v) for v in new], it)
        if verbose:
            print(f"  it {it}: |E|={float(abs(E)):.6e} max={max_err:.6e}")
        # Step 4: convergence.
        if max_err - float(abs(E)) <= tol * float(abs(E)):
            last.converged = True
            return last
        # Step 6: early abort.
        if target is not None and float(np.min(err_new)) > target:
            raise RemezFailure(f"target {target:g} unreachable in R_{n},{m}: "
                               f"min node error {float(np.min(err_new)):.3e}")
        nodes = np.sort(new)
    if last is None:
        raise RemezFailure("no iteration succeeded")
    return last


def walsh_search(f, rho, a, b, target, d_min=1, d_max=24, accept=None, verbose=False, **kw):
    """Degree choice of Sec. II D: walk the anti-diagonals n + m = d of the
    Walsh table from d_min upwards and return, on the first anti-diagonal
    with at least one entry meeting ``target``, the entry of smallest error.

    ``accept(result)`` may veto an entry (for example after rounding its
    coefficients to the working precision); it returns (ok, error)."""
    for d in range(d_min, d_max + 1):
        ok_entries = []
        for m in range(0, d + 1):
            n = d - m
            try:
                r = remez(f, rho, a, b, n, m, target=target, **kw)
            except RemezFailure as e:
                if verbose:
                    print(f"  ({n},{m}): {e}")
                continue
            err = r.max_err
            good = err <= target
            if good and accept is not None:
                good, err = accept(r)
            if verbose:
                print(f"  ({n},{m}): err {r.max_err:.3e} converged={r.converged} accept={good} ({err:.3e})")
            if good:
                ok_entries.append((err, r))
        if ok_entries:
            ok_entries.sort(key=lambda t: t[0])
            return ok_entries[0][1]
    raise RemezFailure(f"no entry with n + m <= {d_max} meets {target:g}")


# ---------------------------------------------------------------------------
# Region constants (Sec. II C).

def region_x0(kmax: int) -> float:
    """x0 = max{1, (prod_{n<kmax} (n+1/2))^(1/kmax)}: smallest x from which the
    upward recurrence to order kmax does not amplify errors."""
    if kmax == 0:
        return 1.0
    lp = sum(math.log(n + 0.5) for n in range(kmax))
    return max(1.0, math.exp(lp / kmax))


def region_x1(kmax: int, eps: float, guess: float = 20.0) -> float:
    """x1 solving Gamma(kmax+1/2, x1) / (2 x1^(kmax+1/2)) = eps (the asymptote's
    error for F_kmax), by Newton's method in mpmath."""
    with mp.workdps(40):
        s = kmax + mp.mpf(1) / 2
        g = lambda x: mp.gammainc(s, x) / (2 * x ** s) - eps
        return float(mp.findroot(g, guess))
