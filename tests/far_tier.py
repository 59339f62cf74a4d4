"""Host-side statement of the far-tier rule of the FP32 Voigt sum, for tests.

A line farther than the layer's reach from every grid point of a wave is
summed with the wing polynomial cut after r^3 (value) and r^4 (tangent).  The
reach is the smallest one at which a bound of the dropped terms stays within
the largest values that bound takes at the fixed ratio beta^2 r = 2e-5.
Beyond a second, outer reach both polynomials stop at r^2 within the same
bounds.
"""
import math

import numpy as np


def far_monomial(p, q, U, gr):
    m = U ** p
    if q == 0:
        return m
    t = min(gr, q / p)
    return m * t ** q / (1.0 + t) ** (p + q)


def far_bound_holds(U, gr, t3=True, kv=None, kt=None):
    """Bounds of the dropped wing terms: the value keeps c_0..c_(kv-1) (after
    r^3 by default), the tangent t_0..t_(kt-1) (after r^4, or r^3 with
    t3=False; kt=8: no tangent), with
    u^p v^q <= U^p max_g (g/R)^q / (1 + g/R)^(p+q)."""
    kv = 3 if kv is None else kv
    kt = (4 if t3 else 3) if kt is None else kt
    M = lambda p, q: far_monomial(p, q, U, gr)
    A = [0.0, 3 * M(1, 0), 15 * M(2, 0) + 4 * M(1, 1), 105 * M(3, 0) + 60 * M(2, 1),
         48 * M(2, 2) + 840 * M(3, 1), 1680 * M(3, 2), 960 * M(3, 3), 0.0]
    Av = [0.0, 3 * M(1, 1), 15 * M(2, 1) + 4 * M(1, 2), 105 * M(3, 1) + 60 * M(2, 2),
          48 * M(2, 3) + 840 * M(3, 2), 1680 * M(3, 3), 960 * M(3, 4)]
    ev = 0.0
    for k in range(kv, 7):
        ev += A[k]
    et = 0.0
    for k in range(kt, 8):
        et += k * (A[k] + Av[k - 1])
    return ev <= 4.8e-9 and et <= 1.42e-8


def _search(bmax, gmax, lo, hi, t3=True, kv=None, kt=None):
    """Two-level search on ln R with 64 candidates per level (the first that
    holds); None if the bound does not hold at hi."""
    a, b, found = lo, hi, False
    for _ in range(2):
        xs = [a + (b - a) * (k + 1) * (1.0 / 64.0) for k in range(64)]
        ok = [far_bound_holds(bmax / math.exp(x), gmax / math.exp(x), t3, kv, kt) for x in xs]
        if not any(ok):
            break
        k1 = ok.index(True)
        bn = xs[k1]
        a = a if k1 == 0 else a + (b - a) * k1 * (1.0 / 64.0)
        b, found = bn, True
    return b if found else None


def _far_x(bmax, gmax, tangent):
    lo, hi = math.log(222.0 * bmax), math.log(bmax / 2e-5)
    x, t3 = hi, True
    x3 = _search(bmax, gmax, lo, hi, True)
    if x3 is not None:
        x = x3
    if tangent:
        x2 = _search(bmax, gmax, lo, hi, False)
        if x2 is not None and x2 <= x + 0.6931471805599453:
            x, t3 = x2, False
    return x, t3


def far_reach2(bmax, gmax, tangent=False):
    """(squared far-tier reach, tangent keeps r^4) of a layer: the smallest R in
    [222 b, b / 2e-5] at which the bounds stay within the largest values they
    take at U = 2e-5; in tangent mode the cut after r^3 is taken where the
    reach it needs is at most twice that R."""
    x, t3 = _far_x(bmax, gmax, tangent)
    return float(np.float32(math.exp(x) * (1.0 + 1e-6))), t3


def far_outer2(bmax, gmax, tangent=False):
    """Squared outer reach of a layer: the smallest R' in [R, 1e4 R] (a search
    in ln R') beyond which the value and, in tangent mode, the tangent may stop
    at r^2 within the same bounds; FLT_MAX if none."""
    x, _ = _far_x(bmax, gmax, tangent)
    r = float(np.float32(math.exp(x) * (1.0 + 1e-6)))
    xo = _search(bmax, gmax, x, x + math.log(1e4), kv=2, kt=2 if tangent else 8)
    ro = float(np.finfo(np.float32).max) if xo is None else float(np.float32(math.exp(xo) * (1.0 + 1e-6)))
    return max(ro, r)
