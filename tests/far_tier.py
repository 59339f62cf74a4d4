"""Host-side statement of the far-tier rule of the FP32 Voigt sum, for tests.

A line farther than the layer's reach from every grid point of a wave is
summed with the wing polynomial cut after r^3 (value) and r^4 (tangent).  The
reach is the smallest one at which a bound of the dropped terms stays within
the largest values that bound takes at the fixed ratio beta^2 r = 2e-5.
"""
import math

import numpy as np


def far_monomial(p, q, U, gr):
    m = U ** p
    if q == 0:
        return m
    t = min(gr, q / p)
    return m * t ** q / (1.0 + t) ** (p + q)


def far_bound_holds(U, gr, t3=True):
    """Bounds of the dropped wing terms (value after r^3; tangent after r^4,
    or after r^3 with t3=False), with u^p v^q <= U^p max_g (g/R)^q / (1 + g/R)^(p+q)."""
    M = lambda p, q: far_monomial(p, q, U, gr)
    A3, A4 = 105 * M(3, 0) + 60 * M(2, 1), 48 * M(2, 2) + 840 * M(3, 1)
    A5, A6 = 1680 * M(3, 2), 960 * M(3, 3)
    Av2 = 15 * M(2, 1) + 4 * M(1, 2)
    Av3, Av4 = 105 * M(3, 1) + 60 * M(2, 2), 48 * M(2, 3) + 840 * M(3, 2)
    Av5, Av6 = 1680 * M(3, 3), 960 * M(3, 4)
    ev = A3 + A4 + A5 + A6
    et = 4 * A4 + 5 * A5 + 6 * A6 + 4 * Av3 + 5 * Av4 + 6 * Av5 + 7 * Av6
    if not t3:
        et += 3 * A3 + 3 * Av2
    return ev <= 4.8e-9 and et <= 1.42e-8


def _search(bmax, gmax, lo, hi, t3):
    """Two-level search on ln R with 64 candidates per level (the first that
    holds); None if the bound does not hold at hi."""
    a, b, found = lo, hi, False
    for _ in range(2):
        xs = [a + (b - a) * (k + 1) * (1.0 / 64.0) for k in range(64)]
        ok = [far_bound_holds(bmax / math.exp(x), gmax / math.exp(x), t3) for x in xs]
        if not any(ok):
            break
        k1 = ok.index(True)
        bn = xs[k1]
        a = a if k1 == 0 else a + (b - a) * k1 * (1.0 / 64.0)
        b, found = bn, True
    return b if found else None


def far_reach2(bmax, gmax, tangent=False):
    """(squared far-tier reach, tangent keeps r^4) of a layer: the smallest R in
    [222 b, b / 2e-5] at which the bounds stay within the largest values they
    take at U = 2e-5; in tangent mode the cut after r^3 is taken where the
    reach it needs is at most twice that R."""
    lo, hi = math.log(222.0 * bmax), math.log(bmax / 2e-5)
    x, t3 = hi, True
    x3 = _search(bmax, gmax, lo, hi, True)
    if x3 is not None:
        x = x3
    if tangent:
        x2 = _search(bmax, gmax, lo, hi, False)
        if x2 is not None and x2 <= x + 0.6931471805599453:
            x, t3 = x2, False
    return float(np.float32(math.exp(x) * (1.0 + 1e-6))), t3
