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


def far_reach2(bmax, gmax):
    """Squared far-tier reach of a layer: the smallest R in [222 b, b / 2e-5]
    at which the bounds of the dropped wing terms, with
    u^p v^q <= U^p max_g (g/R)^q / (1 + g/R)^(p+q), stay within the largest
    values they take at U = 2e-5; found by a two-level search on ln R with 64
    candidates per level (the first candidate that holds)."""
    def holds(U, gr):
        M = lambda p, q: far_monomial(p, q, U, gr)
        A3, A4 = 105 * M(3, 0) + 60 * M(2, 1), 48 * M(2, 2) + 840 * M(3, 1)
        A5, A6 = 1680 * M(3, 2), 960 * M(3, 3)
        Av3, Av4 = 105 * M(3, 1) + 60 * M(2, 2), 48 * M(2, 3) + 840 * M(3, 2)
        Av5, Av6 = 1680 * M(3, 3), 960 * M(3, 4)
        ev = A3 + A4 + A5 + A6
        et = 4 * A4 + 5 * A5 + 6 * A6 + 4 * Av3 + 5 * Av4 + 6 * Av5 + 7 * Av6
        return ev <= 4.8e-9 and et <= 1.42e-8
    lo, hi = math.log(222.0 * bmax), math.log(bmax / 2e-5)
    a, b, x = lo, hi, hi
    for _ in range(2):
        ok = [holds(bmax / math.exp(a + (b - a) * (k + 1) * (1.0 / 64.0)),
                    gmax / math.exp(a + (b - a) * (k + 1) * (1.0 / 64.0))) for k in range(64)]
        if not any(ok):
            break
        k1 = ok.index(True)
        bn = a + (b - a) * (k1 + 1) * (1.0 / 64.0)
        a = a if k1 == 0 else a + (b - a) * k1 * (1.0 / 64.0)
        b = x = bn
    return float(np.float32(math.exp(x) * (1.0 + 1e-6)))
