"""CPU checks of the far-tier truncation rule (no GPU)."""
import math

import numpy as np

from far_tier import far_outer2, far_reach2


def test_far_reach_bound_covers_truncation():
    """Host-side check of the far-tier rule: at the reach it picks, dropping the
    wing terms beyond r^3 (value) and r^4 (tangent) changes no far pair by more
    than the stated bounds (dense scan over gamma^2 <= g_max, dnu^2 >= R)."""
    for bmax, gmax in [(1e-4, 0.0), (1e-4, 1e-8), (1e-4, 1e-4), (1e-4, 1e-2), (1e-4, 1.0), (1e-4, 100.0)]:
        R, _ = far_reach2(bmax, gmax)
        assert 222.0 * bmax <= R <= bmax / 2e-5 * (1 + 1e-5)
        g = np.concatenate([[0.0], gmax * np.logspace(-6, 0, 200)])[:, None]
        D = R * np.logspace(0, 3, 300)[None, :] + g
        r, b = 1.0 / D, bmax
        c = [np.ones_like(D), 3 * b + 0 * g, 15 * b * b - 4 * b * g, 105 * b ** 3 - 60 * b * b * g,
             48 * b * b * g * g - 840 * b ** 3 * g, 1680 * b ** 3 * g * g, -960 * b ** 3 * g ** 3]
        dropped = sum(c[k] * r ** k for k in range(3, 7))
        assert np.max(np.abs(dropped)) <= 4.8e-9
        # tangent: derivatives along b and g with unit log-steps (scale 1 per log-derivative)
        dcb = [0 * D, 3 * b + 0 * g, 30 * b * b - 4 * b * g, 315 * b ** 3 - 120 * b * b * g,
               96 * b * b * g * g - 2520 * b ** 3 * g, 5040 * b ** 3 * g * g, -2880 * b ** 3 * g ** 3]
        dcg = [0 * D, 0 * D, -4 * b * g, -60 * b * b * g, 96 * b * b * g * g - 840 * b ** 3 * g,
               3360 * b ** 3 * g * g, -2880 * b ** 3 * g ** 3]
        tb = sum(dcb[k] * r ** k for k in range(4, 7))
        tg = sum(dcg[k] * r ** k for k in range(4, 7)) - sum((k + 1) * c[k] * r ** k * (g * r) for k in range(3, 7))
        tE = sum(c[k] * r ** k for k in range(4, 7))
        assert np.max(np.abs(tb) + np.abs(tg) + np.abs(tE)) <= 1.42e-8 * 3


def test_far_tangent_cut_after_r3_bound():
    """Where the tangent stops at r^3 (tangent mode, narrow Lorentz widths), the
    dropped tangent terms from r^4 on stay within the stated bound, and where
    the Lorentz widths are wide the r^4 term is kept."""
    n_cut = 0
    for bmax, gmax in [(1e-4, 0.0), (1e-4, 1e-10), (1e-4, 1e-6), (1e-4, 1e-4), (1e-4, 1e-2), (1e-4, 1.0)]:
        R, t3 = far_reach2(bmax, gmax, tangent=True)
        if t3:
            continue
        n_cut += 1
        g = np.concatenate([[0.0], gmax * np.logspace(-6, 0, 200)])[:, None]
        D = R * np.logspace(0, 3, 300)[None, :] + g
        r, b = 1.0 / D, bmax
        c = [np.ones_like(D), 3 * b + 0 * g, 15 * b * b - 4 * b * g, 105 * b ** 3 - 60 * b * b * g,
             48 * b * b * g * g - 840 * b ** 3 * g, 1680 * b ** 3 * g * g, -960 * b ** 3 * g ** 3]
        dcb = [0 * D, 3 * b + 0 * g, 30 * b * b - 4 * b * g, 315 * b ** 3 - 120 * b * b * g,
               96 * b * b * g * g - 2520 * b ** 3 * g, 5040 * b ** 3 * g * g, -2880 * b ** 3 * g ** 3]
        dcg = [0 * D, 0 * D, -4 * b * g, -60 * b * b * g, 96 * b * b * g * g - 840 * b ** 3 * g,
               3360 * b ** 3 * g * g, -2880 * b ** 3 * g ** 3]
        tb = sum(dcb[k] * r ** k for k in range(3, 7))
        tg = sum(dcg[k] * r ** k for k in range(3, 7)) - sum((k + 1) * c[k] * r ** k * (g * r) for k in range(2, 7))
        tE = sum(c[k] * r ** k for k in range(3, 7))
        assert np.max(np.abs(tb) + np.abs(tg) + np.abs(tE)) <= 1.42e-8 * 3
    assert n_cut >= 3
    assert far_reach2(1e-4, 100.0, tangent=True)[1]



def _wing_terms(b, g, D):
    """c_k r^k and their log-derivatives along b and g on a (g, D) mesh."""
    c = [np.ones_like(D), 3 * b + 0 * g, 15 * b * b - 4 * b * g, 105 * b ** 3 - 60 * b * b * g,
         48 * b * b * g * g - 840 * b ** 3 * g, 1680 * b ** 3 * g * g, -960 * b ** 3 * g ** 3]
    dcb = [0 * D, 3 * b + 0 * g, 30 * b * b - 4 * b * g, 315 * b ** 3 - 120 * b * b * g,
           96 * b * b * g * g - 2520 * b ** 3 * g, 5040 * b ** 3 * g * g, -2880 * b ** 3 * g ** 3]
    dcg = [0 * D, 0 * D, -4 * b * g, -60 * b * b * g, 96 * b * b * g * g - 840 * b ** 3 * g,
           3360 * b ** 3 * g * g, -2880 * b ** 3 * g ** 3]
    return c, dcb, dcg


def test_far_outer_bound_covers_truncation():
    """Beyond the outer reach the value and the tangent stop at r^2: at the
    reach the rule picks, the dropped terms (from c_2 r^2 on) stay within the
    same bounds as in the far tier (dense scan over gamma^2 <= g_max and
    dnu^2 >= R'), in forward mode (value only) and in tangent mode."""
    n_outer = 0
    for bmax, gmax in [(1e-4, 0.0), (1e-4, 1e-8), (1e-4, 1e-4), (1e-4, 1e-2), (1e-4, 1.0), (1e-4, 100.0),
                       (3e-3, 1e-3)]:
        for tangent in (False, True):
            R, _ = far_reach2(bmax, gmax, tangent)
            Ro = far_outer2(bmax, gmax, tangent)
            assert Ro >= R
            if Ro >= 1e38:
                continue
            assert Ro <= R * 1e4 * (1 + 1e-5)
            n_outer += 1
            g = np.concatenate([[0.0], gmax * np.logspace(-6, 0, 200)])[:, None]
            D = Ro * np.logspace(0, 3, 300)[None, :] + g
            r, b = 1.0 / D, bmax
            c, dcb, dcg = _wing_terms(b, g, D)
            dropped = sum(c[k] * r ** k for k in range(2, 7))
            assert np.max(np.abs(dropped)) <= 4.8e-9
            if tangent:
                tb = sum(dcb[k] * r ** k for k in range(2, 7))
                tg = sum(dcg[k] * r ** k for k in range(2, 7)) - sum(
                    (k + 1) * c[k] * r ** k * (g * r) for k in range(1, 7))
                tE = sum(c[k] * r ** k for k in range(2, 7))
                assert np.max(np.abs(tb) + np.abs(tg) + np.abs(tE)) <= 1.42e-8 * 3
    assert n_outer >= 8


def test_far_outer_reach_scales_with_widths():
    """Narrow lines (Doppler only) get an outer reach a few times the far
    reach in distance; wide Lorentz widths push it out."""
    b = 1.27e-4   # beta^2 of a mass-18 line at 4360 cm^-1 and 1300 K
    R0, Ro0 = far_reach2(b, 0.0, True)[0], far_outer2(b, 0.0, True)
    assert 2.0 < math.sqrt(Ro0 / R0) < 10.0
    Ro1 = far_outer2(b, 1.0, True)
    assert Ro1 > 10.0 * Ro0
