"""Pins of the weak-line pre-selection oracle (App. G).

The contribution function e^{-tau} dtau/dlnP peaks where tau = 1 when the
optical depth grows in proportion to the pressure (a Doppler-broadened line
centre, tau = kappa P), and where tau = 1 as well for tau = c P^2 / 2 (the
collision-induced continuum, dtau proportional to P dP), i.e. at c P^2 = 2.
These closed forms, the margin rule and the monotonicity in line strength pin
the oracle without reusing its arithmetic.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import oracle as O
from oracle import selection as SEL


def test_argmax_of_pressure_proportional_depth():
    P = np.logspace(-6, 2, 400)
    dP = O.layer_dP_bar(P)
    prev = P[0] * P[0] / P[1]
    for kappa in (3e-4, 0.1, 7.0, 2e3):
        n, _ = SEL.contribution_argmax((kappa * dP)[:, None], P, dP)
        tau = kappa * (P - prev)
        assert n[0] == int(np.argmax(tau * np.exp(-tau)))
        if tau[-1] > 1.5:   # the photosphere lies inside the grid: tau ~ 1 (grid step 0.05 in ln P)
            assert abs(math.log(tau[n[0]])) < 0.05
        else:               # the column stays thin: the deepest layer contributes most
            assert n[0] == P.size - 1


def test_argmax_of_continuum_depth():
    P = np.logspace(-6, 2, 400)
    dP = O.layer_dP_bar(P)
    for c in (1e-3, 1.0, 40.0):
        dtau = c * P * dP
        n, _ = SEL.contribution_argmax(dtau[:, None], P, dP)
        assert abs(math.log(c * P[n[0]] ** 2 / 2.0)) < 0.1   # tau ~ c P^2 / 2 = 1


def _case(seed, n=400):
    rng = np.random.default_rng(seed)
    wl = synth.make_config(2, "tiny")
    nu_c = np.sort(rng.uniform(4340, 4380, n))
    ll = synth.LineList(nu_c, 10 ** rng.uniform(-27, -19, n), rng.exponential(3000, n),
                        rng.uniform(0.01, 0.1, n), rng.uniform(0.5, 0.8, n), 18.0, 0, np.array([1.5]))
    atm = replace(wl.atmos, P_bar=np.logspace(-8, 2, 100))
    return ll, atm


def test_margin_rule_and_extremes():
    ll, atm = _case(1)
    keep, n_line, n_cia = SEL.select_lines(ll, math.log10(0.0023), atm, 1700.0, margin=2)
    assert np.array_equal(keep, n_line <= n_cia + 2)
    counts = [SEL.select_lines(ll, math.log10(0.0023), atm, 1700.0, margin=m)[0].sum() for m in range(4)]
    assert counts == sorted(counts)
    # the strongest lines (at the isothermal temperature) are kept and the weakest dropped
    S = O.line_strength(ll.S0, ll.E_low, ll.nu_c, 1700.0, O.qr_ratio(1700.0, ll.qr_kind, ll.qr_params))
    assert keep[np.argsort(S)[-10:]].all()
    assert not keep[np.argsort(S)[:10]].any()


def test_stronger_lines_never_drop():
    """Scanning strengths over more temperatures only raises S_eff, so it can
    only add lines; scaling every strength up keeps a superset."""
    ll, atm = _case(2)
    lx = math.log10(0.0023)
    k1 = SEL.select_lines(ll, lx, atm, 1700.0)[0]
    k2 = SEL.select_lines(ll, lx, atm, 1700.0, T_strength=np.arange(500.0, 1701.0, 100.0))[0]
    assert np.all(k2 >= k1) and k2.sum() >= k1.sum()
    k3 = SEL.select_lines(replace(ll, S0=ll.S0 * 10.0), lx, atm, 1700.0)[0]
    assert np.all(k3 >= k1)


def test_line_centre_depth_is_column_times_profile_at_centre():
    """App. G: a line's optical depth at its own centre in layer n is the layer's
    column (Eq. dtau_line2) times S V(0; beta, gamma_n).  V(0) here comes from
    the oracle's Voigt profile (Re w by wofz) of that one line, evaluated at
    its centre: the selection's closed form uses erfcx instead.  With a list of
    strength temperatures, S is the largest S(T) over the list while the
    widths stay at T_atm."""
    ll, atm = _case(3, n=60)
    lx, T_atm = math.log10(0.0023), 1700.0
    P = atm.P_bar
    col = O.column_factor(O.layer_dP_bar(P), 10.0 ** lx, ll.mass_amu, atm.g_cgs)
    T_scan = [900.0, 1300.0, 1700.0]
    d1 = SEL.line_centre_dtau(ll, lx, atm, T_atm, [T_atm])
    d3 = SEL.line_centre_dtau(ll, lx, atm, T_atm, T_scan)
    for l in (0, 17, 59):
        one = replace(ll, nu_c=ll.nu_c[l:l + 1], S0=ll.S0[l:l + 1], E_low=ll.E_low[l:l + 1],
                      alpha_ref=ll.alpha_ref[l:l + 1], n_texp=ll.n_texp[l:l + 1])
        S = lambda T: float(O.line_strength(one.S0, one.E_low, one.nu_c, T,
                                            O.qr_ratio(T, one.qr_kind, one.qr_params))[0])
        boost = max(S(T) for T in T_scan) / S(T_atm)
        for n in (0, 40, 77, 99):
            sig = float(O.cross_section(one, T_atm, P[n], one.nu_c)[0])
            assert d1[n, l] == pytest.approx(col[n] * sig, rel=1e-12)
            assert d3[n, l] == pytest.approx(col[n] * sig * boost, rel=1e-12)
