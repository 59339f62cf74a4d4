"""Pins of the MODIT oracle (Sec. 2.1.2) against facts that do not come from
the oracle itself: Poisson summation (the inverse DFT of the Voigt profile's
Fourier transform sampled at f = m/N is the N-periodic sum of the profile
sampled at the grid points), the linear weights of the lineshape density,
strength conservation (the transform is 1 at f = 0), and agreement with the
direct line-by-line sum within the paper's stated residual (App. B: below
1 % in FP64 away from the line bottoms of a wide dynamic range)."""
import math

import numpy as np
import pytest

import synth
from oracle import oracle as O
from oracle import modit as M


def _periodic_voigt(i, x0, beta_t, gamma_t, n_fft, images=60):
    """sum_p V(i - x0 + p n_fft) by direct evaluation of Re w (scipy wofz) for
    |p| <= images, plus the Lorentz tail of the remaining images,
    2 (gamma/pi) / n_fft^2 * sum_{p > images} 1/p^2 (the trigamma function)."""
    from scipy.special import polygamma
    i = np.asarray(i, float)
    acc = np.zeros(i.size)
    for p in range(-images, images + 1):
        acc += O.voigt_profile(i - x0 + p * n_fft, beta_t, gamma_t)
    return acc + 2.0 * gamma_t / math.pi / n_fft ** 2 * float(polygamma(1, images + 1))


@pytest.mark.parametrize("beta_t,gamma_t", [(2.3, 0.7), (0.8, 6.0), (4.0, 1e-3)])
def test_single_line_on_node_is_periodic_voigt(beta_t, gamma_t):
    n, n_fft, j0 = 300, 1024, 120
    lsd = np.zeros((n, 2))
    lsd[j0, 0] = 1.0
    sq = M.sigma_q_periodic(lsd, beta_t, np.array([gamma_t, 2 * gamma_t]), n_fft)
    ref = _periodic_voigt(np.arange(n_fft), j0, beta_t, gamma_t, n_fft)
    assert np.max(np.abs(sq - ref)) < 1e-9 * np.max(ref)


def test_linear_weights_in_position_and_width():
    """A line between grid nodes and between width bins splits over the four
    neighbouring nodes with the linear weights."""
    n, d = 200, 0.1
    x = np.array([50.3, 120.0])
    g0 = 1.5
    lng = np.log(np.array([g0, g0 * math.exp(1.5 * d)]))
    S = np.array([2.0, 3.0])
    lng0, dd, K = M.width_grid(lng, d)
    assert (lng0, K) == (math.log(g0), 3) and dd == d
    lsd = M.lineshape_density(x, lng, S, n, lng0, dd, K)
    exp = np.zeros((n, K))
    exp[50, 0], exp[51, 0] = 2.0 * 0.7, 2.0 * 0.3
    exp[120, 1], exp[120, 2] = 3.0 * 0.5, 3.0 * 0.5
    np.testing.assert_allclose(lsd, exp, rtol=1e-12, atol=1e-15)
    # and the convolution of that density is the same combination of profiles
    bt, n_fft = 1.7, 512
    gk = np.exp(lng0 + dd * np.arange(K))
    sq = M.sigma_q_periodic(lsd, bt, gk, n_fft)
    i = np.arange(n_fft)
    ref = (1.4 * _periodic_voigt(i, 50, bt, gk[0], n_fft) + 0.6 * _periodic_voigt(i, 51, bt, gk[0], n_fft)
           + 1.5 * _periodic_voigt(i, 120, bt, gk[1], n_fft) + 1.5 * _periodic_voigt(i, 120, bt, gk[2], n_fft))
    assert np.max(np.abs(sq - ref)) < 1e-9 * np.max(ref)


def test_line_position_is_linear_in_log_nu():
    nu = 4340.0 * np.exp(np.arange(100) / 1e6)
    nu_c = np.array([nu[10], math.sqrt(nu[20] * nu[21]), nu[-1], nu[0] * 0.999, nu[-1] * 1.001])
    x = M.line_positions(nu, nu_c)
    np.testing.assert_allclose(x[:3], [10.0, 20.5, 99.0], rtol=0, atol=1e-7)
    assert np.isnan(x[3]) and np.isnan(x[4])


def _lines(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return synth.LineList(np.sort(rng.uniform(lo, hi, n)), 10 ** rng.uniform(-23, -20, n),
                          rng.exponential(1000, n), rng.uniform(0.01, 0.1, n), rng.uniform(0.5, 0.8, n),
                          18.0, 0, np.array([1.5]))


def test_strength_is_conserved():
    nu = 4340.0 * np.exp(np.arange(3000) / 1e6)
    ll = _lines(200, nu[0], nu[-1], 1)
    sig, parts = M.modit_cross_section(ll, 1200.0, 0.3, nu, want_parts=True)
    assert parts["sigma_q"].sum() == pytest.approx(parts["S"].sum(), rel=1e-12)
    assert parts["lsd"].sum() == pytest.approx(parts["S"].sum(), rel=1e-12)


@pytest.mark.parametrize("R0,T,P,bound", [(1e6, 1000.0, 1.0, 1e-2), (3e6, 2000.0, 0.05, 1e-2),
                                           (1e7, 2000.0, 0.05, 3e-3)])
def test_modit_matches_direct_sum(R0, T, P, bound):
    """Resolved lines inside the window: MODIT close to the direct sum wherever
    the cross-section is above 1e-2 of its maximum, and closer as the grid
    resolves the Doppler width better.  Splitting a line over two grid nodes
    errs by about V''/8, i.e. ~1/(8 beta~^2) of the peak, so at R0 = 1e6 a
    Doppler-dominated line (beta~ ~ 3 grid steps) is only good to a few %."""
    nu = 4340.0 * np.exp(np.arange(4000) / R0)
    ll = _lines(300, nu[200], nu[-200], 2)
    sig = M.modit_cross_section(ll, T, P, nu)
    ref = O.cross_section(ll, T, P, nu)
    keep = ref > 1e-2 * ref.max()
    err = np.max(np.abs(sig[keep] - ref[keep]) / ref[keep])
    assert err < bound, err


def _emission_case(R0, n_nu, seed=7):
    """A single-species atmosphere (config-3 small layers) whose lines sit
    inside the window, with low lower-state energies so that the 100 bar
    column is not opaque at every wavenumber (median line depth ~0.5)."""
    from dataclasses import replace
    wl = synth.make_config(3, "small")
    nu = 4340.0 * np.exp(np.arange(n_nu) / R0)
    rng = np.random.default_rng(seed)
    n = 300
    ll = replace(wl.lines[0], nu_c=np.sort(rng.uniform(nu[200], nu[-200], n)),
                 S0=10 ** np.clip(rng.normal(-23.0, 1.67, n), -28, -18), E_low=rng.exponential(300.0, n),
                 alpha_ref=rng.uniform(0.01, 0.1, n), n_texp=rng.uniform(0.5, 0.8, n))
    wl = replace(wl, nu=nu, lines=[ll])
    return wl, np.array([1300.0, 0.10, -3.0])


def test_modit_emission_converges_to_direct():
    """The emission spectrum with MODIT opacities (the paper's use of MODIT in
    place of the direct LPF) approaches the direct-sum spectrum as the grid
    resolves the coldest layer's Doppler width: beta~ = 1.0 grid step at
    R0 = 1e6 (206 K top layer), 3.1 at R0 = 3e6, where the linear line-shape
    density's smearing of a profile core falls to ~1 %."""
    from dataclasses import replace
    errs = []
    for R0, n_nu in ((1e6, 2500), (3e6, 6000)):
        wl, th = _emission_case(R0, n_nu)
        F_lpf = O.emission_F0(wl, th)
        F_modit = O.emission_F0(replace(wl, atmos=replace(wl.atmos, opacity="modit")), th)
        rel = np.abs(F_modit - F_lpf) / F_lpf
        errs.append((rel.max(), np.median(rel)))
    (m1, med1), (m3, med3) = errs
    assert m3 < 2e-2 and med3 < 2e-3, errs
    assert m1 > 2 * m3, errs                     # coarser grid, larger error
    assert m3 > 1e-6                             # the two paths really differ


def test_modit_emission_rejects_tangents():
    from dataclasses import replace
    wl, th = _emission_case(1e6, 600)
    wl = replace(wl, atmos=replace(wl.atmos, opacity="modit"))
    with pytest.raises(ValueError):
        O.optical_depths(wl, th, want_dT=True)
    with pytest.raises(ValueError):
        O.optical_depths(wl, th, nu_idx=[0, 1])
