"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: 1e-4 relative (max over points) on cross-sections and fluxes,
1e-3 on gradients (per component, relative to max(|g*|, 1e-6 ||g*||_inf)).
The GPU's hjert approximates Re w to ~1e-6; FP32 rounding and the blocked
compensated sum add ~1e-6.
"""
import math
import os
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from far_tier import far_outer2, far_reach2

pytestmark = pytest.mark.gpu

RTOL_FLUX = 1e-4
RTOL_GRAD = 1e-3


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def exo():
    import paper_2105_14782_amd as pkg
    pkg.load_library()
    from paper_2105_14782_amd import api
    return api


def maxrel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b) / np.abs(b)))


# ------------------------------------------------------------------ special functions

def test_hjert_f32_error_map(exo):
    _say("hjert_f32 error map")
    xs = np.concatenate([[0.0], np.logspace(-4, 5, 181)])
    as_ = np.concatenate([[0.0], np.logspace(-9, -4.2, 13), np.logspace(-4, 5, 91)])
    X, A = np.meshgrid(xs, as_)
    x, a = X.ravel(), A.ravel()
    H, Lg = exo.hjert_f32(torch.tensor(x, dtype=torch.float32, device="cuda"),
                          torch.tensor(a, dtype=torch.float32, device="cuda"), want_L=True)
    H, Lg = H.cpu().double().numpy(), Lg.cpu().double().numpy()
    w = O.faddeeva(x.astype(np.float32).astype(float) + 1j * a.astype(np.float32).astype(float))
    errH = np.abs(H - w.real)
    # paper bound (Sec. 2.1.1, App. A): |hjert - Re wofz| < 1e-6
    assert errH.max() < 1e-6, (errH.max(), x[errH.argmax()], a[errH.argmax()])
    # relative accuracy wherever H is not vanishingly small
    big = w.real > 1e-30
    rel = errH[big] / w.real[big]
    assert np.max(rel[(x[big] ** 2 + a[big] ** 2) >= 111]) < 2e-6
    core = (x ** 2 + a ** 2) < 111
    assert np.max(np.abs(Lg[core] - w.imag[core])) < 2e-6
    # the core branch: the rational approximation of w for a >= 1e-5, its
    # first-order expansion about the real axis below; relative accuracy of
    # H and of L in both parts, down to the Lorentz tail of the core (FP32
    # inputs and outputs included)
    a32 = a.astype(np.float32).astype(float)
    for name, part in (("a >= 1e-5", a32 >= 1e-5), ("a < 1e-5", a32 < 1e-5)):
        sel = core & part & (w.real > 1e-30)
        assert sel.sum() > 100
        relr = errH[sel] / w.real[sel]
        sel_l = core & part & (np.abs(w.imag) > 1e-30)
        rell = np.abs(Lg[sel_l] - w.imag[sel_l]) / np.abs(w.imag[sel_l])
        _say(f"  core {name}: max rel err H {relr.max():.2e}, L {rell.max():.2e}")
        assert relr.max() < 1e-6, (name, relr.max(), x[sel][relr.argmax()], a[sel][relr.argmax()])
        assert rell.max() < 1e-6, (name, rell.max())


def test_hjert_f64_error_map(exo):
    xs = np.concatenate([[0.0], np.logspace(-4, 5, 121)])
    as_ = np.concatenate([[0.0], np.logspace(-4, 5, 61)])
    X, A = np.meshgrid(xs, as_)
    x, a = X.ravel(), A.ravel()
    H = exo.hjert_f64(torch.tensor(x, device="cuda"), torch.tensor(a, device="cuda")).cpu().numpy()
    w = O.faddeeva(x + 1j * a).real
    assert np.max(np.abs(H - w)) < 1e-6


def test_trans2e3_against_exact(exo):
    x = np.concatenate([[0.0], np.logspace(-8, 2.5, 400)])
    T, dT = exo.trans2e3(torch.tensor(x, device="cuda"))
    T, dT = T.cpu().numpy(), dT.cpu().numpy()
    exact = O.transmission(x)
    # paper: AS70 2E3 within 5e-8 in F64 (App. A, Table 4)
    assert np.max(np.abs(T - exact)) < 5e-8
    np.testing.assert_allclose(dT, O.dtransmission(x), rtol=2e-6, atol=1e-12)


# ------------------------------------------------------------------ cross-section

def _ctx_with(exo, wl, grid=None):
    c = exo.Context(0)
    for s, ll in enumerate(wl.lines):
        c.set_lines(s, ll)
    c.set_grid(wl.nu if grid is None else grid)
    return c


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp64_tiled"])
def test_cross_section_config1(exo, prec):
    _say(f"cross_section config1 {prec}")
    wl = synth.make_config(1, "full")
    c = _ctx_with(exo, wl)
    sig = c.cross_section(0, wl.T, wl.P_bar, prec).cpu().double().numpy()
    ref = O.cross_section(wl.lines[0], wl.T, wl.P_bar, wl.nu)
    err = maxrel(sig, ref)
    _say(f"  max rel err {err:.3e}")
    assert err < (RTOL_FLUX if prec == "fp32" else 1e-5)


@pytest.mark.parametrize("factor", [1e-8, 1e14, 1e27])
def test_cross_section_strength_scales(exo, factor):
    """The config-1 list with every strength multiplied by `factor` (strengths
    from 1e-33 to 1e7 cm/molecule over the three cases): the FP32 records
    carry a power-of-two scale chosen on the device from the largest
    strength, so the relative error is that of the unscaled list."""
    from dataclasses import replace
    _say(f"cross_section strengths x {factor:g}")
    wl = synth.make_config(1, "full")
    ll = replace(wl.lines[0], S0=wl.lines[0].S0 * factor)
    c = _ctx_with(exo, replace(wl, lines=[ll]))
    ref = O.cross_section(ll, wl.T, wl.P_bar, wl.nu)
    for prec, tol in [("fp32", RTOL_FLUX), ("fp64", 1e-5)]:
        err = maxrel(c.cross_section(0, wl.T, wl.P_bar, prec).cpu().double().numpy(), ref)
        _say(f"  {prec} max rel err {err:.3e}")
        assert err < tol


@pytest.mark.parametrize("n_lines,n_nu", [(1, 2), (1, 7), (33, 257), (97, 1023), (200, 4097)])
def test_cross_section_ragged_shapes(exo, n_lines, n_nu):
    rng = np.random.default_rng(n_lines * 7919 + n_nu)
    nu = np.sort(rng.uniform(4340, 4350, n_nu)) if n_nu > 2 else np.array([4344.0, 4345.0])
    ll = synth.LineList(np.sort(rng.uniform(4339, 4351, n_lines)), 10 ** rng.uniform(-25, -20, n_lines),
                        rng.exponential(1000, n_lines), rng.uniform(0.01, 0.1, n_lines),
                        rng.uniform(0.5, 0.8, n_lines), 18.0, 0, np.array([1.5]))
    c = exo.Context(0)
    c.set_lines(3, ll)
    c.set_grid(nu)
    for T, P in [(800.0, 0.01), (1500.0, 3.0)]:
        ref = O.cross_section(ll, T, P, nu)
        for prec, tol in [("fp32", RTOL_FLUX), ("fp64", 1e-5), ("fp64_tiled", 1e-5)]:
            got = c.cross_section(3, T, P, prec).cpu().double().numpy()
            assert maxrel(got, ref) < tol, (prec, T, P)


def test_cross_section_degenerate_widths(exo):
    """P = 0 (pure Doppler, a = 0), huge pressure (a^2 >= 111 everywhere), natural width."""
    rng = np.random.default_rng(11)
    n = 50
    nu = np.linspace(4340, 4345, 3001)
    ll = synth.LineList(np.sort(rng.uniform(4340.5, 4344.5, n)), 10 ** rng.uniform(-23, -20, n),
                        np.zeros(n), rng.uniform(0.01, 0.1, n), rng.uniform(0.5, 0.8, n), 28.0, 0,
                        np.array([1.0]), gamma_nat=rng.uniform(0, 1e-3, n))
    c = exo.Context(0)
    c.set_lines(0, ll)
    c.set_grid(nu)
    for T, P in [(600.0, 0.0), (1200.0, 300.0), (2500.0, 1e-6)]:
        ref = O.cross_section(ll, T, P, nu)
        got = c.cross_section(0, T, P, "fp32").cpu().double().numpy()
        assert maxrel(got, ref) < RTOL_FLUX, (T, P)
        got = c.cross_section(0, T, P, "fp64_tiled").cpu().numpy()
        assert maxrel(got, ref) < 1e-5, ("fp64_tiled", T, P)


def test_cross_section_is_deterministic(exo):
    wl = synth.make_config(1, "full")
    c = _ctx_with(exo, wl)
    a = c.cross_section(0, 1000.0, 1.0).cpu()
    b = c.cross_section(0, 1000.0, 1.0).cpu()
    assert torch.equal(a, b)


def _lines(rng, centres, mass=18.0):
    n = centres.size
    return synth.LineList(np.sort(centres), 10 ** rng.uniform(-23, -20, n), rng.exponential(1000, n),
                          rng.uniform(0.01, 0.1, n), rng.uniform(0.5, 0.8, n), mass, 0, np.array([1.5]))


def test_cross_section_far_lines_only(exo):
    """Every line is farther than the far-tier reach from the whole grid, so the
    sum runs only the truncated wing polynomial; it must still match the exact
    profile to FP32 accuracy, far inside the 1e-4 bound."""
    _say("cross_section far lines only")
    rng = np.random.default_rng(21)
    centres = np.concatenate([rng.uniform(4250.0, 4330.0, 300), rng.uniform(4356.0, 4450.0, 300)])
    ll = _lines(rng, centres)
    nu = np.linspace(4340.0, 4345.0, 2501)
    c = exo.Context(0)
    c.set_lines(1, ll)
    c.set_grid(nu)
    for T, P in [(2500.0, 1e-3), (1000.0, 30.0)]:
        c.profile(True)
        got = c.cross_section(1, T, P, "fp32").cpu().double().numpy()
        near = c.profile_read_near()
        c.profile(False)
        assert near == 0.0, near
        err = maxrel(got, O.cross_section(ll, T, P, nu))
        _say(f"  T={T} P={P}: max rel err {err:.2e}")
        assert err < 2e-6


@pytest.mark.parametrize("P", [1e-6, 1e-2, 1.0, 30.0, 300.0])
def test_cross_section_outer_tier_pressures(exo, P):
    """Lines spread over a band ten times wider than the grid: from low
    pressure (most pairs beyond the outer reach, both polynomials cut after
    r^2) to 300 bar (wide Lorentz widths, outer reach pushed out or absent),
    the FP32 cross-section matches the exact profile to FP32 accuracy and the
    kernel's outer-pair count matches the host statement of the rule."""
    _say(f"cross_section outer tier P={P}")
    rng = np.random.default_rng(int(1e3 * P) % 997 + 5)
    ll = _lines(rng, rng.uniform(4200.0, 4500.0, 1500))
    nu = np.linspace(4340.0, 4370.0, 3001)
    c = exo.Context(0)
    c.set_lines(0, ll)
    c.set_grid(nu)
    T = 1500.0
    c.profile(True)
    got = c.cross_section(0, T, P, "fp32").cpu().double().numpy()
    outer = c.profile_read_far_outer()
    c.profile(False)
    _, exp_out = _near_pairs_expected(ll, T, nu, P=P)
    ref = O.cross_section(ll, T, P, nu)
    err = maxrel(got, ref)
    _say(f"  outer pairs {outer:.0f} (expected {exp_out}) of {ll.n * nu.size}, max rel err {err:.2e}")
    assert outer == exp_out
    if P <= 1.0:
        assert outer > 0.5 * ll.n * nu.size
    assert err < 2e-6


def _near_pairs_expected(ll, T, nu, wave_points=256, P=1.0):
    """(pairs the near tier should take, outer pairs): lines within the
    layer's far reach of the points a wave owns, and lines beyond its outer
    reach from all of them."""
    kKB, kMU, kC = 1.380649e-16, 1.66053906660e-24, 2.99792458e10
    beta_last = math.sqrt(kKB * T / (ll.mass_amu * kMU)) * ll.nu_c[-1] / kC
    thr = float(np.float32(2.0 * 111.0 * beta_last * beta_last))
    bmax = thr * (1.001 / 222.0)
    gam = ll.alpha_ref * (T / 296.0) ** (-ll.n_texp) * P
    gmax = float(np.max((gam * gam).astype(np.float32))) * 1.001
    reach = math.sqrt(far_reach2(bmax, gmax)[0])
    outer = math.sqrt(far_outer2(bmax, gmax))
    total = n_out = 0
    for j0 in range(0, nu.size, wave_points):
        j1 = min(j0 + wave_points, nu.size) - 1
        lo, hi = nu[j0] - reach, nu[j1] + reach
        n_near = np.searchsorted(ll.nu_c, hi, side="right") - np.searchsorted(ll.nu_c, lo, side="left")
        total += int(n_near) * (j1 - j0 + 1)
        lo, hi = nu[j0] - outer, nu[j1] + outer
        n_in = np.searchsorted(ll.nu_c, hi, side="right") - np.searchsorted(ll.nu_c, lo, side="left")
        n_out += int(ll.n - n_in) * (j1 - j0 + 1)
    return total, n_out


@pytest.mark.parametrize("n_nu", [1000, 4097])
def test_near_tier_pair_count(exo, n_nu):
    """The kernel's near / far / outer split equals the classification it is
    designed to make (lines sorted by centre, reaches from the largest Doppler
    and Lorentz widths)."""
    rng = np.random.default_rng(n_nu)
    ll = _lines(rng, rng.uniform(4330.0, 4370.0, 3000))
    nu = np.linspace(4340.0, 4360.0, n_nu)
    c = exo.Context(0)
    c.set_lines(0, ll)
    c.set_grid(nu)
    n_outer = 0
    for T in (300.0, 2000.0):
        c.profile(True)
        c.cross_section(0, T, 1.0, "fp32")
        n, ms, evals = c.profile_read()
        near = c.profile_read_near()
        outer = c.profile_read_far_outer()
        c.profile(False)
        exp, exp_out = _near_pairs_expected(ll, T, nu)
        _say(f"  n_nu={n_nu} T={T}: near {near:.0f} expected {exp}, outer {outer:.0f} expected {exp_out} "
             f"of {evals:.0f}")
        assert evals == ll.n * n_nu
        assert near == exp
        assert outer == exp_out
        n_outer += outer
    assert n_outer > 0


# ------------------------------------------------------------------ emission

def _atmos(exo, wl, theta=None, **kw):
    return exo.Atmos.from_workload(wl.atmos, list(range(len(wl.lines))), theta, **kw)


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp64_tiled"])
def test_emission_small_with_response(exo, prec):
    _say(f"emission small {prec}")
    wl = synth.make_config(2, "small")
    c = _ctx_with(exo, wl)
    F = c.emission_flux(_atmos(exo, wl), exo.Response.from_workload(wl.response), prec).cpu().double().numpy()
    ref = O.emission_flux(wl, wl.theta_star)
    err = maxrel(F, ref)
    _say(f"  max rel err {err:.3e}")
    assert err < (RTOL_FLUX if prec == "fp32" else 1e-5)


def test_emission_small_F0_zero_bottom(exo):
    wl = synth.make_config(2, "small")
    wl.atmos.bottom = 1
    c = _ctx_with(exo, wl)
    F0 = c.emission_flux(_atmos(exo, wl), None, "fp32").cpu().double().numpy()
    ref = O.emission_F0(wl, wl.theta_star)
    assert maxrel(F0, ref) < RTOL_FLUX


def test_emission_and_gradient_at_the_layer_limit(exo):
    """4096 layers, the most an atmosphere may have (thin layers from 1e-8 to
    1e2 bar): the spectrum in FP32 and FP64 and the VJP of a random cotangent
    (every parameter and every layer) against the oracle; 4097 are refused."""
    from dataclasses import replace
    import paper_2105_14782_amd as pkg
    _say("emission and gradient at 4096 layers")
    wl0 = synth.make_config(4, "tiny")
    wl = replace(wl0, atmos=replace(wl0.atmos, P_bar=np.logspace(-8.0, 2.0, 4096)))
    c = _ctx_with(exo, wl)
    th = wl.theta
    atm = _atmos(exo, wl, th)
    resp = exo.Response.from_workload(wl.response, th)
    t = O.flux_tangents(wl, th, per_layer=True)
    for prec, tol in [("fp32", RTOL_FLUX), ("fp64", 1e-5)]:
        err = maxrel(c.emission_flux(atm, resp, prec).cpu().double().numpy(), t["F"])
        _say(f"  {prec} max rel err {err:.3e}")
        assert err < tol
    cot = np.random.default_rng(4096).normal(size=resp.out_len).astype(np.float32)
    g, gl, _ = c.flux_vjp(atm, resp, torch.tensor(cot, device="cuda"), want_layers=True)
    err = _check_grad(g, t["dF"] @ cot.astype(np.float64), RTOL_GRAD)
    errl = _check_grad(gl, t["dF_dTn"] @ cot.astype(np.float64), RTOL_GRAD)
    _say(f"  grad rel err {err.max():.2e}; per-layer max rel err {errl.max():.2e}")
    assert np.all(err < RTOL_GRAD) and np.all(errl < RTOL_GRAD)
    over = _atmos(exo, replace(wl, atmos=replace(wl.atmos, P_bar=np.logspace(-8.0, 2.0, 4097))), th)
    with pytest.raises(pkg.ExoError) as e:
        c.emission_flux(over, resp)
    assert e.value.code == pkg.EXO_EINVAL


def test_emission_sub_grid_window(exo):
    """A model grid that is a window of the registered grid gives the window's spectrum."""
    wl = synth.make_config(2, "small")
    c = _ctx_with(exo, wl)
    b, n = 311, 700
    F0w = c.emission_flux(_atmos(exo, wl, grid_begin=b, grid_len=n), None, "fp32").cpu()
    F0 = c.emission_flux(_atmos(exo, wl), None, "fp32").cpu()
    np.testing.assert_allclose(F0w.numpy(), F0[b:b + n].numpy(), rtol=1e-6)


def test_emission_full_config2_sampled(exo):
    """Full configuration-2 size, in the bench's launch shapes: F0 at 64 grid
    points (both ends and 62 random ones) against the oracle (all lines, all
    layers)."""
    _say("emission full config2 sampled")
    wl = synth.make_config(2, "full")
    c = _ctx_with(exo, wl)
    rng = np.random.default_rng(2024)
    idx = np.sort(rng.choice(np.arange(1, wl.nu.size - 1), 62, replace=False))
    idx = np.concatenate([[0], idx, [wl.nu.size - 1]])
    ref = O.emission_F0(wl, wl.theta_star, nu_idx=idx)
    for prec, tol in [("fp32", RTOL_FLUX), ("fp64", 1e-5), ("fp64_tiled", 1e-5)]:
        F0 = c.emission_flux(_atmos(exo, wl), None, prec).cpu().double().numpy()
        err = maxrel(F0[idx], ref)
        _say(f"  {prec} max rel err {err:.3e} over {idx.size} points")
        assert err < tol
    # the response stage at full size, on a seeded synthetic input spectrum
    F0s = 1e4 * (1 + 0.3 * np.sin(np.arange(wl.nu.size) / 37.0) * np.cos(np.arange(wl.nu.size) / 5.1))
    r = exo.Response.from_workload(wl.response)
    got = c.broaden(torch.tensor(F0s, device="cuda"), r).cpu().numpy()
    ref = O.response(F0s, wl.nu, wl.response)
    assert maxrel(got, ref) < 1e-11


def test_emission_config3_medium_sampled(exo):
    """The throughput workload's line density at 1e6 lines (config 3 medium:
    100,000-point grid at R0 = 1e6, 100 layers, 1e13 pairs; the line records
    are processed in several layer chunks): FP32 F0 at sampled grid points
    against the oracle."""
    _say("emission config3 medium sampled")
    wl = synth.make_config(3, "medium")
    c = _ctx_with(exo, wl)
    theta = np.array([wl.atmos.T0, wl.atmos.alpha, wl.atmos.log10_mmr[0]])
    rng = np.random.default_rng(2025)
    idx = np.sort(rng.choice(wl.nu.size, 4, replace=False))
    idx[0], idx[-1] = 0, wl.nu.size - 1
    F0 = c.emission_flux(_atmos(exo, wl, theta), None, "fp32").cpu().double().numpy()
    ref = O.emission_F0(wl, theta, nu_idx=idx)
    err = maxrel(F0[idx], ref)
    _say(f"  fp32 max rel err {err:.3e}")
    assert err < RTOL_FLUX


def test_emission_full_config3_sampled(exo):
    """The whole throughput workload (config 3: 1e7 lines, 100,000-point grid
    at R0 = 1e6, 100 layers, 1e14 pairs) in the launch shapes of the bench's
    config-3 record: FP32 F0 at 16 grid points (both ends and 14 random ones)
    against the oracle over all lines and all layers."""
    _say("emission full config3 sampled: synthesising 1e7 lines")
    wl = synth.make_config(3, "full")
    c = _ctx_with(exo, wl)
    theta = np.array([wl.atmos.T0, wl.atmos.alpha, wl.atmos.log10_mmr[0]])
    _say("  GPU spectrum (FP32, 1e14 pairs)")
    F0 = c.emission_flux(_atmos(exo, wl, theta), None, "fp32").cpu().double().numpy()
    c.close()
    rng = np.random.default_rng(2026)
    idx = np.sort(rng.choice(np.arange(1, wl.nu.size - 1), 14, replace=False))
    idx = np.concatenate([[0], idx, [wl.nu.size - 1]])
    _say("  oracle at 16 points (1.6e10 evaluations)")
    ref = O.emission_F0(wl, theta, nu_idx=idx)
    err = maxrel(F0[idx], ref)
    _say(f"  fp32 max rel err {err:.3e}")
    assert err < RTOL_FLUX


def test_response_rejects_out_of_range(exo):
    import paper_2105_14782_amd as pkg
    wl = synth.make_config(2, "small")
    c = _ctx_with(exo, wl)
    r = exo.Response.from_workload(wl.response)
    r.out_begin, r.out_len = 0, wl.nu.size      # taps would reach past both grid ends
    with pytest.raises(pkg.ExoError) as e:
        c.emission_flux(_atmos(exo, wl), r)
    assert e.value.code == pkg.EXO_EINVAL
    r = exo.Response.from_workload(wl.response)
    r.vsini_kms = 0.1                            # narrower than two grid spacings
    with pytest.raises(pkg.ExoError) as e:
        c.emission_flux(_atmos(exo, wl), r)
    assert e.value.code == pkg.EXO_EINVAL
    bad = _atmos(exo, wl)
    bad.P_bar = bad.P_bar[::-1].copy()          # pressures must ascend
    with pytest.raises(pkg.ExoError) as e:
        c.emission_flux(bad, None)
    assert e.value.code == pkg.EXO_EINVAL
    bad = _atmos(exo, wl)
    bad.species = [0, 7]                         # slot 7 was never registered
    with pytest.raises(pkg.ExoError) as e:
        c.emission_flux(bad, None)
    assert e.value.code == pkg.EXO_ENOTSET


# ------------------------------------------------------------------ gradients

def _grad_case(size):
    wl = synth.make_config(4, size)
    F_star = O.emission_flux(wl, wl.theta_star)
    rng = np.random.default_rng(4004)
    data = F_star * (1 + 0.01 * rng.normal(size=F_star.size))
    sigma = 0.01 * F_star
    return wl, data, sigma


def _check_grad(g, g_ref, tol):
    scale = np.maximum(np.abs(g_ref), 1e-6 * np.max(np.abs(g_ref)))
    err = np.abs(g - g_ref) / scale
    return err


def test_flux_vjp_small_against_oracle(exo):
    _say("flux_vjp small")
    wl, data, sigma = _grad_case("small")
    c = _ctx_with(exo, wl)
    th = wl.theta
    atm = _atmos(exo, wl, th)
    resp = exo.Response.from_workload(wl.response, th)
    F = c.emission_flux(atm, resp, "fp32").double()
    d = torch.tensor(data, device="cuda")
    s = torch.tensor(sigma, device="cuda")
    cot = (-(d - F) / s ** 2).float().contiguous()
    g, gl, Fv = c.flux_vjp(atm, resp, cot, want_layers=True, want_flux=True)
    assert torch.equal(Fv.cpu(), F.float().cpu())
    # oracle gradient of the same loss with the oracle's F
    Lo, g_ref, gl_ref = O.loss_gradient(wl, th, data, sigma, per_layer=True)
    err = _check_grad(g, g_ref, RTOL_GRAD)
    _say(f"  grad rel err {err}")
    assert np.all(err < RTOL_GRAD), (g, g_ref)
    errl = np.abs(gl - gl_ref) / np.maximum(np.abs(gl_ref), 1e-6 * np.abs(gl_ref).max())
    _say(f"  per-layer gradient max rel err {errl.max():.2e}")
    assert np.max(errl) < RTOL_GRAD


def test_flux_vjp_reduced_against_oracle(exo):
    """Gradient at the reduced configuration-4 size (1e3 lines per species,
    2,000 points, 100 layers, the full response): every parameter and every
    layer's dL/dT_n against the oracle's forward-mode gradient, 1e-3."""
    _say("flux_vjp reduced config-4 size")
    wl, data, sigma = _grad_case("reduced")
    c = _ctx_with(exo, wl)
    th = wl.theta
    atm = _atmos(exo, wl, th)
    resp = exo.Response.from_workload(wl.response, th)
    F = c.emission_flux(atm, resp, "fp32").double()
    cot = (-(torch.tensor(data, device="cuda") - F) / torch.tensor(sigma, device="cuda") ** 2).float().contiguous()
    g, gl, _ = c.flux_vjp(atm, resp, cot, want_layers=True)
    _, g_ref, gl_ref = O.loss_gradient(wl, th, data, sigma, per_layer=True)
    err = _check_grad(g, g_ref, RTOL_GRAD)
    errl = np.abs(gl - gl_ref) / np.maximum(np.abs(gl_ref), 1e-6 * np.abs(gl_ref).max())
    _say(f"  grad rel err {err}; per-layer max rel err {errl.max():.2e}")
    assert np.all(err < RTOL_GRAD), (g, g_ref)
    assert np.max(errl) < RTOL_GRAD


@pytest.mark.parametrize("size", ["small", "reduced"])
def test_flux_vjp_fp64_against_oracle(exo, size):
    """The FP64 gradient (the tiled FP64 form in tangent mode, forward and
    adjoint in double precision): every parameter and every layer's dL/dT_n
    against the oracle at 1e-5, and the spectrum it returns equal to the
    tiled FP64 forward spectrum."""
    _say(f"flux_vjp FP64 {size}")
    wl, data, sigma = _grad_case(size)
    c = _ctx_with(exo, wl)
    th = wl.theta
    atm = _atmos(exo, wl, th)
    resp = exo.Response.from_workload(wl.response, th)
    F = c.emission_flux(atm, resp, "fp64_tiled")
    cot = (-(torch.tensor(data, device="cuda") - F) / torch.tensor(sigma, device="cuda") ** 2).contiguous()
    for prec in ("fp64_tiled", "fp64"):
        g, gl, Fv = c.flux_vjp(atm, resp, cot, want_layers=True, want_flux=True, precision=prec)
        assert torch.equal(Fv.cpu(), F.cpu())
    _, g_ref, gl_ref = O.loss_gradient(wl, th, data, sigma, per_layer=True)
    err = _check_grad(g, g_ref, 1e-5)
    errl = np.abs(gl - gl_ref) / np.maximum(np.abs(gl_ref), 1e-6 * np.abs(gl_ref).max())
    _say(f"  grad rel err {err}; per-layer max rel err {errl.max():.2e}")
    assert np.all(err < 1e-5), (g, g_ref)
    assert np.max(errl) < 1e-5


def test_emission_autograd_function(exo):
    wl, data, sigma = _grad_case("tiny")
    c = _ctx_with(exo, wl)
    atm = _atmos(exo, wl)
    resp = exo.Response.from_workload(wl.response)
    theta = torch.tensor(wl.theta, dtype=torch.float64, requires_grad=True)
    F = exo.EmissionFlux.apply(theta, c, atm, resp)
    d = torch.tensor(data, device="cuda", dtype=torch.float32)
    s = torch.tensor(sigma, device="cuda", dtype=torch.float32)
    loss = 0.5 * torch.sum(((d - F) / s) ** 2)
    loss.backward()
    _, g_ref = O.loss_gradient(wl, wl.theta, data, sigma)
    err = _check_grad(theta.grad.numpy(), g_ref, RTOL_GRAD)
    _say(f"  EmissionFlux backward: max rel err {err.max():.2e}")
    assert np.all(err < RTOL_GRAD), (theta.grad, g_ref)
