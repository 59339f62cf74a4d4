"""Pins of the FP64 oracle against mathematics and physics it must satisfy.

None of these re-types an oracle formula: each compares the oracle with an
independent route (mpmath at 40 digits, quadrature of a defining integral, a
second formula the paper states for the same quantity, a closed form of a
special case, a conservation law, or finite differences).
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special

import synth
from oracle import oracle as O

HERE = os.path.dirname(__file__)
BOUNDS = json.load(open(os.path.join(HERE, "golden", "paper_bounds.json")))


# ---------------------------------------------------------------- Faddeeva

def _mp_w(z):
    mp.mp.dps = 40
    zz = mp.mpc(z.real, z.imag)
    return complex(mp.exp(-zz * zz) * mp.erfc(-1j * zz))


@pytest.mark.parametrize("x", [0.0, 1e-3, 0.3, 1.7, 4.0, 9.9, 10.6, 35.0, 400.0, 3e4])
@pytest.mark.parametrize("y", [1e-9, 1e-3, 0.2, 1.0, 5.0, 80.0])
def test_faddeeva_vs_mpmath(x, y):
    z = complex(x, y)
    ref = _mp_w(z)
    got = complex(O.faddeeva(z))
    assert abs(got - ref) <= 1e-13 * abs(ref) + 1e-300


def test_w_on_imaginary_axis_is_erfcx():
    y = np.array([1e-6, 0.1, 1.0, 3.0, 30.0, 1e4])
    np.testing.assert_allclose(O.faddeeva(1j * y).real, special.erfcx(y), rtol=1e-14)


def test_gaussian_limit_and_dawson():
    x = np.linspace(-6, 6, 241)
    np.testing.assert_allclose(O.voigt_hjerting(x, 0.0), np.exp(-x * x), rtol=1e-13, atol=1e-300)
    L = O.faddeeva(x + 0j).imag
    np.testing.assert_allclose(L, 2.0 * special.dawsn(x) / math.sqrt(math.pi), rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("x,a", [(0.0, 0.5), (1.3, 0.05), (4.0, 2.0), (12.0, 0.3)])
def test_hjert_defining_integral(x, a):
    """H(x,a) = a/pi * int exp(-y^2)/((x-y)^2 + a^2) dy by adaptive quadrature (Sec. 2.1.1)."""
    f = lambda y: math.exp(-y * y) / ((x - y) ** 2 + a * a)
    pts = sorted({x, 0.0})
    val = 0.0
    edges = [-12.0] + pts + [12.0]
    for lo, hi in zip(edges[:-1], edges[1:]):
        if hi > lo:
            val += integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-13, limit=400)[0]
    val *= a / math.pi
    assert O.voigt_hjerting(x, a) == pytest.approx(val, rel=1e-9)


def test_voigt_symmetry_normalisation_and_limits():
    beta, gam = 0.0098, 0.04
    d = np.linspace(0.1, 3.0, 7)
    np.testing.assert_allclose(O.voigt_profile(d, beta, gam), O.voigt_profile(-d, beta, gam), rtol=1e-15)
    # unit area: integral over [-Lw, Lw] plus the two Lorentzian tails 2 gamma/(pi Lw)
    Lw = 50.0
    val = integrate.quad(lambda t: float(O.voigt_profile(t, beta, gam)), -Lw, Lw,
                         points=[0.0], limit=2000, epsabs=0, epsrel=1e-12)[0]
    assert val + 2 * gam / (math.pi * Lw) == pytest.approx(1.0, abs=2e-9)
    # Lorentz limit (beta -> 0) and Gaussian limit (gamma -> 0)
    dd = np.array([0.05, 0.3, 2.0])
    lor = gam / math.pi / (dd ** 2 + gam ** 2)
    np.testing.assert_allclose(O.voigt_profile(dd, 1e-7, gam), lor, rtol=1e-6)
    dd = np.array([0.05, 0.3, 0.8])
    gau = np.exp(-dd ** 2 / (2 * 0.2 ** 2)) / (math.sqrt(2 * math.pi) * 0.2)
    np.testing.assert_allclose(O.voigt_profile(dd, 0.2, 1e-12), gau, rtol=1e-9)


# ---------------------------------------------------------------- line parameters

def test_line_strength_reference_and_exomol_route():
    """Eq. Slog with s0 from Eq. STexomol at T_ref must equal Eq. STexomol at any T (Sec. 2.2.2)."""
    nu = np.array([4341.2, 4355.0, 4379.9])
    E = np.array([0.0, 1234.5, 8000.0])
    A, gup = np.array([3.1, 0.02, 55.0]), np.array([3.0, 21.0, 7.0])
    # partition function Q(T) = Q0 (T/296)^1.5: q_r = (T/296)^1.5
    Q = lambda T: 41.0 * (T / 296.0) ** 1.5
    # Eq. STexomol with h, c, k_B written separately (not through c2)
    hck = O.H_PLANCK * O.C_LIGHT / O.K_BOLTZ

    def s_exomol(T):
        return gup / Q(T) * A / (8 * math.pi * O.C_LIGHT * nu ** 2) * np.exp(-hck * E / T) * (1 - np.exp(-hck * nu / T))

    S0 = s_exomol(296.0)
    for T in (296.0, 700.0, 1300.0, 2600.0):
        S = O.line_strength(S0, E, nu, T, O.qr_ratio(T, 0, [1.5]))
        np.testing.assert_allclose(S, s_exomol(T), rtol=1e-12)
    # the paper's printed c2
    assert O.C2 == pytest.approx(BOUNDS["c2_printed_cmK"]["value"], rel=5e-7)


def test_doppler_width_from_maxwell_velocity():
    # 1-D Maxwell velocity dispersion sqrt(kT/m) in SI units, times nu/c
    kB, mu, c = 1.380649e-23, 1.66053906660e-27, 2.99792458e8
    v = math.sqrt(kB * 1000.0 / (18 * mu))
    assert O.doppler_beta(4350.0, 1000.0, 18.0) == pytest.approx(4350.0 * v / c, rel=1e-14)
    assert O.doppler_beta(4350.0, 1000.0, 18.0) == pytest.approx(9.8616e-3, rel=1e-4)


def test_pressure_broadening_scalings():
    a, n = np.array([0.05]), np.array([0.6])
    assert O.lorentz_gamma(a, n, 296.0, 1.0)[0] == pytest.approx(0.05, rel=1e-15)
    assert O.lorentz_gamma(a, n, 592.0, 1.0)[0] == pytest.approx(0.05 * 2 ** -0.6, rel=1e-14)
    assert O.lorentz_gamma(a, n, 700.0, 3.0)[0] == pytest.approx(3 * O.lorentz_gamma(a, n, 700.0, 1.0)[0], rel=1e-15)
    assert O.lorentz_gamma(a, n, 700.0, 1.0, 0.01)[0] == pytest.approx(O.lorentz_gamma(a, n, 700.0, 1.0)[0] + 0.01)


def test_line_tangents_by_finite_differences():
    wl = synth.make_config(2, "tiny")
    ll = wl.lines[0]
    T, P, h = 1234.0, 0.3, 1e-3
    st = O.line_state(ll, T, P)
    sp, sm = O.line_state(ll, T + h, P), O.line_state(ll, T - h, P)
    np.testing.assert_allclose(st.dlnS_dT, (np.log(sp.S) - np.log(sm.S)) / (2 * h), rtol=1e-7)
    np.testing.assert_allclose(st.dbeta_dT, (sp.beta - sm.beta) / (2 * h), rtol=1e-8)
    np.testing.assert_allclose(st.dgamma_dT, (sp.gamma - sm.gamma) / (2 * h), rtol=1e-8)


# ---------------------------------------------------------------- cross-section

def test_cross_section_brute_force_mpmath():
    """sigma = sum_l S_l V_l with every profile from mpmath's erfc (independent of scipy)."""
    wl = synth.make_config(1, "tiny")
    ll = wl.lines[0]
    nu = wl.nu[::7]
    sig = O.cross_section(ll, 1000.0, 1.0, nu)
    kB, mu, c = 1.380649e-16, 1.66053906660e-24, 2.99792458e10
    hck = 6.62607015e-27 * c / kB
    ref = []
    for v in nu:
        acc = mp.mpf(0)
        for l in range(ll.n):
            S = ll.S0[l] * (1 - math.exp(-hck * ll.nu_c[l] / 1000.0)) / (1 - math.exp(-hck * ll.nu_c[l] / 296.0))
            beta = math.sqrt(kB * 1000.0 / (18 * mu)) * ll.nu_c[l] / c
            gam = ll.alpha_ref[l]
            z = complex(v - ll.nu_c[l], gam) / (math.sqrt(2) * beta)
            acc += S * _mp_w(z).real / (math.sqrt(2 * math.pi) * beta)
        ref.append(float(acc))
    np.testing.assert_allclose(sig, ref, rtol=1e-12)


def test_cross_section_tangent_fd():
    wl = synth.make_config(2, "tiny")
    ll = wl.lines[1]
    nu = wl.nu[::10]
    T, P, h = 950.0, 0.02, 1e-2
    s, ds = O.cross_section(ll, T, P, nu, want_dT=True)
    fd = (O.cross_section(ll, T + h, P, nu) - O.cross_section(ll, T - h, P, nu)) / (2 * h)
    np.testing.assert_allclose(ds, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())


# ---------------------------------------------------------------- transmission / RT

def test_transmission_vs_mpmath_and_recurrence():
    mp.mp.dps = 30
    x = np.array([1e-8, 1e-4, 0.01, 0.3, 1.0, 2.5, 10.0, 60.0])
    ref = np.array([float(2 * mp.expint(3, mp.mpf(v))) for v in x])
    np.testing.assert_allclose(O.transmission(x), ref, rtol=1e-13)
    assert O.transmission(0.0) == 1.0
    # E3 = (e^-x - x E2)/2  and  dT/dtau = -2 E2
    E1 = special.exp1(x)
    E2 = np.exp(-x) - x * E1
    E3 = (np.exp(-x) - x * E2) / 2
    np.testing.assert_allclose(O.transmission(x), 2 * E3, rtol=1e-12)
    h = 1e-6 * np.maximum(x, 1e-3)
    fd = (O.transmission(x + h) - O.transmission(x - h)) / (2 * h)
    np.testing.assert_allclose(O.dtransmission(x), fd, rtol=1e-6)


def test_rt_isothermal_and_slab_closed_forms():
    nu = np.linspace(4300, 4400, 5)
    B = O.planck_pi(1100.0, nu)
    rng = np.random.default_rng(3)
    dtau = rng.uniform(0.0, 0.7, (13, nu.size))
    FB = O.planck_pi(1500.0, nu)
    F0, _ = O.rt_recurrence(dtau, np.broadcast_to(B, dtau.shape), FB)
    Tprod = np.prod(O.transmission(dtau), axis=0)
    np.testing.assert_allclose(F0, B * (1 - Tprod) + Tprod * FB, rtol=1e-13)
    # F_B = B: an isothermal atmosphere emits exactly B
    F0b, _ = O.rt_recurrence(dtau, np.broadcast_to(B, dtau.shape), B)
    np.testing.assert_allclose(F0b, B, rtol=1e-14)
    # single slab
    tau = np.array([[0.4, 3.0, 1e-6, 0.0, 40.0]])
    F1, _ = O.rt_recurrence(tau, B[None, :], FB)
    t3 = np.array([float(2 * mp.expint(3, mp.mpf(v))) if v > 0 else 1.0 for v in tau[0]])
    np.testing.assert_allclose(F1, B * (1 - t3) + t3 * FB, rtol=1e-13)
    # opaque top layer -> pi B(T_0); transparent -> F_B
    assert F1[4] == pytest.approx(B[4], rel=1e-15)
    assert F1[3] == FB[3]


def test_rt_recurrence_equals_cumprod_form():
    """Eq. rerr (recurrence) against Eq. lart, F0 = (Phi o Q)^T u with Q_N = F_B (Sec. 3.1)."""
    rng = np.random.default_rng(5)
    N, J = 17, 6
    dtau = rng.exponential(0.3, (N, J))
    S = rng.uniform(1e3, 5e3, (N, J))
    FB = rng.uniform(1e3, 5e3, J)
    Tm = O.transmission(dtau)
    Qm = np.vstack([(1 - Tm) * S, FB[None]])
    tv = np.vstack([np.ones((1, J)), Tm])
    Phi = np.cumprod(tv, axis=0)
    np.testing.assert_allclose(O.rt_recurrence(dtau, S, FB)[0], np.sum(Phi * Qm, axis=0), rtol=1e-13)


def test_planck_integrates_to_stefan_boltzmann():
    T = 1300.0
    sigma_sb = 2 * math.pi ** 5 * O.K_BOLTZ ** 4 / (15 * O.C_LIGHT ** 2 * O.H_PLANCK ** 3)
    val = integrate.quad(lambda n: float(O.planck_pi(T, n)), 1e-3, 2e5, limit=400, epsrel=1e-12)[0]
    assert val == pytest.approx(sigma_sb * T ** 4, rel=1e-9)


def test_layer_thickness_and_column():
    P = np.logspace(-8, 2, 100)
    dP = O.layer_dP_bar(P)
    r = 10 ** (10 / 99)
    np.testing.assert_allclose(dP, P * (1 - 1 / r), rtol=1e-12)
    # the layers tile the column: sum dP telescopes to P_bottom - P_top/r
    assert np.sum(dP) == pytest.approx(P[-1] - P[0] / r, rel=1e-12)


def test_cia_against_number_density_route():
    """Eq. taucont: n^2 alpha Delta r with Delta r = H dP/P and n = xi P/(k T) (Sec. 2.4)."""
    atm = synth.make_config(2, "tiny").atmos
    T, P, dP, nu = 1234.0, 0.7, 0.05, np.array([4350.0, 4370.0])
    n = atm.vmr_h2 * P * 1e6 / (O.K_BOLTZ * T)
    Hs = O.K_BOLTZ * T / (atm.mmw * O.M_U * atm.g_cgs)
    alpha = O.cia_coefficient(T, nu, atm.cia_alpha0, atm.cia_Tpow, atm.cia_slope, atm.cia_nu_c)
    np.testing.assert_allclose(O.dtau_cia(T, P, dP, nu, atm), n * n * alpha * Hs * dP / P, rtol=1e-14)


# ---------------------------------------------------------------- response

def test_rotation_kernel_matches_disk_integral_and_is_normalised():
    u1, u2 = 0.5367, 0.3578

    def disk(x):
        s = math.sqrt(1 - x * x)
        I = lambda y: 1 - u1 * (1 - math.sqrt(max(0.0, 1 - x * x - y * y))) - u2 * (1 - math.sqrt(max(0.0, 1 - x * x - y * y))) ** 2
        return integrate.quad(I, -s, s, epsabs=0, epsrel=1e-12)[0]

    tot = integrate.quad(disk, -1, 1, epsabs=0, epsrel=1e-10, limit=200)[0]
    for x in (0.0, 0.3, 0.77, 0.99):
        assert O.rotation_kernel(x, u1, u2) == pytest.approx(disk(x) / tot, rel=1e-8)
    assert integrate.quad(lambda x: float(O.rotation_kernel(x, u1, u2)), -1, 1)[0] == pytest.approx(1.0, rel=1e-9)
    xs = np.linspace(-0.99, 0.99, 9)
    np.testing.assert_allclose(O.rotation_kernel(xs, 0, 0), 2 * np.sqrt(1 - xs ** 2) / math.pi, rtol=1e-14)
    h = 1e-6
    np.testing.assert_allclose(O.drotation_kernel(xs, u1, u2),
                               (O.rotation_kernel(xs + h, u1, u2) - O.rotation_kernel(xs - h, u1, u2)) / (2 * h), rtol=1e-6)


def _eslog(n=3000):
    return synth.eslog_grid(4340.0, 4380.0, n)


def test_response_flat_stays_flat_and_delta_gives_kernel():
    nu = _eslog()
    resp = synth.Response(28.1, 16.2, 0.5367, 0.3578, 1e5, 500, 2000)
    F = O.response(np.full(nu.size, 7.25), nu, resp)
    np.testing.assert_allclose(F, 7.25, rtol=1e-14)
    # a delta at j0 through rotation only: G_i = k_R(v_i - v_j0 + RV)/norm
    j0 = 1500
    d = np.zeros(nu.size)
    d[j0] = 1.0
    v = O.C_KMS * np.log(nu)
    idx = np.arange(1000, 2000)
    G = O.rotate(d, nu, idx, 28.1, 16.2, 0.5367, 0.3578)
    expect = O.rotation_kernel((v[idx] - v[j0] + 28.1) / 16.2, 0.5367, 0.3578)
    nz = expect > 0
    ratio = G[nz] / expect[nz]
    assert np.ptp(ratio) < 2e-3 * ratio.mean()   # one normalisation for all i (up to grid non-uniformity)


def test_response_line_centroid_moves_by_rv():
    nu = _eslog(6000)
    nu0 = 4360.0
    F0 = 1.0 - 0.5 * np.exp(-0.5 * ((nu - nu0) / 0.01) ** 2)
    resp = synth.Response(28.1, 16.2, 0.5367, 0.3578, 1e5, 1200, 3600)
    F = O.response(F0, nu, resp)
    nu_out = nu[1200:1200 + 3600]
    depth = 1.0 - F
    centroid = np.sum(nu_out * depth) / np.sum(depth)
    assert centroid == pytest.approx(nu0 * math.exp(-28.1 / O.C_KMS), abs=2e-4)


def test_ip_of_gaussian_adds_variances():
    nu = _eslog(8000)
    v = O.C_KMS * np.log(nu)
    vc = v[4000]
    s0 = 3.0
    G = np.exp(-0.5 * ((v - vc) / s0) ** 2)
    idx = np.arange(3000, 5000)
    F = O.instrumental(G, nu, idx, 1e5)[0]
    b = O.ip_beta_kms(1e5)
    s = math.sqrt(s0 ** 2 + b ** 2)
    expect = (s0 / s) * np.exp(-0.5 * ((v[idx] - vc) / s) ** 2)
    np.testing.assert_allclose(F, expect, rtol=2e-5, atol=1e-9)


# ---------------------------------------------------------------- gradients

def test_flux_tangents_by_central_differences():
    wl = synth.make_config(4, "tiny")
    th = wl.theta
    t = O.flux_tangents(wl, th, per_layer=True)
    steps = np.array([0.05, 1e-7, 1e-5, 1e-5, 1e-4, 1e-4])
    for k in range(6):
        e = np.zeros(6)
        e[k] = steps[k]
        fd = (O.emission_flux(wl, th + e) - O.emission_flux(wl, th - e)) / (2 * steps[k])
        np.testing.assert_allclose(t["dF"][k], fd, rtol=2e-6, atol=1e-7 * np.abs(fd).max(), err_msg=f"param {k}")
    # per-layer: dF/dT0 = sum_n dF/dT_n * T_n/T0
    T = O.temperatures(wl.atmos.P_bar, th[0], th[1])
    np.testing.assert_allclose(t["dF_dTn"].T @ (T / th[0]), t["dF"][0], rtol=1e-10)


def test_layer_temperatures_reproduce_power_law():
    """A layer-by-layer profile equal to the power law gives the same spectrum,
    and its per-layer tangents are those of the power-law model."""
    from dataclasses import replace
    wl = synth.make_config(4, "tiny")
    th = wl.theta
    T = O.temperatures(wl.atmos.P_bar, th[0], th[1])
    wl_l = replace(wl, atmos=replace(wl.atmos, T_layers=T))
    np.testing.assert_array_equal(O.emission_flux(wl_l, th), O.emission_flux(wl, th))
    a = O.flux_tangents(wl, th, per_layer=True)
    b = O.flux_tangents(wl_l, th, per_layer=True)
    np.testing.assert_array_equal(a["dF_dTn"], b["dF_dTn"])
    # (T0, alpha) no longer act on the layer-by-layer model; the other tangents are unchanged
    assert np.all(b["dF"][:2] == 0.0)
    np.testing.assert_array_equal(a["dF"][2:], b["dF"][2:])


def test_per_layer_tangents_by_central_differences():
    """dF/dT_n of a layer-by-layer profile (a non-monotonic one) against central
    differences of the oracle in T_n."""
    from dataclasses import replace
    wl = synth.make_config(4, "tiny")
    th = wl.theta
    NL = wl.atmos.P_bar.size
    rng = np.random.default_rng(3)
    T = O.temperatures(wl.atmos.P_bar, th[0], th[1]) * (1 + 0.1 * rng.uniform(-1, 1, NL))
    wl_l = replace(wl, atmos=replace(wl.atmos, T_layers=T))
    t = O.flux_tangents(wl_l, th, per_layer=True)
    sens = np.abs(t["dF_dTn"]).max(axis=1)
    layers = np.argsort(sens)[-3:]          # the three layers the spectrum depends on most
    assert sens[layers].min() > 1e-3 * sens.max()
    for n in layers:
        h = 1e-5 * T[n]
        Tp, Tm = T.copy(), T.copy()
        Tp[n] += h
        Tm[n] -= h
        fd = (O.emission_flux(replace(wl, atmos=replace(wl.atmos, T_layers=Tp)), th)
              - O.emission_flux(replace(wl, atmos=replace(wl.atmos, T_layers=Tm)), th)) / (2 * h)
        np.testing.assert_allclose(t["dF_dTn"][n], fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max(),
                                   err_msg=f"layer {n}")


def test_flux_jvp_is_the_tangent_combination():
    """J dtheta from flux_jvp equals the central difference along dtheta."""
    from dataclasses import replace
    wl = synth.make_config(4, "tiny")
    th = wl.theta
    NL = wl.atmos.P_bar.size
    rng = np.random.default_rng(8)
    dth = rng.normal(size=6) * np.array([5.0, 1e-3, 1e-2, 1e-2, 0.1, 0.1])
    F, jv = O.flux_jvp(wl, th, dth)
    h = 1e-4
    fd = (O.emission_flux(wl, th + h * dth) - O.emission_flux(wl, th - h * dth)) / (2 * h)
    np.testing.assert_allclose(jv, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
    # per-layer direction on a layer-by-layer profile
    T = O.temperatures(wl.atmos.P_bar, th[0], th[1])
    wl_l = replace(wl, atmos=replace(wl.atmos, T_layers=T))
    dT = rng.normal(size=NL) * 3.0
    F, jv = O.flux_jvp(wl_l, th, np.zeros(6), dT)
    fd = (O.emission_flux(replace(wl, atmos=replace(wl.atmos, T_layers=T + h * dT)), th)
          - O.emission_flux(replace(wl, atmos=replace(wl.atmos, T_layers=T - h * dT)), th)) / (2 * h)
    np.testing.assert_allclose(jv, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())


def test_loss_gradient_by_central_differences():
    wl = synth.make_config(4, "tiny")
    F_star = O.emission_flux(wl, wl.theta_star)
    rng = np.random.default_rng(44)
    data = F_star * (1 + 0.01 * rng.normal(size=F_star.size))
    sig = 0.01 * F_star
    L, g = O.loss_gradient(wl, wl.theta, data, sig)
    for k, h in enumerate([0.02, 1e-7, 1e-5, 1e-5, 1e-4, 1e-4]):
        e = np.zeros(6)
        e[k] = h
        fd = (O.gaussian_loss(O.emission_flux(wl, wl.theta + e), data, sig)
              - O.gaussian_loss(O.emission_flux(wl, wl.theta - e), data, sig)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-8 * abs(L))


# ---------------------------------------------------------------- column, IP width, Q(T) table

def test_column_factor_is_number_density_times_hydrostatic_thickness():
    """Eq. dtau_line2: the molecules of species m above unit area in a layer are
    n_m dz, with n_m = (X mu / M) P / (k_B T) (X a mass mixing ratio, mu the mean
    molecular weight, M the molecule's mass) and the hydrostatic thickness
    dz = H dP / P, H = k_B T / (mu m_u g) (Sec. 3).  T and mu cancel; the
    route keeps them to show it.  Constants written out in cgs here."""
    kB, m_u, bar = 1.380649e-16, 1.66053906660e-24, 1.0e6
    cases = [(1e-3, 2.3e-4, 900.0, 0.0023, 18.0, 2.33, 10 ** 5.03),
             (0.7, 0.05, 1300.0, 0.0058, 28.0, 2.33, 10 ** 5.03),
             (80.0, 6.1, 2400.0, 1e-6, 44.0, 2.9, 2.2e3)]
    for P, dP, T, X, M, mu, g in cases:
        n_m = (X * mu / M) * (P * bar) / (kB * T)
        H = kB * T / (mu * m_u * g)
        dz = H * dP / P
        assert float(O.column_factor(dP, X, M, g)) == pytest.approx(n_m * dz, rel=1e-13)
    # vectorised over layers, as the emission model uses it
    P = np.logspace(-8, 2, 100)
    dP = O.layer_dP_bar(P)
    col = O.column_factor(dP, 0.0023, 18.0, 10 ** 5.03)
    np.testing.assert_allclose(col, (0.0023 * 2.33 / 18.0) * dP * bar / (2.33 * m_u * 10 ** 5.03), rtol=1e-13)


def test_ip_width_is_c_over_R_at_half_maximum():
    """Sec. 4.2: an instrument of resolving power R has a Gaussian profile whose
    full width at half maximum is c/R in velocity.  Measured on the output of
    instrumental() for a delta input (half-maximum crossings located by linear
    interpolation on a grid 0.01 km/s apart), without calling ip_beta_kms."""
    c_kms = 299792.458
    for R in (1e5, 3e4):
        dv = 0.01
        n = 10001
        nu = 4350.0 * np.exp(np.arange(n) * dv / c_kms)   # log-uniform: uniform in velocity
        j0 = n // 2
        G = np.zeros(n)
        G[j0] = 1.0
        half_reach = int(1.5 * (c_kms / R) / dv)              # 1.5 FWHM either side
        idx = np.arange(j0 - half_reach, j0 + half_reach + 1)
        F = O.instrumental(G, nu, idx, R)[0]
        v = c_kms * np.log(nu[idx])
        k = int(np.argmax(F))
        assert idx[k] == j0
        h = 0.5 * F[k]
        i = k
        while F[i] > h:
            i += 1
        vr = v[i - 1] + (h - F[i - 1]) * (v[i] - v[i - 1]) / (F[i] - F[i - 1])
        i = k
        while F[i] > h:
            i -= 1
        vl = v[i] + (h - F[i]) * (v[i + 1] - v[i]) / (F[i + 1] - F[i])
        assert vr - vl == pytest.approx(c_kms / R, rel=2e-5)


def _q_table(nodes, Q):
    return np.concatenate([nodes, Q(nodes)])


def test_partition_table_interpolation_and_derivative():
    """Sec. 2.3: Q(T) tabulated on temperature nodes and interpolated linearly,
    q_r = Q(T)/Q(296).  The table samples Q = 41 (T/296)^1.5: exact at the
    nodes, the weighted mean of the two end values inside an interval, the end
    value held outside the nodes; d ln q_r/dT against central differences of
    ln q_r (inside intervals, below and above the nodes) and, at a node, the
    one-sided difference from the right."""
    tn = np.array([200.0, 296.0, 500.0, 800.0, 1200.0, 1700.0, 2400.0])
    Q = lambda T: 41.0 * (np.asarray(T, float) / 296.0) ** 1.5
    prm = _q_table(tn, Q)
    np.testing.assert_allclose(O.qr_ratio(tn, 1, prm), (tn / 296.0) ** 1.5, rtol=1e-14)
    for i in range(tn.size - 1):
        for f in (0.25, 0.5, 0.9):
            T = tn[i] + f * (tn[i + 1] - tn[i])
            expect = ((1 - f) * Q(tn[i]) + f * Q(tn[i + 1])) / Q(296.0)
            assert float(O.qr_ratio(T, 1, prm)) == pytest.approx(float(expect), rel=1e-13)
    assert float(O.qr_ratio(150.0, 1, prm)) == pytest.approx(float(Q(200.0) / Q(296.0)), rel=1e-14)
    assert float(O.qr_ratio(3000.0, 1, prm)) == pytest.approx(float(Q(2400.0) / Q(296.0)), rel=1e-14)
    lq = lambda T: math.log(float(O.qr_ratio(T, 1, prm)))
    h = 1e-3
    for T in (150.0, 250.0, 400.0, 1000.0, 2000.0, 2600.0, 5000.0):
        fd = (lq(T + h) - lq(T - h)) / (2 * h)
        assert float(O.dlog_qr_dT(T, 1, prm)) == pytest.approx(fd, rel=1e-7, abs=1e-13), T
    # at a node: q_r is linear on the interval to its right, so a forward
    # difference of q_r (not of ln q_r) is exact up to rounding
    q = lambda T: float(O.qr_ratio(T, 1, prm))
    for T in (200.0, 500.0, 2400.0):
        fd_right = (q(T + 1.0) - q(T)) / 1.0
        assert float(O.dlog_qr_dT(T, 1, prm)) * q(T) == pytest.approx(fd_right, rel=1e-10, abs=1e-15), T
    # a fine table converges to the power law and its log-derivative k/T
    fine = np.linspace(150.0, 3000.0, 4001)
    prm_f = _q_table(fine, Q)
    T = np.array([233.3, 777.7, 1999.9])
    np.testing.assert_allclose(O.qr_ratio(T, 1, prm_f), (T / 296.0) ** 1.5, rtol=2e-6)
    np.testing.assert_allclose(O.dlog_qr_dT(T, 1, prm_f), 1.5 / T, rtol=1e-3)


def test_strength_tangent_with_partition_table():
    """d ln S/dT (Eq. Slog) with a tabulated q_r against central differences of
    ln S, including temperatures outside the table where q_r is held."""
    from dataclasses import replace
    wl = synth.make_config(2, "tiny")
    tn = np.array([300.0, 600.0, 1000.0, 1500.0, 2000.0])
    ll = replace(wl.lines[0], qr_kind=1, qr_params=_q_table(tn, lambda T: 7.0 + 0.02 * np.asarray(T) ** 1.2))
    h = 1e-3
    for T in (250.0, 777.0, 1234.0, 2500.0):
        st = O.line_state(ll, T, 0.3)
        lp = np.log(O.line_state(ll, T + h, 0.3).S)
        lm = np.log(O.line_state(ll, T - h, 0.3).S)
        np.testing.assert_allclose(st.dlnS_dT, (lp - lm) / (2 * h), rtol=1e-6, atol=1e-12)


def test_sampled_tangents_equal_full_grid_tangents():
    """Without the response every grid point's column is independent, so the
    tangents at selected points equal those of the whole grid there."""
    from dataclasses import replace
    wl = replace(synth.make_config(4, "tiny"), response=None)
    idx = np.array([0, 5, 77, 300, wl.nu.size - 1])
    a = O.flux_tangents(wl, wl.theta, per_layer=True)
    b = O.flux_tangents(wl, wl.theta, per_layer=True, nu_idx=idx)
    np.testing.assert_array_equal(a["F"][idx], b["F"])
    np.testing.assert_array_equal(a["dF"][:, idx], b["dF"])
    np.testing.assert_array_equal(a["dF_dTn"][:, idx], b["dF_dTn"])
    with pytest.raises(ValueError):
        O.flux_tangents(synth.make_config(4, "tiny"), wl.theta, nu_idx=idx)
