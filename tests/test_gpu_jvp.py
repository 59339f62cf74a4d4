"""Forward-mode derivatives (exo_flux_jvp) and the layer-by-layer temperature
model (Sec. 6.1) through the C ABI, against the FP64 oracle.

Tolerances: J dtheta per output point relative to max |J dtheta| (1e-3, the
gradient tolerance); gradients per component as in the VJP parity tests; the
dot-product identity <cot, J dtheta> = <J^T cot, dtheta> between the GPU's own
JVP and VJP to 1e-5 (both use the same FP32 Voigt tangents).
"""
import sys
from dataclasses import replace

import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

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


def _ctx(exo, wl):
    c = exo.Context(0)
    for s, ll in enumerate(wl.lines):
        c.set_lines(s, ll)
    c.set_grid(wl.nu)
    return c


def _inputs(exo, wl, th):
    atm = exo.Atmos.from_workload(wl.atmos, list(range(len(wl.lines))), th)
    resp = exo.Response.from_workload(wl.response, th) if wl.response is not None else None
    return atm, resp


def _rel(a, ref):
    a, ref = np.asarray(a, float), np.asarray(ref, float)
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def _dtheta(rng):
    return rng.normal(size=6) * np.array([5.0, 1e-3, 1e-2, 1e-2, 0.1, 0.1])


def _layer_profile(wl, th, seed):
    rng = np.random.default_rng(seed)
    T = O.temperatures(wl.atmos.P_bar, th[0], th[1])
    return T * (1 + 0.08 * rng.uniform(-1, 1, T.size))


def test_jvp_against_oracle(exo):
    _say("flux_jvp small vs oracle")
    wl = synth.make_config(4, "small")
    th = wl.theta
    c = _ctx(exo, wl)
    atm, resp = _inputs(exo, wl, th)
    dth = _dtheta(np.random.default_rng(1))
    F, dF = c.flux_jvp(atm, resp, dth)
    assert torch.equal(F.cpu(), c.emission_flux(atm, resp, "fp32").cpu())
    _, ref = O.flux_jvp(wl, th, dth)
    err = _rel(dF.cpu().double().numpy(), ref)
    _say(f"  J dtheta max rel err {err:.2e}")
    assert err < RTOL_GRAD


def test_jvp_single_directions_without_response(exo):
    """Each parameter direction alone on F0 (no response), against the oracle."""
    wl = replace(synth.make_config(4, "small"), response=None)
    th = wl.theta
    c = _ctx(exo, wl)
    atm, _ = _inputs(exo, wl, th)
    t = O.flux_tangents(wl, th)
    for k in range(4):
        e = np.zeros(6)
        e[k] = 1.0
        F, dF = c.flux_jvp(atm, None, e)
        err = _rel(dF.cpu().double().numpy(), t["dF"][k])
        _say(f"  direction {k}: max rel err {err:.2e}")
        assert err < RTOL_GRAD, k


def test_jvp_full_config2_against_fp64_differences(exo):
    """Full configuration-4 size (the config-2 atmosphere: 2 x 1e5 lines,
    20,000 points, 100 layers), in the launch shapes the bench times: the FP32
    forward-mode derivative along T0 and along alpha, which runs the tangent
    Voigt sums with the per-layer far reach and the far tier's cut tangent,
    against central differences of the plain FP64 spectrum (no FP32 tangent
    records involved).  The spectrum is far from linear in alpha at this size
    (near strong lines a step of 1e-4 already moves the central difference
    by 3-15 % of the derivative, and the oracle's own differences
    converge to its forward-mode tangent only below 1e-5), so the steps are
    0.01 K and 1e-6; the FP64 sums resolve such steps to ~1e-9 of the
    derivative.  Tolerance 1e-3 of max |J e_k|."""
    _say("flux_jvp full config-2 size vs FP64 central differences")
    wl = synth.make_config(4, "full")
    th = np.array(wl.theta, dtype=float)
    c = _ctx(exo, wl)
    for k, h in [(0, 0.01), (1, 1e-6)]:
        e = np.zeros(6)
        e[k] = 1.0
        atm, resp = _inputs(exo, wl, th)
        _, dF = c.flux_jvp(atm, resp, e)
        Fs = []
        for sgn in (1.0, -1.0):
            atm_s, resp_s = _inputs(exo, wl, th + sgn * h * e)
            Fs.append(c.emission_flux(atm_s, resp_s, "fp64").cpu().numpy())
        fd = (Fs[0] - Fs[1]) / (2.0 * h)
        err = _rel(dF.cpu().double().numpy(), fd)
        _say(f"  direction {k}: max rel err {err:.2e}")
        assert err < RTOL_GRAD, (k, err)
    c.close()


def test_full_config4_sampled_derivatives_against_oracle(exo):
    """Full configuration-4 size (2 x 1e5 lines, 20,000 points, 100 layers) in
    the bench's launch shapes, without the response so that every grid
    point's column is independent: J e_k along T0, alpha and both mixing
    ratios at 64 sampled points (both ends and 62 random ones), and the VJP of
    a cotangent carried by those points (every parameter and every layer's
    dL/dT_n), against the oracle's forward-mode tangents at those points."""
    _say("full config-4 size, sampled points: JVP and VJP vs oracle")
    wl = replace(synth.make_config(4, "full"), response=None)
    th = np.array(wl.theta, dtype=float)
    c = _ctx(exo, wl)
    atm, _ = _inputs(exo, wl, th)
    rng = np.random.default_rng(2027)
    ng = wl.nu.size
    idx = np.concatenate([[0], np.sort(rng.choice(np.arange(1, ng - 1), 62, replace=False)), [ng - 1]])
    t = O.flux_tangents(wl, th, per_layer=True, nu_idx=idx)
    for k in range(4):
        e = np.zeros(6)
        e[k] = 1.0
        _, dF = c.flux_jvp(atm, None, e, want_flux=False)
        err = _rel(dF.cpu().double().numpy()[idx], t["dF"][k])
        _say(f"  J e_{k}: max rel err {err:.2e}")
        assert err < RTOL_GRAD, (k, err)
    cot = np.zeros(ng)
    cot[idx] = rng.normal(size=idx.size)
    g, gl, _ = c.flux_vjp(atm, None, torch.tensor(cot, dtype=torch.float32, device="cuda"), want_layers=True)
    g_ref = t["dF"][:4] @ cot[idx]
    gl_ref = t["dF_dTn"] @ cot[idx]
    err = np.abs(g[:4] - g_ref) / np.maximum(np.abs(g_ref), 1e-6 * np.abs(g_ref).max())
    errl = np.abs(gl - gl_ref) / np.maximum(np.abs(gl_ref), 1e-6 * np.abs(gl_ref).max())
    _say(f"  VJP rel err {err}; per-layer max rel err {errl.max():.2e}")
    assert np.all(err < RTOL_GRAD), (g, g_ref)
    assert errl.max() < RTOL_GRAD
    c.close()


def test_jvp_vjp_dot_product(exo):
    wl = synth.make_config(4, "small")
    th = wl.theta
    c = _ctx(exo, wl)
    atm, resp = _inputs(exo, wl, th)
    rng = np.random.default_rng(2)
    dth = _dtheta(rng)
    dT = rng.normal(size=wl.atmos.P_bar.size) * 2.0
    cot = torch.tensor(rng.normal(size=resp.out_len), dtype=torch.float32, device="cuda")
    _, dF = c.flux_jvp(atm, resp, dth, dT, want_flux=False)
    g, gl, _ = c.flux_vjp(atm, resp, cot, want_layers=True)
    lhs = float(torch.dot(cot.double(), dF.double()))
    rhs = float(np.dot(g, dth) + np.dot(gl, dT))
    _say(f"  <cot, J dth> = {lhs:.10e}, <J^T cot, dth> = {rhs:.10e}")
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs))


def test_layer_profile_equal_to_power_law(exo):
    wl = synth.make_config(4, "small")
    th = wl.theta
    c = _ctx(exo, wl)
    atm, resp = _inputs(exo, wl, th)
    T = O.temperatures(wl.atmos.P_bar, th[0], th[1])
    F_pl = c.emission_flux(atm, resp, "fp32").cpu().double().numpy()
    F_l = c.emission_flux(replace(atm, T_layers=T), resp, "fp32").cpu().double().numpy()
    assert _rel(F_l, F_pl) < 1e-6


def test_layer_profile_gradients_against_oracle(exo):
    """VJP (per-layer gradient) and JVP (per-layer direction) of a
    non-monotonic layer-by-layer profile."""
    _say("layer-by-layer profile: VJP and JVP vs oracle")
    wl = synth.make_config(4, "small")
    th = wl.theta
    T = _layer_profile(wl, th, 5)
    wl_l = replace(wl, atmos=replace(wl.atmos, T_layers=T))
    c = _ctx(exo, wl_l)
    atm, resp = _inputs(exo, wl_l, th)
    assert atm.T_layers is not None
    t = O.flux_tangents(wl_l, th, per_layer=True)
    F_star = t["F"]
    rng = np.random.default_rng(6)
    data = F_star * (1 + 0.01 * rng.normal(size=F_star.size))
    sigma = 0.01 * F_star

    def rel(g, g_ref):
        return np.abs(g - g_ref) / np.maximum(np.abs(g_ref), 1e-6 * np.abs(g_ref).max())

    # the VJP itself: one FP32 cotangent (the likelihood's at the oracle's
    # flux) given to both sides
    cot32 = (-(data - F_star) / sigma ** 2).astype(np.float32)
    g, gl, _ = c.flux_vjp(atm, resp, torch.tensor(cot32, device="cuda"), want_layers=True)
    g_ref, gl_ref = t["dF"] @ cot32.astype(np.float64), t["dF_dTn"] @ cot32.astype(np.float64)
    assert g[0] == 0.0 and g[1] == 0.0
    _say(f"  same cotangent: per-layer gradient max rel err {rel(gl, gl_ref).max():.2e}, "
         f"theta {rel(g[2:], g_ref[2:]).max():.2e}")
    assert np.all(rel(g[2:], g_ref[2:]) < RTOL_GRAD), (g, g_ref)
    assert np.max(rel(gl, gl_ref)) < RTOL_GRAD
    # the loss gradient end to end: each side forms the residual from its own
    # flux.  The FP32 flux error (~1e-7 of F) enters the residual (1e-2 of F)
    # with the same sign pattern at every point, while the residual's noise
    # cancels in sum_j cot_j dF_j/dT_n, so this error is the larger one.
    F = c.emission_flux(atm, resp, "fp32").double()
    cot = (-(torch.tensor(data, device="cuda") - F) / torch.tensor(sigma, device="cuda") ** 2).float()
    g, gl, _ = c.flux_vjp(atm, resp, cot.contiguous(), want_layers=True)
    _, g_ref, gl_ref = O.loss_gradient(wl_l, th, data, sigma, per_layer=True)
    _say(f"  loss gradient end to end: per-layer max rel err {rel(gl, gl_ref).max():.2e}, "
         f"theta {rel(g[2:], g_ref[2:]).max():.2e}")
    assert np.all(rel(g[2:], g_ref[2:]) < RTOL_GRAD), (g, g_ref)
    assert np.max(rel(gl, gl_ref)) < RTOL_GRAD
    dT = rng.normal(size=T.size) * 3.0
    dth = _dtheta(rng)
    _, dF = c.flux_jvp(atm, resp, dth, dT, want_flux=False)
    _, ref = O.flux_jvp(wl_l, th, dth, dT)
    err = _rel(dF.cpu().double().numpy(), ref)
    _say(f"  J (dtheta, dT) max rel err {err:.2e}")
    assert err < RTOL_GRAD


def test_forward_mode_autograd(exo):
    import torch.autograd.forward_ad as fwAD
    wl = synth.make_config(4, "tiny")
    th = wl.theta
    c = _ctx(exo, wl)
    atm, resp = _inputs(exo, wl, None)
    dth = _dtheta(np.random.default_rng(7))
    with fwAD.dual_level():
        theta = fwAD.make_dual(torch.tensor(th, dtype=torch.float64), torch.tensor(dth))
        F = exo.EmissionFlux.apply(theta, c, atm, resp)
        dF = fwAD.unpack_dual(F).tangent
    _, ref = O.flux_jvp(wl, th, dth)
    assert _rel(dF.cpu().double().numpy(), ref) < RTOL_GRAD


def test_layer_autograd_function(exo):
    """LayerEmissionFlux: backward gives dL/dT_n and dL/dphi, forward mode J (dT, dphi)."""
    import torch.autograd.forward_ad as fwAD
    wl = synth.make_config(4, "tiny")
    th = wl.theta
    T = _layer_profile(wl, th, 9)
    wl_l = replace(wl, atmos=replace(wl.atmos, T_layers=T))
    c = _ctx(exo, wl_l)
    atm, resp = _inputs(exo, wl_l, None)
    F_star = O.emission_flux(wl_l, th)
    rng = np.random.default_rng(10)
    data = F_star * (1 + 0.01 * rng.normal(size=F_star.size))
    sigma = 0.01 * F_star
    Tt = torch.tensor(T, dtype=torch.float64, requires_grad=True)
    phi = torch.tensor(th[2:], dtype=torch.float64, requires_grad=True)
    F = exo.LayerEmissionFlux.apply(Tt, phi, c, atm, resp)
    d = torch.tensor(data, device="cuda", dtype=torch.float32)
    s = torch.tensor(sigma, device="cuda", dtype=torch.float32)
    (0.5 * torch.sum(((d - F) / s) ** 2)).backward()
    _, g_ref, gl_ref = O.loss_gradient(wl_l, th, data, sigma, per_layer=True)
    errl = np.abs(Tt.grad.numpy() - gl_ref) / np.maximum(np.abs(gl_ref), 1e-6 * np.abs(gl_ref).max())
    _say(f"  LayerEmissionFlux backward: per-layer max rel err {errl.max():.2e}")
    assert errl.max() < RTOL_GRAD
    errp = np.abs(phi.grad.numpy() - g_ref[2:]) / np.maximum(np.abs(g_ref[2:]), 1e-6 * np.abs(g_ref[2:]).max())
    _say(f"  LayerEmissionFlux backward: mixing-ratio max rel err {errp.max():.2e}")
    assert errp.max() < RTOL_GRAD
    dT = rng.normal(size=T.size) * 3.0
    dphi = np.array([1e-2, -1e-2, 0.1, 0.1])
    with fwAD.dual_level():
        Td = fwAD.make_dual(torch.tensor(T), torch.tensor(dT))
        pd = fwAD.make_dual(torch.tensor(th[2:]), torch.tensor(dphi))
        dF = fwAD.unpack_dual(exo.LayerEmissionFlux.apply(Td, pd, c, atm, resp)).tangent
    _, ref = O.flux_jvp(wl_l, th, np.concatenate([[0.0, 0.0], dphi]), dT)
    assert _rel(dF.cpu().double().numpy(), ref) < RTOL_GRAD


def test_jvp_and_layer_profile_errors(exo):
    import paper_2105_14782_amd as pkg
    wl = synth.make_config(4, "tiny")
    th = wl.theta
    c = _ctx(exo, wl)
    atm, resp = _inputs(exo, wl, th)
    with pytest.raises(pkg.ExoError) as e:
        c.emission_flux(replace(atm, T_layers=np.full(wl.atmos.P_bar.size, 0.5)), resp)
    assert e.value.code == pkg.EXO_EINVAL
    bad = np.zeros(6)
    bad[3] = np.nan
    with pytest.raises(pkg.ExoError) as e:
        c.flux_jvp(atm, resp, bad)
    assert e.value.code == pkg.EXO_EINVAL
    with pytest.raises(pkg.ExoError) as e:
        c.flux_jvp(replace(atm, P_bar=np.logspace(-8, 2, 5000)), resp, np.zeros(6))
    assert e.value.code == pkg.EXO_EINVAL
