"""Tabulated partition functions (EXO_QR_TABLE, Sec. 2.3: Q(T) interpolated
linearly on temperature nodes) through the C ABI, against the FP64 oracle.

The nodes (300-1800 K) leave the coldest layers of the power-law atmosphere
(~206 K at 1e-8 bar) below the table and the deepest (~2060 K) above it, so
the held end values and their zero log-derivative are exercised as well as
the interior intervals.  Tolerances as in the other parity tests: 1e-4 on
cross-sections and fluxes in FP32, 1e-5 in FP64, 1e-3 on gradients.
"""
import sys
from dataclasses import replace

import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

NODES = np.array([300.0, 420.0, 600.0, 900.0, 1300.0, 1800.0])


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def exo():
    import paper_2105_14782_amd as pkg
    pkg.load_library()
    from paper_2105_14782_amd import api
    return api


def _tabulate(ll, k):
    """The same list with Q(T) tabulated from a smooth curve that is not a power law."""
    Q = 30.0 + 0.05 * NODES ** k + 2e-5 * NODES ** 2
    return replace(ll, qr_kind=1, qr_params=np.concatenate([NODES, Q]))


def _workload(size):
    wl = synth.make_config(4, size)
    return replace(wl, lines=[_tabulate(wl.lines[0], 1.4), _tabulate(wl.lines[1], 1.0)])


def _ctx(exo, wl):
    c = exo.Context(0)
    for s, ll in enumerate(wl.lines):
        c.set_lines(s, ll)
    c.set_grid(wl.nu)
    return c


def maxrel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b) / np.abs(b)))


@pytest.mark.parametrize("T", [250.0, 777.0, 1300.0, 2200.0])
def test_cross_section_with_table(exo, T):
    wl = _workload("small")
    c = _ctx(exo, wl)
    for s, ll in enumerate(wl.lines):
        ref = O.cross_section(ll, T, 0.3, wl.nu)
        for prec, tol in [("fp32", 1e-4), ("fp64", 1e-5)]:
            got = c.cross_section(s, T, 0.3, prec).cpu().double().numpy()
            err = maxrel(got, ref)
            _say(f"  species {s} T={T} {prec}: max rel err {err:.2e}")
            assert err < tol, (s, T, prec, err)
    c.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_emission_with_table(exo, prec):
    wl = _workload("small")
    T = O.temperatures(wl.atmos.P_bar, wl.theta[0], wl.theta[1])
    assert T.min() < NODES[0] and T.max() > NODES[-1]
    c = _ctx(exo, wl)
    atm = exo.Atmos.from_workload(wl.atmos, [0, 1], wl.theta)
    resp = exo.Response.from_workload(wl.response, wl.theta)
    F = c.emission_flux(atm, resp, prec).cpu().double().numpy()
    ref = O.emission_flux(wl, wl.theta)
    err = maxrel(F, ref)
    _say(f"  emission {prec}: max rel err {err:.2e}")
    assert err < (1e-4 if prec == "fp32" else 1e-5)
    c.close()


def test_gradient_with_table(exo):
    """flux_vjp (all six parameters and every layer's dL/dT_n) against the
    oracle's gradient; the strength tangent d ln S/dT carries -d ln q_r/dT of
    the table, zero in the layers outside the nodes."""
    wl = _workload("small")
    th = wl.theta
    F_star = O.emission_flux(wl, wl.theta_star)
    rng = np.random.default_rng(4005)
    data = F_star * (1 + 0.01 * rng.normal(size=F_star.size))
    sigma = 0.01 * F_star
    c = _ctx(exo, wl)
    atm = exo.Atmos.from_workload(wl.atmos, [0, 1], th)
    resp = exo.Response.from_workload(wl.response, th)
    F = c.emission_flux(atm, resp, "fp32").double()
    cot = (-(torch.tensor(data, device="cuda") - F) / torch.tensor(sigma, device="cuda") ** 2).float().contiguous()
    g, gl, _ = c.flux_vjp(atm, resp, cot, want_layers=True)
    _, g_ref, gl_ref = O.loss_gradient(wl, th, data, sigma, per_layer=True)
    err = np.abs(g - g_ref) / np.maximum(np.abs(g_ref), 1e-6 * np.abs(g_ref).max())
    errl = np.abs(gl - gl_ref) / np.maximum(np.abs(gl_ref), 1e-6 * np.abs(gl_ref).max())
    _say(f"  grad rel err {err}; per-layer max rel err {errl.max():.2e}")
    assert np.all(err < 1e-3), (g, g_ref)
    assert errl.max() < 1e-3
    c.close()
