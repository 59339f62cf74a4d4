"""Weak-line pre-selection (App. G) on the GPU against its oracle.

The keep mask is an integer decision taken from FP64 arithmetic on both
sides, so it must match exactly, except where the oracle's own contribution
function has two layers within 1e-12 (relative) of each other at the top:
there either argmax is correct, and the test checks that the GPU's choice is
one of them.
"""
import math
import sys
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import oracle as O
from oracle import selection as SEL

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def exo():
    import paper_2105_14782_amd as pkg
    pkg.load_library()
    from paper_2105_14782_amd import api
    return api


def _lines(rng, n, mass, gnat=False):
    # deliberately not sorted: the mask must come back in the caller's order
    return synth.LineList(rng.uniform(4340, 4380, n), 10 ** rng.uniform(-28, -18, n), rng.exponential(3000, n),
                          rng.uniform(0.01, 0.1, n), rng.uniform(0.5, 0.8, n), mass, 0,
                          np.array([1.5 if mass == 18.0 else 1.0]),
                          gamma_nat=rng.uniform(0, 1e-3, n) if gnat else None)


def _near_ties(psi, rtol=1e-12):
    s = np.sort(psi, axis=0)
    return (s[-1] - s[-2]) <= rtol * s[-1]


def _check(exo, ll, atm, lx, T_atm, T_strength, margin):
    c = exo.Context(0)
    c.set_lines(0, ll)
    a = exo.Atmos.from_workload(atm, [0])
    keep, n_kept = c.select_lines(0, lx, a, T_atm, T_strength, margin)
    keep = keep.cpu().numpy().astype(bool)
    ref, n_line, n_cia = SEL.select_lines(ll, lx, atm, T_atm, T_strength, margin)
    assert n_kept == int(keep.sum())
    bad = np.nonzero(keep != ref)[0]
    if bad.size:
        P = np.asarray(atm.P_bar, float)
        dP = O.layer_dP_bar(P)
        Ts = [T_atm] if T_strength is None else T_strength
        _, psi = SEL.contribution_argmax(SEL.line_centre_dtau(ll, lx, atm, T_atm, Ts), P, dP)
        dc = np.stack([O.dtau_cia(T_atm, P[n], dP[n], np.asarray(ll.nu_c), atm) for n in range(P.size)])
        _, psic = SEL.contribution_argmax(dc, P, dP)
        amb = _near_ties(psi) | _near_ties(psic)
        assert amb[bad].all(), (bad[~amb[bad]], n_line[bad], n_cia[bad])
    _say(f"  kept {n_kept} of {ll.n} (mismatches at near-ties: {bad.size})")
    return keep


@pytest.mark.parametrize("mass,margin", [(18.0, 2), (28.0, 2), (18.0, 0), (28.0, 5)])
def test_selection_matches_oracle(exo, mass, margin):
    rng = np.random.default_rng(int(mass) + margin)
    ll = _lines(rng, 20000, mass)
    atm = synth.make_config(2, "tiny").atmos
    atm = replace(atm, P_bar=np.logspace(-8, 2, 100))
    _check(exo, ll, atm, math.log10(0.0058), 1700.0, np.arange(500.0, 1701.0, 100.0), margin)


def test_selection_single_temperature_natural_width_other_grid(exo):
    rng = np.random.default_rng(7)
    ll = _lines(rng, 5000, 18.0, gnat=True)
    atm = replace(synth.make_config(2, "tiny").atmos, P_bar=np.logspace(-5, 1.5, 37), g_cgs=10 ** 4.5)
    keep = _check(exo, ll, atm, math.log10(0.0023), 1300.0, None, 2)
    assert 0 < keep.sum() < ll.n


def test_selection_errors(exo):
    import paper_2105_14782_amd as pkg
    rng = np.random.default_rng(8)
    c = exo.Context(0)
    c.set_lines(0, _lines(rng, 100, 18.0))
    a = exo.Atmos.from_workload(synth.make_config(2, "tiny").atmos, [0])
    for kw in (dict(T_atm=0.5), dict(T_atm=1000.0, margin=-1), dict(T_atm=1000.0, T_strength=[0.0])):
        with pytest.raises(pkg.ExoError) as e:
            c.select_lines(0, -3.0, a, **kw)
        assert e.value.code == pkg.EXO_EINVAL
    with pytest.raises(pkg.ExoError) as e:
        c.select_lines(1, -3.0, a, 1000.0)
    assert e.value.code == pkg.EXO_ENOTSET


def test_selection_full_config3_sampled(exo):
    """The full 1e7-line config-3 list on its 100-layer atmosphere, as the
    bench selects it (isothermal 1700 K, strengths scanned over 500-1700 K,
    margin 2): the GPU mask of 20,000 random lines against the oracle's
    selection of those lines (each line's decision depends on that line
    alone)."""
    wl = synth.make_config(3, "full")
    full = wl.lines[0]
    c = exo.Context(0)
    c.set_lines(0, full)
    a = exo.Atmos.from_workload(wl.atmos, [0])
    T_scan = np.arange(500.0, 1701.0, 100.0)
    lx = math.log10(0.0023)
    keep, n_kept = c.select_lines(0, lx, a, 1700.0, T_scan, 2)
    keep = keep.cpu().numpy().astype(bool)
    assert n_kept == int(keep.sum())
    idx = np.sort(np.random.default_rng(303).choice(full.n, 20000, replace=False))
    sub = replace(full, nu_c=full.nu_c[idx], S0=full.S0[idx], E_low=full.E_low[idx],
                  alpha_ref=full.alpha_ref[idx], n_texp=full.n_texp[idx])
    ref, _, _ = SEL.select_lines(sub, lx, wl.atmos, 1700.0, T_scan, 2)
    bad = np.nonzero(keep[idx] != ref)[0]
    if bad.size:
        P = np.asarray(wl.atmos.P_bar, float)
        dP = O.layer_dP_bar(P)
        sb = replace(sub, nu_c=sub.nu_c[bad], S0=sub.S0[bad], E_low=sub.E_low[bad],
                     alpha_ref=sub.alpha_ref[bad], n_texp=sub.n_texp[bad])
        _, psi = SEL.contribution_argmax(SEL.line_centre_dtau(sb, lx, wl.atmos, 1700.0, T_scan), P, dP)
        dc = np.stack([O.dtau_cia(1700.0, P[n], dP[n], np.asarray(sb.nu_c), wl.atmos) for n in range(P.size)])
        _, psic = SEL.contribution_argmax(dc, P, dP)
        assert (_near_ties(psi) | _near_ties(psic)).all(), bad
    _say(f"  kept {n_kept} of {full.n}; sampled 20000: {int(ref.sum())} kept by the oracle, "
         f"mismatches at near-ties: {bad.size}")
    c.close()
