"""Plain FP64 CPU oracle of the weak-line pre-selection of App. G: which lines
can affect the emission spectrum, judged by where their line-centre
contribution function peaks relative to that of the H2-H2 continuum.

TEST INFRASTRUCTURE ONLY, like ``oracle.oracle``.

Steps, in the appendix's order:

1. An isothermal atmosphere at T_atm on the pressure grid; every line gets
   the strength S_eff = max over a list of temperatures of S(T) (the paper
   scans 500-1700 K for water; a single temperature reproduces its CO case).
2. The line-centre optical depth of the line alone in layer n,
   dtau_n = dP_n/(m_u g) X/M S_eff/(sqrt(2 pi) beta) erfcx(gamma_n/(sqrt2 beta)),
   with beta at T_atm and gamma_n at (T_atm, P_n); tau_n = sum_{k <= n} dtau_k.
3. The contribution function psi_n = e^{-tau_n} dtau_n P_n / dP_n (the Planck
   factor is the same in every layer of an isothermal atmosphere) and its
   argmax n_line (the first one on ties).
4. The same for the continuum at the line centre, n_CIA.
5. Keep the line iff n_line <= n_CIA + margin.

Readings (also the HIP path's): tau_n includes layer n; "the CIA line minus
two layers" is read as a margin of two layers on the side of keeping lines,
i.e. a line whose contribution peaks up to two layers below the continuum's
is kept.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from .oracle import (column_factor, doppler_beta, dtau_cia, layer_dP_bar, line_strength,
                     lorentz_gamma, qr_ratio)


def contribution_argmax(dtau, P, dP):
    """argmax_n of e^{-tau_n} dtau_n P_n / dP_n over the layer axis (axis 0)."""
    tau = np.cumsum(dtau, axis=0)
    psi = np.exp(-tau) * dtau * (np.asarray(P) / np.asarray(dP))[:, None]
    return np.argmax(psi, axis=0), psi


def line_centre_dtau(ll, log10_mmr, atm, T_atm, T_strength):
    """[layer, line] line-centre optical depth of each line alone."""
    P = np.asarray(atm.P_bar, float)
    dP = layer_dP_bar(P)
    nu_c = np.asarray(ll.nu_c, float)
    S = np.max([line_strength(ll.S0, ll.E_low, nu_c, T, qr_ratio(T, ll.qr_kind, ll.qr_params))
                for T in T_strength], axis=0)
    beta = doppler_beta(nu_c, T_atm, ll.mass_amu)
    col = column_factor(dP, 10.0 ** log10_mmr, ll.mass_amu, atm.g_cgs)
    out = np.empty((P.size, nu_c.size))
    for n in range(P.size):
        gam = lorentz_gamma(ll.alpha_ref, ll.n_texp, T_atm, P[n])
        if ll.gamma_nat is not None:
            gam = gam + ll.gamma_nat
        out[n] = col[n] * S / (math.sqrt(2.0 * math.pi) * beta) * special.erfcx(gam / (math.sqrt(2.0) * beta))
    return out


def select_lines(ll, log10_mmr, atm, T_atm, T_strength=None, margin=2):
    """Boolean mask over the lines (in the order given) of the lines kept, and
    the two argmax layers per line."""
    T_strength = [T_atm] if T_strength is None else list(T_strength)
    P = np.asarray(atm.P_bar, float)
    dP = layer_dP_bar(P)
    dtau = line_centre_dtau(ll, log10_mmr, atm, T_atm, T_strength)
    n_line, _ = contribution_argmax(dtau, P, dP)
    nu_c = np.asarray(ll.nu_c, float)
    dcia = np.stack([dtau_cia(T_atm, P[n], dP[n], nu_c, atm) for n in range(P.size)])
    n_cia, _ = contribution_argmax(dcia, P, dP)
    return n_line <= n_cia + margin, n_line, n_cia
