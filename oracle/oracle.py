"""Plain FP64 CPU oracle of the direct line-by-line emission spectrum model.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  The product
path (the HIP library and its Python binding) never calls it, and this module
imports nothing from the product path.

Everything is written from the definitions in arXiv:2105.14782 (Kawahara et
al., "Auto-differentiable spectrum model for high-dispersion characterization
of exoplanets and brown dwarfs"), in float64, without tiling, fusion or
approximation beyond what the definitions state:

* The Voigt profile is taken from its definition as the real part of the
  Faddeeva function (Sec. 2.1.1, Eq. crosssec and the H = Re w identity) using
  ``scipy.special.wofz`` as the library primitive, *not* the paper's
  Algorithm-916/asymptotic approximation ("hjert") that the GPU evaluates.
* The transmission uses the exact exponential integral (``scipy.special.expn``)
  in T = 2 E3(dtau) (Eq. trans), not the AS70 fit.
* Radiative transfer is the plain recurrence of Eq. rerr, bottom to top.
* The response is the direct sum of Eq. responsenu with the rotation kernel
  integrated from its stated limb-darkened definition (Sec. 4.1).
* Gradients are forward-mode tangents written out step by step.

Readings of points the paper leaves open or prints inconsistently (they are
also the HIP path's readings):

* Bottom boundary F_B = pi B(T of the deepest layer) (or zero on request).
* Layer thickness dP_n = P_n - P_{n-1} with P_{-1} = P_0^2 / P_1.
* Rotation kernel: closed form of the limb-darkened disk integral (the printed
  u2 terms do not integrate to one); response normalised by the sum of the
  same, velocity-shifted taps; IP Gaussian truncated at 6 sigma.
* c2 = h c / k_B from the exact SI constants.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
from scipy import special

# ---------------------------------------------------------------------------
# Constants (cgs).  Exact SI definitions of h, c, k_B; CODATA 2018 m_u.
# ---------------------------------------------------------------------------
H_PLANCK = 6.62607015e-27          # erg s
C_LIGHT = 2.99792458e10            # cm s^-1
K_BOLTZ = 1.380649e-16             # erg K^-1
M_U = 1.66053906660e-24            # g
C2 = H_PLANCK * C_LIGHT / K_BOLTZ  # cm K   (second radiation constant)
T_REF = 296.0                      # K (HITRAN/ExoMol reference temperature)
BAR = 1.0e6                        # dyn cm^-2
C_KMS = 2.99792458e5               # km s^-1
SQRT_PI = math.sqrt(math.pi)

def _default_threads():
    """Threads for the chunked sums: the CPUs this process may run on, at most
    16 (a one-GPU host's share of its CPUs)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


N_THREADS = int(os.environ.get("ORACLE_THREADS", _default_threads()))


def _pool_map(fn, items):
    items = list(items)
    if N_THREADS <= 1 or len(items) <= 1:
        return [fn(it) for it in items]
    with ThreadPoolExecutor(max_workers=N_THREADS) as ex:
        return list(ex.map(fn, items))


# ---------------------------------------------------------------------------
# Faddeeva / Voigt (Sec. 2.1.1)
# ---------------------------------------------------------------------------

def faddeeva(z):
    """w(z) = exp(-z^2) erfc(-i z) (library primitive)."""
    return special.wofz(np.asarray(z, dtype=np.complex128))


def voigt_hjerting(x, a):
    """H(x, a) = Re w(x + i a)."""
    return faddeeva(np.asarray(x, float) + 1j * np.asarray(a, float)).real


def voigt_profile(dnu, beta, gamma):
    """Normalised Voigt profile V(dnu; beta, gamma_L), Eq. crosssec.

    beta is the Gaussian standard deviation, gamma the Lorentzian HWHM:
    V = Re w(z) / (sqrt(2 pi) beta),  z = (dnu + i gamma) / (sqrt(2) beta).
    """
    dnu = np.asarray(dnu, float)
    z = (dnu + 1j * gamma) / (math.sqrt(2.0) * beta)
    return faddeeva(z).real / (math.sqrt(2.0 * math.pi) * beta)


# ---------------------------------------------------------------------------
# Line parameters (Sec. 2.1.1 Eq. thermal, Sec. 2.2 Eq. Slog, Eq. gammaexomol,
# Eq. naturalgamma, Sec. 2.3 partition function)
# ---------------------------------------------------------------------------

def qr_ratio(T, kind: int, params):
    """q_r(T) = Q(T)/Q(T_ref) (Sec. 2.3: Q interpolated on a grid of temperatures).

    kind 0: (T/T_ref)^k with params = [k].
    kind 1: linear interpolation of a Q(T) table, params = [T_0..T_{n-1}, Q_0..Q_{n-1}];
    outside [T_0, T_{n-1}] the end value is held (np.interp).
    """
    T = np.asarray(T, float)
    params = np.asarray(params, float)
    if kind == 0:
        return (T / T_REF) ** params[0]
    n = params.size // 2
    tn, qn = params[:n], params[n:]
    return np.interp(T, tn, qn) / np.interp(T_REF, tn, qn)


def dlog_qr_dT(T, kind: int, params):
    """d ln q_r / dT of qr_ratio.  For the table, the derivative from the right:
    the slope of the interval [T_i, T_{i+1}) holding T, and zero where the end
    value is held (T < T_0 or T >= T_{n-1})."""
    T = np.asarray(T, float)
    params = np.asarray(params, float)
    if kind == 0:
        return params[0] / T
    n = params.size // 2
    tn, qn = params[:n], params[n:]
    i = np.clip(np.searchsorted(tn, T, side="right") - 1, 0, n - 2)
    slope = (qn[i + 1] - qn[i]) / (tn[i + 1] - tn[i])
    slope = np.where((T >= tn[0]) & (T < tn[-1]), slope, 0.0)
    return slope / np.interp(T, tn, qn)


def line_strength(S0, E_low, nu_c, T, qr):
    """S(T) of Eq. Slog: S0 / q_r * exp(-c2 E (1/T - 1/Tref)) * stim(T)/stim(Tref)."""
    S0 = np.asarray(S0, float)
    boltz = np.exp(-C2 * np.asarray(E_low, float) * (1.0 / T - 1.0 / T_REF))
    stim = (1.0 - np.exp(-C2 * nu_c / T)) / (1.0 - np.exp(-C2 * nu_c / T_REF))
    return S0 / qr * boltz * stim


def dlog_line_strength_dT(E_low, nu_c, T, dlogqr):
    """d ln S / dT for Eq. Slog."""
    e = np.exp(-C2 * nu_c / T)
    return -dlogqr + C2 * np.asarray(E_low, float) / T ** 2 - (C2 * nu_c / T ** 2) * e / (1.0 - e)


def doppler_beta(nu_c, T, mass_amu):
    """Thermal Gaussian standard deviation, Eq. thermal."""
    return np.sqrt(K_BOLTZ * T / (mass_amu * M_U)) * np.asarray(nu_c, float) / C_LIGHT


def lorentz_gamma(alpha_ref, n_texp, T, P_bar, gamma_nat=None):
    """gamma_L = alpha_ref (T/Tref)^-n (P / 1 bar) + gamma_nat (Eq. gammaexomol, naturalgamma)."""
    g = np.asarray(alpha_ref, float) * (T / T_REF) ** (-np.asarray(n_texp, float)) * P_bar
    if gamma_nat is not None:
        g = g + gamma_nat
    return g


@dataclass
class LineState:
    """Per-line quantities of one absorber at one (T, P)."""
    S: np.ndarray
    beta: np.ndarray
    gamma: np.ndarray
    dlnS_dT: np.ndarray
    dbeta_dT: np.ndarray
    dgamma_dT: np.ndarray


def line_state(ll, T: float, P_bar: float) -> LineState:
    qr = qr_ratio(T, ll.qr_kind, ll.qr_params)
    S = line_strength(ll.S0, ll.E_low, ll.nu_c, T, qr)
    beta = doppler_beta(ll.nu_c, T, ll.mass_amu)
    gp = lorentz_gamma(ll.alpha_ref, ll.n_texp, T, P_bar)
    gamma = gp + (ll.gamma_nat if ll.gamma_nat is not None else 0.0)
    dlnS = dlog_line_strength_dT(ll.E_low, ll.nu_c, T, dlog_qr_dT(T, ll.qr_kind, ll.qr_params))
    return LineState(S, beta, gamma, dlnS, beta / (2.0 * T), -np.asarray(ll.n_texp) * gp / T)


# ---------------------------------------------------------------------------
# Cross-section: direct line-by-line sum (Sec. 2.1.1 direct LPF, Sec. 3.1)
# ---------------------------------------------------------------------------
_LINE_CHUNK = 4096


def _xs_chunk(args):
    nu, nu_c, st, lo, hi, want_dT = args
    dnu = nu[None, :] - nu_c[lo:hi, None]
    beta = st.beta[lo:hi, None]
    gam = st.gamma[lo:hi, None]
    S = st.S[lo:hi, None]
    z = (dnu + 1j * gam) / (math.sqrt(2.0) * beta)
    w = faddeeva(z)
    k = 1.0 / (math.sqrt(2.0 * math.pi) * beta)
    V = w.real * k
    sig = np.sum(S * V, axis=0)
    if not want_dT:
        return sig, None
    # dV/dT with w'(z) = -2 z w + 2i/sqrt(pi) and z = (dnu + i gamma)/(sqrt2 beta)
    rb = st.dbeta_dT[lo:hi, None] / beta
    dz = 1j * st.dgamma_dT[lo:hi, None] / (math.sqrt(2.0) * beta) - z * rb
    wp = -2.0 * z * w + 2j / SQRT_PI
    dV = (wp * dz).real * k - V * rb
    dsig = np.sum(S * (st.dlnS_dT[lo:hi, None] * V + dV), axis=0)
    return sig, dsig


def cross_section(ll, T: float, P_bar: float, nu, want_dT: bool = False, parallel: bool = True):
    """sigma(nu_j) = sum_l S_l V(nu_j - nu_l; beta_l, gamma_l)  [cm^2 / molecule].

    With want_dT also returns d sigma / dT at fixed P.  The lines go in chunks
    (threads over chunks unless parallel is False); the chunk sums are added
    in chunk order either way.
    """
    nu = np.asarray(nu, float)
    st = line_state(ll, T, P_bar)
    nu_c = np.asarray(ll.nu_c, float)
    chunk = max(1, min(_LINE_CHUNK, int(2e6 // max(nu.size, 1))))
    tasks = [(nu, nu_c, st, lo, min(lo + chunk, ll.n), want_dT) for lo in range(0, ll.n, chunk)]
    parts = _pool_map(_xs_chunk, tasks) if parallel else [_xs_chunk(t) for t in tasks]
    sig = np.sum(np.stack([p[0] for p in parts]), axis=0)
    if not want_dT:
        return sig
    dsig = np.sum(np.stack([p[1] for p in parts]), axis=0)
    return sig, dsig


# ---------------------------------------------------------------------------
# Atmosphere, optical depth, CIA, Planck (Sec. 2.4, Sec. 3)
# ---------------------------------------------------------------------------

def temperatures(P_bar, T0, alpha):
    """Power-law T-P profile T = T0 (P / 1 bar)^alpha (Sec. 5.2)."""
    return T0 * np.asarray(P_bar, float) ** alpha


def layer_temperatures(atm, T0, alpha):
    """T_n of every layer: the atmosphere's own layer-by-layer profile when it
    has one (the layer-by-layer temperature model of Sec. 6.1), else the
    power law in (T0, alpha)."""
    if getattr(atm, "T_layers", None) is not None:
        return np.asarray(atm.T_layers, float).copy()
    return temperatures(atm.P_bar, T0, alpha)


def layer_dP_bar(P_bar):
    """dP_n = P_n - P_{n-1}, with P_{-1} = P_0^2/P_1 (the top layer keeps the grid ratio)."""
    P = np.asarray(P_bar, float)
    prev = np.concatenate([[P[0] * P[0] / P[1]], P[:-1]])
    return P - prev


def column_factor(dP_bar, mmr, mass_amu, g_cgs):
    """dP/(m_u g) * X/M (Eq. dtau_line2) [molecules cm^-2]."""
    return np.asarray(dP_bar) * BAR / (M_U * g_cgs) * mmr / mass_amu


def cia_coefficient(T, nu, alpha0, Tpow, slope, nu_c):
    """Synthetic smooth H2-H2 absorption coefficient [cm^5]."""
    return alpha0 * (T / 1000.0) ** Tpow * np.exp(slope * (np.asarray(nu) - nu_c) / 40.0)


def dtau_cia(T, P_bar, dP_bar, nu, atm):
    """Eq. taucont with Eq. scaleheight: xi^2 P dP alpha / (k_B T mu m_u g)."""
    a = cia_coefficient(T, nu, atm.cia_alpha0, atm.cia_Tpow, atm.cia_slope, atm.cia_nu_c)
    return atm.vmr_h2 ** 2 * (P_bar * BAR) * (dP_bar * BAR) * a / (K_BOLTZ * T * atm.mmw * M_U * atm.g_cgs)


def planck_pi(T, nu):
    """pi B_nu(T) in erg s^-1 cm^-2 (cm^-1)^-1 (Eq. sourcepla)."""
    nu = np.asarray(nu, float)
    return math.pi * 2.0 * H_PLANCK * C_LIGHT ** 2 * nu ** 3 / np.expm1(C2 * nu / T)


def dplanck_pi_dT(T, nu):
    nu = np.asarray(nu, float)
    x = C2 * nu / T
    return planck_pi(T, nu) * (x / T) * np.exp(x) / np.expm1(x)


def transmission(dtau):
    """T = 2 E3(dtau) (Eq. trans), T(0) = 1."""
    return 2.0 * special.expn(3, np.asarray(dtau, float))


def dtransmission(dtau):
    """dT/d(dtau) = -2 E2(dtau)."""
    return -2.0 * special.expn(2, np.asarray(dtau, float))


def rt_recurrence(dtau, S, F_B):
    """Upward recurrence F_n = T_n F_{n+1} + (1 - T_n) S_n from F_N = F_B (Eq. rerr).

    dtau, S: [N_layers, N_nu], layer 0 at the top.  Returns (F_0, F_n stack).
    """
    N = dtau.shape[0]
    Tn = transmission(dtau)
    F = np.empty((N + 1,) + dtau.shape[1:])
    F[N] = F_B
    for n in range(N - 1, -1, -1):
        F[n] = Tn[n] * F[n + 1] + (1.0 - Tn[n]) * S[n]
    return F[0], F


# ---------------------------------------------------------------------------
# Response (Sec. 4): rotation then Gaussian IP on the log-uniform grid
# ---------------------------------------------------------------------------

def rotation_kernel(x, u1, u2):
    """zeta(x) from integrating the quadratic limb-darkened disk along y (Sec. 4.1).

    zeta = [2 s (1-u1-u2) + pi/2 (u1+2u2) s^2 - 4/3 u2 s^3] / [pi (1 - u1/3 - u2/6)],
    s = sqrt(1-x^2) for |x| < 1 and 0 otherwise.
    """
    x = np.asarray(x, float)
    inside = np.abs(x) < 1.0
    s = np.sqrt(np.where(inside, 1.0 - x * x, 0.0))
    num = 2.0 * s * (1 - u1 - u2) + 0.5 * math.pi * (u1 + 2 * u2) * s ** 2 - (4.0 / 3.0) * u2 * s ** 3
    return np.where(inside, num / (math.pi * (1.0 - u1 / 3.0 - u2 / 6.0)), 0.0)


def drotation_kernel(x, u1, u2):
    x = np.asarray(x, float)
    inside = np.abs(x) < 1.0
    s = np.sqrt(np.where(inside, 1.0 - x * x, 1.0))
    dnum_ds = 2.0 * (1 - u1 - u2) + math.pi * (u1 + 2 * u2) * s - 4.0 * u2 * s ** 2
    return np.where(inside, dnum_ds * (-x / s) / (math.pi * (1.0 - u1 / 3.0 - u2 / 6.0)), 0.0)


def ip_beta_kms(R):
    """beta_IP = c / (2 sqrt(2 ln 2) R)  (Sec. 4.2)."""
    return C_KMS / (2.0 * math.sqrt(2.0 * math.log(2.0)) * R)


IP_TRUNC_SIGMA = 6.0


def _velocity(nu):
    return C_KMS * np.log(np.asarray(nu, float))


def _rotation_support(v, i, rv, vsini):
    """Index slice of grid points j with |c ln(nu_i/nu_j) + RV| < vsini, plus the scaled argument."""
    neg = -(v[i] - v + rv)                     # increasing in j
    jl = int(np.searchsorted(neg, -vsini, side="right"))
    jh = int(np.searchsorted(neg, vsini, side="left"))
    if jl <= 0 or jh >= v.size:
        raise ValueError("rotation kernel reaches outside the grid")
    sl = slice(jl, jh)
    return sl, (v[i] - v[sl] + rv) / vsini


def rotate(F0, nu, idx, rv, vsini, u1, u2, want_tangent=False):
    """G_i = sum_j k_R(c ln(nu_i/nu_j) + RV) F0_j / sum_j k_R(same), i in idx (Eq. responsenu)."""
    v = _velocity(nu)
    G = np.empty(len(idx))
    dG_rv = np.empty(len(idx))
    dG_vs = np.empty(len(idx))
    for k, i in enumerate(idx):
        sl, x = _rotation_support(v, i, rv, vsini)
        t = rotation_kernel(x, u1, u2)
        st = t.sum()
        G[k] = np.dot(t, F0[sl]) / st
        if want_tangent:
            dz = drotation_kernel(x, u1, u2)
            dt_rv = dz / vsini
            dt_vs = -dz * x / vsini
            dG_rv[k] = (np.dot(dt_rv, F0[sl]) - G[k] * dt_rv.sum()) / st
            dG_vs[k] = (np.dot(dt_vs, F0[sl]) - G[k] * dt_vs.sum()) / st
    if want_tangent:
        return G, dG_rv, dG_vs
    return G


def rotate_linear(X, nu, idx, rv, vsini, u1, u2):
    """Apply the (normalised) rotation operator to several vectors X[..., N_nu]."""
    v = _velocity(nu)
    X = np.atleast_2d(X)
    out = np.empty((X.shape[0], len(idx)))
    for k, i in enumerate(idx):
        sl, x = _rotation_support(v, i, rv, vsini)
        t = rotation_kernel(x, u1, u2)
        out[:, k] = X[:, sl] @ t / t.sum()
    return out


def instrumental(G, nu_mid, idx_out, R):
    """F_i = sum_i' k_G(c ln(nu_i/nu_i')) G_i' / sum k_G(same), |.| <= 6 beta_IP.

    G is given on the contiguous index range nu_mid (the rotation output grid).
    """
    v = _velocity(nu_mid)
    b = ip_beta_kms(R)
    G = np.atleast_2d(G)
    out = np.empty((G.shape[0], len(idx_out)))
    for k, i in enumerate(idx_out):
        d = v[i] - v
        m = np.abs(d) <= IP_TRUNC_SIGMA * b
        if m[0] or m[-1]:
            raise ValueError("IP kernel reaches outside the rotation output")
        kg = np.exp(-0.5 * (d[m] / b) ** 2) / math.sqrt(2.0 * math.pi * b * b)
        out[:, k] = G[:, m] @ kg / kg.sum()
    return out


def _ip_reach_points(nu, R):
    v = _velocity(nu)
    dv = np.min(np.diff(v))
    return int(math.ceil(IP_TRUNC_SIGMA * ip_beta_kms(R) / dv)) + 1


def response(F0, nu, resp, want_tangent=False):
    """k_G * k_R * F0 on output indices [out_begin, out_begin + out_len) (Eq. model)."""
    nu = np.asarray(nu, float)
    K = _ip_reach_points(nu, resp.R_inst)
    lo = resp.out_begin - K
    hi = resp.out_begin + resp.out_len + K
    if lo < 0 or hi > nu.size:
        raise ValueError("output range too close to the grid edge")
    mid = np.arange(lo, hi)
    r = rotate(F0, nu, mid, resp.rv_kms, resp.vsini_kms, resp.u1, resp.u2, want_tangent)
    out_idx = np.arange(K, K + resp.out_len)
    if not want_tangent:
        return instrumental(r, nu[mid], out_idx, resp.R_inst)[0]
    G, G_rv, G_vs = r
    F = instrumental(np.stack([G, G_rv, G_vs]), nu[mid], out_idx, resp.R_inst)
    return F[0], F[1], F[2]


def response_linear(X, nu, resp):
    """The response as a linear map applied to rows of X (tangent propagation)."""
    nu = np.asarray(nu, float)
    K = _ip_reach_points(nu, resp.R_inst)
    lo = resp.out_begin - K
    hi = resp.out_begin + resp.out_len + K
    mid = np.arange(lo, hi)
    G = rotate_linear(X, nu, mid, resp.rv_kms, resp.vsini_kms, resp.u1, resp.u2)
    return instrumental(G, nu[mid], np.arange(K, K + resp.out_len), resp.R_inst)


# ---------------------------------------------------------------------------
# Full forward model and tangents
# ---------------------------------------------------------------------------

@dataclass
class Columns:
    T: np.ndarray            # [N_L]
    dP: np.ndarray           # [N_L] bar
    dtau_mol: np.ndarray     # [N_m, N_L, N_nu]
    ddtau_mol_dT: Optional[np.ndarray]
    dtau_cia: np.ndarray     # [N_L, N_nu]
    ddtau_cia_dT: np.ndarray
    S: np.ndarray            # [N_L, N_nu]  pi B(T_n)
    dS_dT: np.ndarray
    F_B: np.ndarray
    dF_B_dT: np.ndarray


def _xs_layer(args):
    ll, T, P, nu, want = args
    return cross_section(ll, T, P, nu, want_dT=want, parallel=False)


def optical_depths(wl, theta, nu_idx=None, want_dT=False) -> Columns:
    """Per-layer molecular/CIA optical depths and sources at the grid points nu_idx."""
    atm = wl.atmos
    nu = wl.nu if nu_idx is None else wl.nu[np.asarray(nu_idx)]
    T0, alpha = float(theta[0]), float(theta[1])
    nm = len(wl.lines)
    logx = np.asarray(theta[2:2 + nm], float)
    P = atm.P_bar
    T = layer_temperatures(atm, T0, alpha)
    dP = layer_dP_bar(P)
    NL = P.size
    tau = np.zeros((nm, NL, nu.size))
    dtau = np.zeros((nm, NL, nu.size)) if want_dT else None
    modit = getattr(atm, "opacity", "lpf") == "modit"
    if modit and (want_dT or nu_idx is not None):
        raise ValueError("the MODIT opacity is evaluated on the whole grid, without tangents")
    for m, ll in enumerate(wl.lines):
        col = column_factor(dP, 10.0 ** logx[m], ll.mass_amu, atm.g_cgs)
        if modit:
            from .modit import modit_cross_section
            for n in range(NL):
                # the truncated transform rings slightly below zero next to
                # narrow lines; an optical depth is not negative
                tau[m, n] = col[n] * np.maximum(modit_cross_section(ll, T[n], P[n], nu, atm.modit_dln_gamma), 0.0)
            continue
        # one cross-section per layer, the layers spread over threads
        res = _pool_map(_xs_layer, [(ll, T[n], P[n], nu, want_dT) for n in range(NL)])
        for n, r in enumerate(res):
            if want_dT:
                tau[m, n] = col[n] * r[0]
                dtau[m, n] = col[n] * r[1]
            else:
                tau[m, n] = col[n] * r
    tc = np.stack([dtau_cia(T[n], P[n], dP[n], nu, atm) for n in range(NL)])
    dtc = tc * ((atm.cia_Tpow - 1.0) / T)[:, None]
    S = np.stack([planck_pi(T[n], nu) for n in range(NL)])
    dS = np.stack([dplanck_pi_dT(T[n], nu) for n in range(NL)])
    if atm.bottom == 0:
        FB, dFB = S[-1].copy(), dS[-1].copy()
    else:
        FB, dFB = np.zeros(nu.size), np.zeros(nu.size)
    return Columns(T, dP, tau, dtau, tc, dtc, S, dS, FB, dFB)


def emission_F0(wl, theta, nu_idx=None):
    """Top-of-atmosphere flux F_0 at grid points nu_idx (all points by default)."""
    c = optical_depths(wl, theta, nu_idx)
    dt = c.dtau_mol.sum(axis=0) + c.dtau_cia
    return rt_recurrence(dt, c.S, c.F_B)[0]


def cross_section_config(wl, precision_T=None):
    """sigma for a single-layer workload (configuration 1)."""
    return cross_section(wl.lines[0], wl.T, wl.P_bar, wl.nu)


def emission_flux(wl, theta):
    """F on the output grid (Eq. model without the photometric normalisation)."""
    F0 = emission_F0(wl, theta)
    if wl.response is None:
        return F0
    resp = _resp_with(wl.response, theta)
    return response(F0, wl.nu, resp)


def _resp_with(resp, theta):
    from dataclasses import replace
    return replace(resp, rv_kms=float(theta[-2]), vsini_kms=float(theta[-1]))


def flux_tangents(wl, theta, per_layer=False, nu_idx=None):
    """F and dF/dtheta for theta = (T0, alpha, log10 X_1..X_M, RV, vsini).

    Forward-mode: the tangent of every intermediate quantity is carried
    through the recurrence of Eq. rerr and the response.  With per_layer,
    also dF/dT_n for every layer n.  Without a response every grid point's
    column is independent, and nu_idx restricts the result to those points.
    """
    atm = wl.atmos
    nm = len(wl.lines)
    if nu_idx is not None and wl.response is not None:
        raise ValueError("grid points can be selected only without the response")
    c = optical_depths(wl, theta, nu_idx=nu_idx, want_dT=True)
    P = atm.P_bar
    T = c.T
    NL = P.size
    dT_dth = np.zeros((2, NL))
    if getattr(atm, "T_layers", None) is None:   # a layer-by-layer profile ignores (T0, alpha)
        dT_dth[0] = T / theta[0]
        dT_dth[1] = T * np.log(P)
    tau = c.dtau_mol.sum(axis=0) + c.dtau_cia
    dtau_dTn = c.ddtau_mol_dT.sum(axis=0) + c.ddtau_cia_dT
    Tn = transmission(tau)
    dTn = dtransmission(tau)
    F0, F = rt_recurrence(tau, c.S, c.F_B)

    ndir = 2 + nm
    d_tau = np.zeros((ndir, NL, tau.shape[1]))
    d_S = np.zeros_like(d_tau)
    d_FB = np.zeros((ndir, tau.shape[1]))
    for d in range(2):
        d_tau[d] = dtau_dTn * dT_dth[d][:, None]
        d_S[d] = c.dS_dT * dT_dth[d][:, None]
        d_FB[d] = c.dF_B_dT * dT_dth[d][-1]
    for m in range(nm):
        d_tau[2 + m] = math.log(10.0) * c.dtau_mol[m]
    # tangent recurrence: dF_n = dT_n (F_{n+1} - S_n) + T_n dF_{n+1} + (1 - T_n) dS_n
    dF = d_FB.copy()
    for n in range(NL - 1, -1, -1):
        dF = dTn[n] * d_tau[:, n] * (F[n + 1] - c.S[n]) + Tn[n] * dF + (1.0 - Tn[n]) * d_S[:, n]
    dF0 = dF

    dF0_layers = None
    if per_layer:
        Phi = np.concatenate([np.ones((1, tau.shape[1])), np.cumprod(Tn, axis=0)])
        dF0_layers = np.empty((NL, tau.shape[1]))
        for n in range(NL):
            dF0_layers[n] = Phi[n] * (dTn[n] * dtau_dTn[n] * (F[n + 1] - c.S[n])
                                      + (1.0 - Tn[n]) * c.dS_dT[n])
        if atm.bottom == 0:
            dF0_layers[NL - 1] += Phi[NL] * c.dF_B_dT

    if wl.response is None:
        out = {"F": F0, "dF": np.concatenate([dF0, np.zeros((2, F0.size))])}
        if per_layer:
            out["dF_dTn"] = dF0_layers
        return out
    resp = _resp_with(wl.response, theta)
    Fo, F_rv, F_vs = response(F0, wl.nu, resp, want_tangent=True)
    dFo = response_linear(dF0, wl.nu, resp)
    out = {"F": Fo, "dF": np.concatenate([dFo, F_rv[None], F_vs[None]])}
    if per_layer:
        out["dF_dTn"] = response_linear(dF0_layers, wl.nu, resp)
    return out


def flux_jvp(wl, theta, dtheta, dT_layers=None):
    """J dtheta: the directional derivative of F along dtheta (and along the
    per-layer temperature tangent dT_layers, if given), assembled from the
    forward-mode tangents of flux_tangents."""
    t = flux_tangents(wl, theta, per_layer=dT_layers is not None)
    out = np.tensordot(np.asarray(dtheta, float), t["dF"], axes=1)
    if dT_layers is not None:
        out = out + np.asarray(dT_layers, float) @ t["dF_dTn"]
    return t["F"], out


def gaussian_loss(F, data, sigma):
    """Case-I style independent Gaussian loss 0.5 sum ((d - F)/sigma)^2 (Eq. likelihood, no jitter)."""
    return 0.5 * np.sum(((data - F) / sigma) ** 2)


def loss_gradient(wl, theta, data, sigma, per_layer=False):
    """(loss, dloss/dtheta[, dloss/dT_n]) via the forward tangents."""
    t = flux_tangents(wl, theta, per_layer=per_layer)
    F = t["F"]
    cot = -(data - F) / sigma ** 2
    g = t["dF"] @ cot
    L = gaussian_loss(F, data, sigma)
    if per_layer:
        return L, g, t["dF_dTn"] @ cot
    return L, g
