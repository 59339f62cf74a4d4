"""Plain FP64 CPU oracle of MODIT, the paper's cross-section method for many
lines (Sec. 2.1.2): a lineshape density on a log-uniform wavenumber grid,
convolved with the Voigt profile through the discrete Fourier transform.

TEST INFRASTRUCTURE ONLY, like ``oracle.oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
use it; the product path never does.

The steps follow Sec. 2.1.2 in its order and notation, with numpy's FFT as the
library primitive:

1. q = R0 ln(nu): on a log-uniform grid nu_i the grid index i is q up to an
   offset, and the Doppler width in q, beta~ = sqrt(k_B T / (M m_u)) R0 / c,
   is common to all lines of the (species, layer).  gamma~_l = R0 gamma_l / nu_l.
2. The lineshape density S_{jk} on the (q_j, ln gamma~_k) grid: every line adds
   its strength to the four neighbouring nodes with linear weights in q and in
   ln gamma~.
3. sigma(q_i) = sum_k IDFT[ DFT(S_{.k}) exp(-2 pi^2 beta~^2 f^2 - 2 pi gamma~_k |f|) ](i),
   the Voigt profile's Fourier transform in q (Eq. MODIT), and
   sigma(nu_i) = sigma(q_i) dq/dnu = sigma(q_i) R0 / nu_i.

Readings where the paper is silent (also the HIP path's):

* Line position: the fractional grid index, linear in ln(nu) between the two
  neighbouring grid points.  Lines outside [nu_0, nu_{N-1}] are not part of
  the density (it lives on the grid).
* Width grid: ln gamma~_k = ln gamma~_min + k d, k = 0..K-1, with
  K = floor((ln gamma~_max - ln gamma~_min) / d) + 2; when that exceeds
  MAX_BINS the step widens to (range)/(MAX_BINS - 2).  gamma~ is floored at
  1e-3 beta~ (a Lorentz core a thousand times narrower than the Gaussian), so
  that lines with no pressure or natural width keep a finite ln gamma~.
* DFT length: the smallest power of two >= 2N.  The zero padding keeps a
  profile's circular wrap-around out of the window unless its wing reaches
  past N grid points; the aliasing correction the paper mentions is
  unpublished and not applied.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .oracle import C_LIGHT, K_BOLTZ, M_U, line_state

MAX_BINS = 32


@dataclass
class ModitGrid:
    R0: float          # 1 / mean ln spacing of the grid
    n: int             # grid points
    n_fft: int         # DFT length


def modit_grid(nu) -> ModitGrid:
    nu = np.asarray(nu, float)
    R0 = (nu.size - 1) / math.log(nu[-1] / nu[0])
    n_fft = 1
    while n_fft < 2 * nu.size:
        n_fft *= 2
    return ModitGrid(R0, nu.size, n_fft)


def beta_q(T: float, mass_amu: float, R0: float) -> float:
    """Doppler standard deviation in q (Sec. 2.1.2): sqrt(k_B T / (M m_u)) R0 / c."""
    return math.sqrt(K_BOLTZ * T / (mass_amu * M_U)) * R0 / C_LIGHT


def line_positions(nu, nu_c):
    """Fractional grid index of every line (linear in ln nu between grid
    points); NaN for lines outside the grid."""
    nu = np.asarray(nu, float)
    nu_c = np.asarray(nu_c, float)
    x = np.full(nu_c.size, np.nan)
    inside = (nu_c >= nu[0]) & (nu_c <= nu[-1])
    j = np.searchsorted(nu, nu_c[inside], side="right") - 1
    j = np.minimum(j, nu.size - 2)
    ln = np.log(nu)
    x[inside] = j + (np.log(nu_c[inside]) - ln[j]) / (ln[j + 1] - ln[j])
    return x


def width_grid(lng, dlng: float):
    """(ln gamma~_0, step, K) covering the given ln gamma~ values."""
    lo, hi = float(np.min(lng)), float(np.max(lng))
    d = float(dlng)
    K = int(math.floor((hi - lo) / d)) + 2
    if K > MAX_BINS:
        d = (hi - lo) / (MAX_BINS - 2)
        K = int(math.floor((hi - lo) / d)) + 2
        K = min(K, MAX_BINS)
    return lo, d, K


def lineshape_density(x, lng, S, n: int, lng0: float, d: float, K: int):
    """S_{jk}: [n, K], every line split over the four neighbouring nodes with
    linear weights in q (x) and in ln gamma~."""
    lsd = np.zeros((n, K))
    j0 = np.floor(x).astype(np.int64)
    fx = x - j0
    t = (lng - lng0) / d
    k0 = np.minimum(np.floor(t).astype(np.int64), K - 2)
    fk = t - k0
    for dj, wx in ((0, 1.0 - fx), (1, fx)):
        for dk, wk in ((0, 1.0 - fk), (1, fk)):
            jj = j0 + dj
            ok = (jj < n) & (wx * wk != 0.0)
            np.add.at(lsd, (jj[ok], k0[ok] + dk), (S * wx * wk)[ok])
    return lsd


def voigt_ft(f, beta_t: float, gamma_t):
    """Fourier transform of the Voigt profile in q at frequencies f (cycles per
    grid step): exp(-2 pi^2 beta~^2 f^2 - 2 pi gamma~ |f|)."""
    return np.exp(-2.0 * math.pi ** 2 * beta_t ** 2 * f ** 2 - 2.0 * math.pi * gamma_t * np.abs(f))


def sigma_q_periodic(lsd, beta_t: float, gamma_k, n_fft: int):
    """The circular convolution over the whole DFT length (n_fft points)."""
    n, K = lsd.shape
    f = np.fft.fftfreq(n_fft)
    acc = np.zeros(n_fft, complex)
    for k in range(K):
        row = np.zeros(n_fft)
        row[:n] = lsd[:, k]
        acc += np.fft.fft(row) * voigt_ft(f, beta_t, gamma_k[k])
    return np.fft.ifft(acc).real


def modit_cross_section(ll, T: float, P_bar: float, nu, dlng: float = 0.1, want_parts: bool = False):
    """MODIT sigma(nu_i) [cm^2 / molecule] on the log-uniform grid nu."""
    nu = np.asarray(nu, float)
    g = modit_grid(nu)
    st = line_state(ll, T, P_bar)
    bt = beta_q(T, ll.mass_amu, g.R0)
    x = line_positions(nu, ll.nu_c)
    inside = ~np.isnan(x)
    nu_c = np.asarray(ll.nu_c, float)[inside]
    gt = np.maximum(g.R0 * np.asarray(st.gamma, float)[inside] / nu_c, 1e-3 * bt)
    lng = np.log(gt)
    S = np.asarray(st.S, float)[inside]
    if S.size == 0:
        sig = np.zeros(nu.size)
        return (sig, None) if want_parts else sig
    lng0, d, K = width_grid(lng, dlng)
    lsd = lineshape_density(x[inside], lng, S, g.n, lng0, d, K)
    gamma_k = np.exp(lng0 + d * np.arange(K))
    sq = sigma_q_periodic(lsd, bt, gamma_k, g.n_fft)
    sig = sq[:g.n] * g.R0 / nu
    if want_parts:
        return sig, {"grid": g, "beta_t": bt, "lsd": lsd, "gamma_k": gamma_k, "sigma_q": sq,
                     "x": x[inside], "S": S, "lng0": lng0, "dlng": d, "K": K}
    return sig
