"""Seeded synthetic inputs shaped like the paper's K-band fits.

The paper fits CRIRES K-band spectra of Luhman 16A with ExoMol/HITEMP CO and
H2O line lists (Sec. 5, Table 3).  Those data are not available here, so
every input below is drawn from a seeded ``numpy.random.default_rng`` with the
shapes of the paper's workloads: a 40 cm^-1 K-band window, 100 power-law
layers from 1e-8 to 1e2 bar, two absorbers of mass 18 and 28, R = 1e5
instrumental profile, and parameter values near the Table 3 medians.

Nothing here evaluates the spectrum model.  Arrays are float64, C-contiguous.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Seeds: default_rng(1000 + k) for configuration k (1-based).
CONFIG_SEEDS = {k: 1000 + k for k in range(1, 6)}

# Partition-function exponent choices for the synthetic qr(T) = (T/296)^k:
# 1.5 for the bent triatomic (mass 18), 1.0 for the linear rotor (mass 28).
QR_POWER_MASS18 = 1.5
QR_POWER_MASS28 = 1.0


@dataclass
class LineList:
    """One absorber's line list (structure of Table 1, ExoMol-style broadening)."""
    nu_c: np.ndarray            # line centres [cm^-1]
    S0: np.ndarray              # strength at 296 K [cm / molecule]
    E_low: np.ndarray           # lower-state energy [cm^-1]
    alpha_ref: np.ndarray       # broadening coefficient at 296 K, 1 bar [cm^-1 bar^-1]
    n_texp: np.ndarray          # temperature exponent of the broadening
    mass_amu: float             # molecular mass [amu]
    qr_kind: int = 0            # 0: power law (T/296)^k ; 1: table on T nodes
    qr_params: np.ndarray = field(default_factory=lambda: np.array([0.0]))
    gamma_nat: Optional[np.ndarray] = None   # natural width [cm^-1] (None: zero)

    @property
    def n(self) -> int:
        return int(self.nu_c.size)


@dataclass
class Atmosphere:
    """Layer model: pressures ascending (top -> bottom); power-law T-P profile
    unless T_layers gives every layer's temperature."""
    P_bar: np.ndarray
    T0: float
    alpha: float
    log10_mmr: np.ndarray       # one per species in the workload
    g_cgs: float = 10 ** 5.03   # surface gravity of the Luhman 16A fit [cm s^-2]
    mmw: float = 2.33           # mean molecular weight
    cia_alpha0: float = 5e-46   # H2-H2 CIA amplitude at 1000 K [cm^5]
    cia_Tpow: float = 1.0
    cia_slope: float = 0.1      # e-fold per 40 cm^-1 / slope
    cia_nu_c: float = 4360.0
    vmr_h2: float = 0.75 * 2.33 / 2.016
    bottom: int = 0             # 0: F_B = pi B(T_bottom) ; 1: F_B = 0
    T_layers: Optional[np.ndarray] = None   # layer-by-layer T [K]; replaces the power law
    opacity: str = "lpf"        # line opacity: "lpf" (direct sum) or "modit" (Sec. 2.1.2)
    modit_dln_gamma: float = 0.1


@dataclass
class Response:
    rv_kms: float
    vsini_kms: float
    u1: float
    u2: float
    R_inst: float
    out_begin: int
    out_len: int


@dataclass
class Workload:
    name: str
    lines: List[LineList]
    nu: np.ndarray
    atmos: Optional[Atmosphere] = None
    response: Optional[Response] = None
    T: Optional[float] = None          # single-layer cross-section temperature
    P_bar: Optional[float] = None      # single-layer cross-section pressure
    theta_star: Optional[np.ndarray] = None   # (T0, alpha, log10X..., RV, vsini)
    theta: Optional[np.ndarray] = None

    @property
    def evals_per_spectrum(self) -> int:
        nl = self.atmos.P_bar.size if self.atmos is not None else 1
        return int(sum(l.n for l in self.lines) * self.nu.size * nl)


def eslog_grid(nu_lo: float, nu_hi: float, n: int) -> np.ndarray:
    """n points evenly spaced in log(nu), both endpoints included."""
    return np.exp(np.linspace(np.log(nu_lo), np.log(nu_hi), n))


def _limb_darkening(q1: float, q2: float):
    # Kipping's uninformative reparametrisation used by the paper's fit.
    s = np.sqrt(q1)
    return 2.0 * s * q2, s * (1.0 - 2.0 * q2)


def _lines_config2(rng, n_lines, nu_lo, nu_hi, mass, qr_power):
    nu_c = np.sort(rng.uniform(nu_lo, nu_hi, n_lines))
    E_low = rng.exponential(3000.0, n_lines)
    S0 = 10.0 ** rng.normal(-22.0, 1.5, n_lines)
    alpha_ref = rng.uniform(0.01, 0.1, n_lines)
    n_texp = rng.uniform(0.5, 0.8, n_lines)
    return LineList(nu_c, S0, E_low, alpha_ref, n_texp, float(mass), 0,
                    np.array([qr_power]))


_SIZES = ("tiny", "small", "reduced", "medium", "full")


def make_config(k: int, size: str = "full", seed: Optional[int] = None) -> Workload:
    """Workload for configuration ``k`` (1..4) at ``size``.

    full   : the configuration as specified (1..3); 4 = config-2 atmosphere.
    medium : config-2 shape with fewer lines, still many tiles (parity runs).
    small  : several tiles plus ragged tails, oracle finishes in seconds.
    reduced: (configs 2 and 4) 1e3 lines per species, 2,000 points, 100
             layers: the size of the full-gradient oracle comparison.
    tiny   : a handful of lines/points for CPU-only oracle pins.
    """
    if size not in _SIZES:
        raise ValueError(size)
    rng = np.random.default_rng(CONFIG_SEEDS[k] if seed is None else seed)
    if k == 1:
        n_lines, n_nu = {"tiny": (7, 50), "small": (1000, 4000), "reduced": (1000, 4000),
                         "medium": (1000, 4000), "full": (1000, 4000)}[size]
        nu_c = np.sort(rng.uniform(4340.0, 4360.0, n_lines))
        S0 = 10.0 ** rng.uniform(-25.0, -20.0, n_lines)
        gam = rng.uniform(0.01, 0.1, n_lines)
        ll = LineList(nu_c, S0, np.zeros(n_lines), gam, np.zeros(n_lines), 18.0, 0,
                      np.array([0.0]))
        nu = np.linspace(4340.0, 4360.0, n_nu)
        return Workload(f"config1-{size}", [ll], nu, T=1000.0, P_bar=1.0)

    if k in (2, 4):
        # lines per species, grid points, layers, output margin (grid points)
        n_lines, n_nu, n_lay, margin = {
            "tiny": (9, 1201, 12, 60),
            "small": (401, 1537, 100, 160),
            "reduced": (1000, 2000, 100, 100),
            "medium": (20011, 20000, 100, 600),
            "full": (100000, 20000, 100, 600),
        }[size]
        la = _lines_config2(rng, n_lines, 4340.0, 4380.0, 18.0, QR_POWER_MASS18)
        lb = _lines_config2(rng, n_lines, 4340.0, 4380.0, 28.0, QR_POWER_MASS28)
        nu = eslog_grid(4340.0, 4380.0, n_nu)
        P = np.logspace(-8.0, 2.0, n_lay)
        u1, u2 = _limb_darkening(0.8, 0.3)
        logx = np.log10([0.0023, 0.0058])
        atm = Atmosphere(P, 1300.0, 0.10, logx)
        resp = Response(28.1, 16.2, u1, u2, 1.0e5, margin, n_nu - 2 * margin)
        theta_star = np.array([1300.0, 0.10, logx[0], logx[1], 28.1, 16.2])
        wl = Workload(f"config{k}-{size}", [la, lb], nu, atm, resp,
                      theta_star=theta_star)
        if k == 4:
            wl.theta = theta_star + np.array([20.0, 0.005, 0.05, -0.05, 0.2, -0.5])
        return wl

    if k == 3:
        n_lines, n_nu, n_lay = {
            "tiny": (11, 300, 5),
            "small": (3001, 2500, 10),
            "reduced": (3001, 2500, 10),
            "medium": (1_000_000, 100_000, 100),
            "full": (10_000_000, 100_000, 100),
        }[size]
        nu = 4340.0 * np.exp(np.arange(n_nu) / 1.0e6)
        nu_c = np.sort(rng.uniform(4340.0, 4796.44, n_lines))
        S0 = 10.0 ** np.clip(rng.normal(-23.0, 1.67, n_lines), -28.0, -18.0)
        E_low = rng.exponential(3000.0, n_lines)
        alpha_ref = rng.uniform(0.01, 0.1, n_lines)
        n_texp = rng.uniform(0.5, 0.8, n_lines)
        ll = LineList(nu_c, S0, E_low, alpha_ref, n_texp, 18.0, 0,
                      np.array([QR_POWER_MASS18]))
        P = np.logspace(-8.0, 2.0, n_lay)
        atm = Atmosphere(P, 1300.0, 0.10, np.log10([0.0023]),
                         cia_nu_c=float(0.5 * (nu[0] + nu[-1])))
        return Workload(f"config3-{size}", [ll], nu, atm, None)
    raise ValueError(f"no configuration {k}")


# ----------------------------------------------------------------------------
# Serving workload (configuration 5)
# ----------------------------------------------------------------------------

# Table 2 prior ranges of the fitted parameters (T0, alpha, MMR_CO, MMR_H2O,
# RV, vsini) and Table 3 medians (Case II, direct LPF) as starting point.
PRIOR_LO = np.array([1000.0, 0.05, 0.0, 0.0, 26.0, 10.0])
PRIOR_HI = np.array([1700.0, 0.15, 0.01, 0.005, 30.0, 20.0])
MEDIANS = np.array([1295.0, 0.099, 0.0057, 0.0023, 28.1, 16.2])


def hmc_walk(rng, n_steps: int, step_frac: float = 0.02) -> np.ndarray:
    """Reflecting Gaussian random walk inside the prior box (HMC-like stream)."""
    lo, hi = PRIOR_LO, PRIOR_HI
    width = hi - lo
    x = MEDIANS.copy()
    out = np.empty((n_steps, 6))
    for i in range(n_steps):
        x = x + rng.normal(0.0, step_frac, 6) * width
        # reflect into [lo, hi]
        x = np.where(x < lo, 2 * lo - x, x)
        x = np.where(x > hi, 2 * hi - x, x)
        x = np.clip(x, lo + 1e-9 * width, hi)
        out[i] = x
    return out


@dataclass
class ServingRequest:
    arrival_s: float
    species: tuple           # indices into the resident pool
    grid_begin: int          # offset into the resident master grid
    grid_len: int
    n_layers: int
    theta: np.ndarray        # T0, alpha, MMR_a, MMR_b, RV, vsini


def serving_pool(seed: int = CONFIG_SEEDS[5], n_lists: int = 16,
                 min_lines: float = 1e3, max_lines: float = 1e6, scale: float = 1.0):
    """Resident line lists (log-uniform sizes over 3900-5100 cm^-1) and the
    master ESLOG grid at R0 = 1e6 covering 3990-5010 cm^-1."""
    rng = np.random.default_rng(seed)
    lists = []
    for i in range(n_lists):
        n = int(round(10 ** rng.uniform(np.log10(min_lines), np.log10(max_lines)) * scale))
        n = max(n, 16)
        mass = 18.0 if i % 2 == 0 else 28.0
        qr = QR_POWER_MASS18 if mass == 18.0 else QR_POWER_MASS28
        ll = _lines_config2(rng, n, 3900.0, 5100.0, mass, qr)
        lists.append(ll)
    n_master = int(np.floor(1.0e6 * np.log(5010.0 / 3990.0))) + 1
    nu = 3990.0 * np.exp(np.arange(n_master) / 1.0e6)
    return lists, nu


def serving_requests(n: int, rate_hz: float, seed: int = CONFIG_SEEDS[5] + 17,
                     n_lists: int = 16, nu_master: Optional[np.ndarray] = None,
                     min_grid: int = 2000, max_grid: int = 100000,
                     min_layers: int = 50, max_layers: int = 200) -> List[ServingRequest]:
    """Poisson arrivals; windows log-uniform in length, starting in 4000-5000 cm^-1."""
    rng = np.random.default_rng(seed)
    if nu_master is None:
        _, nu_master = serving_pool(n_lists=0)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n)) if rate_hz > 0 else np.zeros(n)
    thetas = hmc_walk(rng, n)
    reqs = []
    for i in range(n):
        nlen = int(round(10 ** rng.uniform(np.log10(min_grid), np.log10(max_grid))))
        start_nu = rng.uniform(4000.0, 5000.0)
        j0 = int(np.searchsorted(nu_master, start_nu))
        j0 = min(j0, nu_master.size - nlen)
        sp = tuple(int(s) for s in rng.choice(n_lists, 2, replace=False))
        nl = int(rng.integers(min_layers, max_layers + 1))
        reqs.append(ServingRequest(float(t[i]), sp, j0, nlen, nl, thetas[i]))
    return reqs


def serving_atmosphere(req: ServingRequest, log10_mmr_floor: float = -12.0):
    """(P_bar, T0, alpha, log10 MMR pair, RV, vsini) of a serving request."""
    P = np.logspace(-8.0, 2.0, req.n_layers)
    th = req.theta
    logx = np.log10(np.maximum(th[2:4], 10.0 ** log10_mmr_floor))
    return P, float(th[0]), float(th[1]), logx, float(th[4]), float(th[5])
