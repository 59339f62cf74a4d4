"""Hamiltonian Monte Carlo driver for the spectrum model (Sec. 5.2): the
No-U-Turn sampler with dual-averaging step-size adaptation, restated from
Hoffman & Gelman (2014, JMLR 15, 1593), drawing the log-posterior and its
gradient from the GPU in one pass per leapfrog step (exo_loss_grad).

The parameters live in a box (the uniform priors of Table 2); the sampler
moves in unconstrained coordinates z with theta = lo + (hi - lo) s(z),
s the logistic function, and the log-density carries the Jacobian
sum log((hi - lo) s (1 - s)).  The mass matrix is the identity in z.

Host-side vector arithmetic on a handful of parameters; the cost per
leapfrog step is one spectrum + gradient evaluation on the device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, Optional, Sequence

import numpy as np


# --------------------------------------------------------------------------- posterior

def _logistic(z):
    # exp of a non-positive argument only: no overflow for large |z|
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def _log_logistic(z):
    """log s(z) = -log(1 + e^{-z}), finite for every finite z."""
    return -np.logaddexp(0.0, -z)


class BoxPosterior:
    """log p(z) and its gradient for a target given in box-bounded parameters.

    logp_theta(theta) -> (log density, gradient w.r.t. theta)
    """

    def __init__(self, logp_theta: Callable, lo: Sequence[float], hi: Sequence[float]):
        self.f = logp_theta
        self.lo = np.asarray(lo, float)
        self.hi = np.asarray(hi, float)
        self.n_eval = 0

    def theta(self, z):
        return self.lo + (self.hi - self.lo) * _logistic(np.asarray(z, float))

    def z_of(self, theta):
        u = (np.asarray(theta, float) - self.lo) / (self.hi - self.lo)
        return np.log(u) - np.log1p(-u)

    def __call__(self, z):
        z = np.asarray(z, float)
        s = _logistic(z)
        w = self.hi - self.lo
        th = self.lo + w * s
        lp, g = self.f(th)
        self.n_eval += 1
        # log((hi - lo) s (1 - s)), with log(1 - s) = log s(-z)
        jac = np.sum(np.log(w) + _log_logistic(z) + _log_logistic(-z))
        return lp + jac, np.asarray(g, float) * w * s * (1.0 - s) + (1.0 - 2.0 * s)


class SpectrumPosterior(BoxPosterior):
    """Gaussian likelihood of a spectrum under the power-law model,
    theta = (T0, alpha, log10 X_1..X_M, RV, vsini), with a box prior."""

    def __init__(self, ctx, atmos, response, data, sigma, lo, hi):
        import torch
        from .api import Atmos, Response
        self.ctx = ctx
        self.atmos = atmos
        self.response = response
        self.data = torch.as_tensor(np.asarray(data, np.float32), device=f"cuda:{ctx.device}").contiguous()
        self.sigma = torch.as_tensor(np.asarray(sigma, np.float32), device=f"cuda:{ctx.device}").contiguous()
        self._Atmos, self._Response = Atmos, Response
        super().__init__(self._logp, lo, hi)

    def _logp(self, th):
        m = len(self.atmos.species)
        a = self._Atmos(**{**self.atmos.__dict__, "T0": th[0], "alpha": th[1], "log10_mmr": list(th[2:2 + m])})
        r = self._Response(**{**self.response.__dict__, "rv_kms": th[2 + m], "vsini_kms": th[3 + m]})
        loss, g, _, _ = self.ctx.loss_grad(a, r, self.data, self.sigma)
        return -loss, -g


# --------------------------------------------------------------------------- NUTS

@dataclass
class NutsResult:
    samples: np.ndarray        # [n_samples, dim] in the constrained parameters
    logp: np.ndarray           # [n_samples]
    step_size: float
    accept: np.ndarray         # [n_samples] mean acceptance statistic of each iteration
    tree_depth: np.ndarray     # [n_samples]
    n_eval: int                # log-density + gradient evaluations
    divergences: int           # divergent trajectories after warmup


def _leapfrog(post, z, r, g, eps):
    r = r + 0.5 * eps * g
    z = z + eps * r
    lp, g = post(z)
    r = r + 0.5 * eps * g
    return z, r, lp, g


def _find_reasonable_eps(post, z, lp, g, rng):
    eps = 1.0
    r = rng.normal(size=z.size)
    H0 = lp - 0.5 * r @ r
    _, r1, lp1, _ = _leapfrog(post, z, r, g, eps)
    H1 = lp1 - 0.5 * r1 @ r1
    a = 1.0 if (np.isfinite(H1) and H1 - H0 > math.log(0.5)) else -1.0
    for _ in range(60):
        _, r1, lp1, _ = _leapfrog(post, z, r, g, eps)
        H1 = lp1 - 0.5 * r1 @ r1
        if not (np.isfinite(H1) and a * (H1 - H0) > -a * math.log(2.0)):
            break
        eps *= 2.0 ** a
    return eps


def nuts(post, z0, n_samples: int, n_warmup: int, rng: np.random.Generator, delta: float = 0.8,
         max_depth: int = 8, delta_max: float = 1000.0) -> NutsResult:
    """The No-U-Turn sampler with dual averaging (Hoffman & Gelman 2014,
    efficient NUTS with slice sampling).  Returns the post-warmup samples."""
    z = np.asarray(z0, float).copy()
    lp, g = post(z)
    eps = _find_reasonable_eps(post, z, lp, g, rng)
    mu, log_eps_bar, H_bar, gamma, t0, kappa = math.log(10.0 * eps), 0.0, 0.0, 0.05, 10.0, 0.75
    out_z, out_lp, out_acc, out_depth = [], [], [], []
    divergences = 0          # after warmup (the adaptation tries large steps on purpose)
    sampling = False

    def build_tree(z, r, g, log_u, v, j, H0):
        nonlocal divergences
        if j == 0:
            z1, r1, lp1, g1 = _leapfrog(post, z, r, g, v * eps)
            H1 = lp1 - 0.5 * r1 @ r1
            if not np.isfinite(H1):
                H1 = -np.inf
            n1 = 1 if log_u <= H1 else 0
            s1 = 1 if H1 > log_u - delta_max else 0
            if not s1 and sampling:
                divergences += 1
            acc = min(1.0, math.exp(min(0.0, H1 - H0))) if np.isfinite(H1) else 0.0
            return z1, r1, g1, z1, r1, g1, z1, lp1, g1, n1, s1, acc, 1
        zm, rm, gm, zp, rp, gp, z1, lp1, g1, n1, s1, a1, na1 = build_tree(z, r, g, log_u, v, j - 1, H0)
        if s1:
            if v < 0:
                zm, rm, gm, _, _, _, z2, lp2, g2, n2, s2, a2, na2 = build_tree(zm, rm, gm, log_u, v, j - 1, H0)
            else:
                _, _, _, zp, rp, gp, z2, lp2, g2, n2, s2, a2, na2 = build_tree(zp, rp, gp, log_u, v, j - 1, H0)
            if n1 + n2 > 0 and rng.uniform() < n2 / (n1 + n2):
                z1, lp1, g1 = z2, lp2, g2
            a1 += a2
            na1 += na2
            dz = zp - zm
            s1 = s2 * int(dz @ rm >= 0) * int(dz @ rp >= 0)
            n1 += n2
        return zm, rm, gm, zp, rp, gp, z1, lp1, g1, n1, s1, a1, na1

    for m in range(1, n_warmup + n_samples + 1):
        sampling = m > n_warmup
        r0 = rng.normal(size=z.size)
        H0 = lp - 0.5 * r0 @ r0
        log_u = H0 + math.log(rng.uniform())
        zm = zp = z
        rm = rp = r0
        gm = gp = g
        n, s, j = 1, 1, 0
        a_sum, na_sum = 0.0, 0
        while s and j < max_depth:
            v = -1.0 if rng.uniform() < 0.5 else 1.0
            if v < 0:
                zm, rm, gm, _, _, _, z1, lp1, g1, n1, s1, a1, na1 = build_tree(zm, rm, gm, log_u, v, j, H0)
            else:
                _, _, _, zp, rp, gp, z1, lp1, g1, n1, s1, a1, na1 = build_tree(zp, rp, gp, log_u, v, j, H0)
            if s1 and rng.uniform() < min(1.0, n1 / n):
                z, lp, g = z1, lp1, g1
            n += n1
            a_sum += a1
            na_sum += na1
            dz = zp - zm
            s = s1 * int(dz @ rm >= 0) * int(dz @ rp >= 0)
            j += 1
        acc = a_sum / max(na_sum, 1)
        if m <= n_warmup:
            eta = 1.0 / (m + t0)
            H_bar = (1.0 - eta) * H_bar + eta * (delta - acc)
            log_eps = mu - math.sqrt(m) / gamma * H_bar
            w = m ** (-kappa)
            log_eps_bar = w * log_eps + (1.0 - w) * log_eps_bar
            eps = math.exp(log_eps)
            if m == n_warmup:
                eps = math.exp(log_eps_bar)
        else:
            out_z.append(post.theta(z) if hasattr(post, "theta") else z.copy())
            out_lp.append(lp)
            out_acc.append(acc)
            out_depth.append(j)
    return NutsResult(np.array(out_z), np.array(out_lp), eps, np.array(out_acc), np.array(out_depth),
                      getattr(post, "n_eval", 0), divergences)
