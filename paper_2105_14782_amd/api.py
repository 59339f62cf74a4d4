"""Python front end of the exohip library.

PyTorch supplies device memory and streams; all arithmetic of the spectrum
model runs in the HIP kernels behind ``include/exohip.h``.  There is no
CPU fallback: without a built library or a HIP device every call raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

PRECISIONS = {"fp32": L.EXO_FP32_KAHAN, "fp64": L.EXO_FP64, "fp64_tiled": L.EXO_FP64_TILED}


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _stream(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


_OPACITY = {"lpf": L.EXO_OPACITY_LPF, "modit": L.EXO_OPACITY_MODIT}


@dataclass
class Atmos:
    """Atmosphere / model-grid description passed to emission_flux and flux_vjp."""
    P_bar: np.ndarray
    T0: float
    alpha: float
    species: Sequence[int]
    log10_mmr: Sequence[float]
    g_cgs: float = 10 ** 5.03
    mmw: float = 2.33
    cia_alpha0: float = 0.0
    cia_Tpow: float = 1.0
    cia_slope: float = 0.0
    cia_nu_c: float = 0.0
    vmr_h2: float = 0.0
    bottom: int = L.EXO_FB_PLANCK_BOTTOM
    grid_begin: int = 0
    grid_len: int = 0
    T_layers: Optional[np.ndarray] = None   # layer-by-layer T [K]; replaces (T0, alpha)
    opacity: str = "lpf"        # line optical depths: "lpf" (direct sum) or "modit" (forward only)
    modit_dln_gamma: float = 0.1

    def to_c(self):
        P = _f64(self.P_bar)
        sp = np.ascontiguousarray(np.asarray(self.species, dtype=np.int32))
        lx = _f64(self.log10_mmr)
        Tl = None if self.T_layers is None else _f64(self.T_layers)
        a = L.ExoAtmos(
            n_layers=P.size, P_bar=L.dptr(P), T0_K=float(self.T0), alpha=float(self.alpha),
            n_species=sp.size, species=sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            log10_mmr=L.dptr(lx), g_cgs=float(self.g_cgs), mmw=float(self.mmw),
            cia_alpha0=float(self.cia_alpha0), cia_Tpow=float(self.cia_Tpow),
            cia_slope=float(self.cia_slope), cia_nu_c=float(self.cia_nu_c),
            vmr_h2=float(self.vmr_h2), bottom=int(self.bottom),
            grid_begin=int(self.grid_begin), grid_len=int(self.grid_len),
            T_layers=L.dptr(Tl) if Tl is not None else None,
            opacity=_OPACITY[self.opacity], modit_dln_gamma=float(self.modit_dln_gamma))
        return a, (P, sp, lx, Tl)   # keep the arrays alive for the call

    @staticmethod
    def from_workload(atm, species, theta=None, grid_begin=0, grid_len=0) -> "Atmos":
        """From a synth.Atmosphere-like object; theta = (T0, alpha, log10X..., [RV, vsini])."""
        nm = len(species)
        T0, al = (atm.T0, atm.alpha) if theta is None else (float(theta[0]), float(theta[1]))
        lx = atm.log10_mmr if theta is None else np.asarray(theta[2:2 + nm], float)
        return Atmos(atm.P_bar, T0, al, list(species), list(lx), atm.g_cgs, atm.mmw,
                     atm.cia_alpha0, atm.cia_Tpow, atm.cia_slope, atm.cia_nu_c, atm.vmr_h2,
                     atm.bottom, grid_begin, grid_len, getattr(atm, "T_layers", None),
                     getattr(atm, "opacity", "lpf"), getattr(atm, "modit_dln_gamma", 0.1))


@dataclass
class Response:
    rv_kms: float
    vsini_kms: float
    u1: float
    u2: float
    R_inst: float
    out_begin: int
    out_len: int

    def to_c(self):
        return L.ExoResponse(float(self.rv_kms), float(self.vsini_kms), float(self.u1), float(self.u2),
                             float(self.R_inst), int(self.out_begin), int(self.out_len))

    @staticmethod
    def from_workload(r, theta=None) -> "Response":
        rv, vs = (r.rv_kms, r.vsini_kms) if theta is None else (float(theta[-2]), float(theta[-1]))
        return Response(rv, vs, r.u1, r.u2, r.R_inst, r.out_begin, r.out_len)


class Context:
    """A device context with resident line lists and wavenumber grid."""

    def __init__(self, device: int = 0):
        self._lib = L.load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("exohip needs a HIP device (torch.cuda.is_available() is False)")
        self.device = device
        h = ctypes.c_void_p()
        L.check(self._lib.exo_create(device, ctypes.byref(h)))
        self._h = h
        self.n_nu = 0
        self._nlines = {}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.exo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- registration -------------------------------------------------------
    def set_lines(self, slot: int, ll) -> None:
        """Register a line list (attributes as synth.LineList)."""
        arrs = [_f64(getattr(ll, k)) for k in ("nu_c", "S0", "E_low", "alpha_ref", "n_texp")]
        gn = None if getattr(ll, "gamma_nat", None) is None else _f64(ll.gamma_nat)
        qp = _f64(ll.qr_params)
        n = arrs[0].size
        L.check(self._lib.exo_set_lines(self._h, int(slot), n, *[L.dptr(a) for a in arrs], L.dptr(gn),
                                        float(ll.mass_amu), int(ll.qr_kind), L.dptr(qp), int(qp.size)))
        self._nlines[int(slot)] = n

    def set_grid(self, nu) -> None:
        nu = _f64(nu)
        L.check(self._lib.exo_set_grid(self._h, nu.size, L.dptr(nu)))
        self.n_nu = nu.size

    # -- evaluation ---------------------------------------------------------
    def cross_section(self, slot: int, T: float, P_bar: float, precision="fp32", out=None, stream=None):
        p = _prec(precision)
        dt = torch.float32 if p == L.EXO_FP32_KAHAN else torch.float64
        if out is None:
            out = torch.empty(self.n_nu, dtype=dt, device=f"cuda:{self.device}")
        assert out.dtype == dt and out.is_contiguous() and out.numel() == self.n_nu
        L.check(self._lib.exo_cross_section(self._h, int(slot), float(T), float(P_bar), p,
                                            ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def cross_section_noalloc(self, slot: int, T: float, P_bar: float, out: torch.Tensor, precision="fp32",
                              stream=None):
        """cross_section into a caller-owned tensor, with no device allocation
        by the library (its scratch is a fixed per-device array shared by all
        such calls on the GPU: overlapping calls race)."""
        p = _prec(precision)
        dt = torch.float32 if p == L.EXO_FP32_KAHAN else torch.float64
        assert out.dtype == dt and out.is_contiguous() and out.numel() == self.n_nu
        L.check(self._lib.exo_cross_section_noalloc(self._h, int(slot), float(T), float(P_bar), p,
                                                    ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def cross_section_modit(self, slot: int, T: float, P_bar: float, precision="fp32", dln_gamma=0.1,
                            out=None, stream=None):
        """MODIT cross-section (Sec. 2.1.2) on the context's log-uniform grid."""
        p = _prec(precision)
        dt = torch.float32 if p == L.EXO_FP32_KAHAN else torch.float64
        if out is None:
            out = torch.empty(self.n_nu, dtype=dt, device=f"cuda:{self.device}")
        assert out.dtype == dt and out.is_contiguous() and out.numel() == self.n_nu
        L.check(self._lib.exo_cross_section_modit(self._h, int(slot), float(T), float(P_bar), p,
                                                  float(dln_gamma), ctypes.c_void_p(out.data_ptr()),
                                                  _stream(stream)))
        return out

    def select_lines(self, slot: int, log10_mmr: float, atmos: Atmos, T_atm: float, T_strength=None,
                     margin: int = 2, stream=None):
        """Weak-line pre-selection (App. G): (keep mask on the device, uint8 in
        the order the lines were given to set_lines; number kept)."""
        n = self._nlines.get(int(slot), 0)
        keep = torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")
        Ts = None if T_strength is None else _f64(T_strength)
        a, keep_alive = atmos.to_c()
        nk = ctypes.c_int64()
        L.check(self._lib.exo_select_lines(self._h, int(slot), float(log10_mmr), ctypes.byref(a), float(T_atm),
                                           L.dptr(Ts), 0 if Ts is None else int(Ts.size), int(margin),
                                           ctypes.c_void_p(keep.data_ptr()), ctypes.byref(nk), _stream(stream)))
        return keep, nk.value

    def _out_len(self, atmos: Atmos, response: Optional[Response]):
        if response is not None:
            return int(response.out_len)
        return int(atmos.grid_len) if atmos.grid_len else self.n_nu

    def emission_flux(self, atmos: Atmos, response: Optional[Response] = None, precision="fp32",
                      out=None, stream=None):
        p = _prec(precision)
        dt = torch.float32 if p == L.EXO_FP32_KAHAN else torch.float64
        n = self._out_len(atmos, response)
        if out is None:
            out = torch.empty(n, dtype=dt, device=f"cuda:{self.device}")
        assert out.dtype == dt and out.is_contiguous() and out.numel() == n
        a, keep = atmos.to_c()
        r = response.to_c() if response is not None else None
        L.check(self._lib.exo_emission_flux(self._h, ctypes.byref(a), ctypes.byref(r) if r is not None else None,
                                            p, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def flux_vjp(self, atmos: Atmos, response: Optional[Response], cot: torch.Tensor,
                 want_layers: bool = False, want_flux: bool = False, stream=None, precision="fp32"):
        """(grad[2 + M + 2], dL/dT_n or None, F or None) for cotangent dL/dF
        (float32 for "fp32", float64 for the FP64 forms)."""
        p = _prec(precision)
        dt = torch.float32 if p == L.EXO_FP32_KAHAN else torch.float64
        n = self._out_len(atmos, response)
        assert cot.dtype == dt and cot.is_contiguous() and cot.numel() == n
        m = len(atmos.species)
        grad = np.zeros(4 + m)
        layers = np.zeros(len(atmos.P_bar)) if want_layers else None
        flux = torch.empty(n, dtype=dt, device=cot.device) if want_flux else None
        a, keep = atmos.to_c()
        r = response.to_c() if response is not None else None
        L.check(self._lib.exo_flux_vjp(
            self._h, ctypes.byref(a), ctypes.byref(r) if r is not None else None, p,
            ctypes.c_void_p(cot.data_ptr()), L.dptr(grad), L.dptr(layers),
            ctypes.c_void_p(flux.data_ptr()) if flux is not None else None, _stream(stream)))
        return grad, layers, flux

    def loss_grad(self, atmos: Atmos, response: Optional[Response], data: torch.Tensor, sigma: torch.Tensor,
                  want_layers: bool = False, want_flux: bool = False, stream=None):
        """(loss, grad[2 + M + 2], dloss/dT_n or None, F or None) for the Gaussian
        likelihood loss = 1/2 sum ((data - F)/sigma)^2, in one forward pass."""
        n = self._out_len(atmos, response)
        for t in (data, sigma):
            assert t.dtype == torch.float32 and t.is_contiguous() and t.numel() == n
        m = len(atmos.species)
        grad = np.zeros(4 + m)
        layers = np.zeros(len(atmos.P_bar)) if want_layers else None
        flux = torch.empty(n, dtype=torch.float32, device=data.device) if want_flux else None
        loss = ctypes.c_double()
        a, keep = atmos.to_c()
        r = response.to_c() if response is not None else None
        L.check(self._lib.exo_loss_grad(
            self._h, ctypes.byref(a), ctypes.byref(r) if r is not None else None, L.EXO_FP32_KAHAN,
            ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(sigma.data_ptr()), ctypes.byref(loss),
            L.dptr(grad), L.dptr(layers), ctypes.c_void_p(flux.data_ptr()) if flux is not None else None,
            _stream(stream)))
        return loss.value, grad, layers, flux

    def flux_jvp(self, atmos: Atmos, response: Optional[Response], dtheta, dT_layers=None,
                 want_flux: bool = True, stream=None):
        """(F or None, J dtheta) on the device: the spectrum and its directional
        derivative along dtheta = (dT0, dalpha, dlog10X..., dRV, dvsini) plus the
        optional per-layer temperature tangent dT_layers."""
        n = self._out_len(atmos, response)
        m = len(atmos.species)
        dth = _f64(dtheta)
        assert dth.size == 4 + m
        dTl = None if dT_layers is None else _f64(dT_layers)
        assert dTl is None or dTl.size == len(atmos.P_bar)
        dev = f"cuda:{self.device}"
        flux = torch.empty(n, dtype=torch.float32, device=dev) if want_flux else None
        dflux = torch.empty(n, dtype=torch.float32, device=dev)
        a, keep = atmos.to_c()
        r = response.to_c() if response is not None else None
        L.check(self._lib.exo_flux_jvp(
            self._h, ctypes.byref(a), ctypes.byref(r) if r is not None else None, L.EXO_FP32_KAHAN,
            L.dptr(dth), L.dptr(dTl), ctypes.c_void_p(flux.data_ptr()) if flux is not None else None,
            ctypes.c_void_p(dflux.data_ptr()), _stream(stream)))
        return flux, dflux

    def broaden(self, F0: torch.Tensor, response: Response, grid_begin=0, grid_len=0, stream=None):
        assert F0.dtype == torch.float64 and F0.is_contiguous()
        out = torch.empty(int(response.out_len), dtype=torch.float64, device=F0.device)
        r = response.to_c()
        L.check(self._lib.exo_broaden(self._h, int(grid_begin), int(grid_len), ctypes.byref(r),
                                      ctypes.c_void_p(F0.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      _stream(stream)))
        return out

    # -- timing of the Voigt-sum kernel --------------------------------------
    def profile(self, on: bool = True):
        L.check(self._lib.exo_profile_enable(self._h, int(on)))

    def profile_read(self):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        ev = ctypes.c_double()
        L.check(self._lib.exo_profile_read(self._h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(ev)))
        return n.value, ms.value, ev.value

    def profile_read_near(self) -> float:
        """Pair evaluations of the profiled FP32 launches done in the near tier."""
        ev = ctypes.c_double()
        L.check(self._lib.exo_profile_read_near(self._h, ctypes.byref(ev)))
        return ev.value

    def profile_read_far_cut(self) -> float:
        """Far-tier pair evaluations of the profiled tangent launches, inside
        the outer reach, whose T-derivative polynomial stops at r^3."""
        ev = ctypes.c_double()
        L.check(self._lib.exo_profile_read_far_cut(self._h, ctypes.byref(ev)))
        return ev.value

    def profile_read_far_outer(self) -> float:
        """Far-tier pair evaluations of the profiled FP32 launches beyond the
        outer reach (value and tangent polynomials cut after r^2)."""
        ev = ctypes.c_double()
        L.check(self._lib.exo_profile_read_far_outer(self._h, ctypes.byref(ev)))
        return ev.value


def hjert_f32(x: torch.Tensor, a: torch.Tensor, want_L: bool = False, stream=None):
    lib = L.load_library()
    assert x.dtype == torch.float32 and a.dtype == torch.float32 and x.shape == a.shape
    x, a = x.contiguous(), a.contiguous()
    H = torch.empty_like(x)
    Lt = torch.empty_like(x) if want_L else None
    L.check(lib.exo_hjert_f32(x.numel(), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                              ctypes.c_void_p(H.data_ptr()),
                              ctypes.c_void_p(Lt.data_ptr()) if Lt is not None else None, _stream(stream)))
    return (H, Lt) if want_L else H


def hjert_f64(x: torch.Tensor, a: torch.Tensor, stream=None):
    lib = L.load_library()
    assert x.dtype == torch.float64 and a.dtype == torch.float64 and x.shape == a.shape
    x, a = x.contiguous(), a.contiguous()
    H = torch.empty_like(x)
    L.check(lib.exo_hjert_f64(x.numel(), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                              ctypes.c_void_p(H.data_ptr()), _stream(stream)))
    return H


def trans2e3(x: torch.Tensor, stream=None):
    lib = L.load_library()
    assert x.dtype == torch.float64
    x = x.contiguous()
    T = torch.empty_like(x)
    dT = torch.empty_like(x)
    L.check(lib.exo_trans2e3(x.numel(), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                             ctypes.c_void_p(dT.data_ptr()), _stream(stream)))
    return T, dT


class EmissionFlux(torch.autograd.Function):
    """F(theta), theta = (T0, alpha, log10 X_1..X_M, RV, vsini), with the HIP adjoint as backward.

    theta: float64 CPU tensor.  Returns the FP32 spectrum on the device.
    """

    @staticmethod
    def forward(ctx, theta: torch.Tensor, exo: Context, atmos: Atmos, response: Optional[Response]):
        th = theta.detach().cpu().numpy().astype(np.float64)
        m = len(atmos.species)
        a = Atmos(**{**atmos.__dict__, "T0": th[0], "alpha": th[1], "log10_mmr": list(th[2:2 + m])})
        r = None
        if response is not None:
            r = Response(**{**response.__dict__, "rv_kms": th[2 + m], "vsini_kms": th[3 + m]})
        ctx.exo, ctx.atmos, ctx.response = exo, a, r
        ctx.theta_dtype, ctx.ntheta = theta.dtype, theta.numel()
        return exo.emission_flux(a, r, "fp32")

    @staticmethod
    def backward(ctx, gF):
        g, _, _ = ctx.exo.flux_vjp(ctx.atmos, ctx.response, gF.detach().to(torch.float32).contiguous())
        out = torch.as_tensor(g[:ctx.ntheta], dtype=ctx.theta_dtype)
        return out, None, None, None

    @staticmethod
    def jvp(ctx, gtheta, *unused):
        """Forward mode (torch.autograd.forward_ad) through exo_flux_jvp."""
        dth = np.zeros(4 + len(ctx.atmos.species))
        g = gtheta.detach().cpu().numpy().astype(np.float64)
        dth[:g.size] = g
        _, dF = ctx.exo.flux_jvp(ctx.atmos, ctx.response, dth, want_flux=False)
        return dF


class LayerEmissionFlux(torch.autograd.Function):
    """F(T_layers, phi), phi = (log10 X_1..X_M, RV, vsini): the layer-by-layer
    temperature model (one free temperature per layer), with the HIP adjoint
    as backward and exo_flux_jvp as forward-mode derivative.

    T_layers: float64 CPU tensor [n_layers]; phi: float64 CPU tensor [M + 2].
    Returns the FP32 spectrum on the device.
    """

    @staticmethod
    def forward(ctx, T_layers: torch.Tensor, phi: torch.Tensor, exo: Context, atmos: Atmos,
                response: Response):
        T = T_layers.detach().cpu().numpy().astype(np.float64)
        ph = phi.detach().cpu().numpy().astype(np.float64)
        m = len(atmos.species)
        a = Atmos(**{**atmos.__dict__, "T_layers": T, "log10_mmr": list(ph[:m])})
        r = Response(**{**response.__dict__, "rv_kms": ph[m], "vsini_kms": ph[m + 1]})
        ctx.exo, ctx.atmos, ctx.response = exo, a, r
        ctx.dtypes = (T_layers.dtype, phi.dtype)
        return exo.emission_flux(a, r, "fp32")

    @staticmethod
    def backward(ctx, gF):
        g, gT, _ = ctx.exo.flux_vjp(ctx.atmos, ctx.response, gF.detach().to(torch.float32).contiguous(),
                                    want_layers=True)
        return (torch.as_tensor(gT, dtype=ctx.dtypes[0]), torch.as_tensor(g[2:], dtype=ctx.dtypes[1]),
                None, None, None)

    @staticmethod
    def jvp(ctx, gT, gphi, *unused):
        dth = np.zeros(4 + len(ctx.atmos.species))
        dTl = None
        if gphi is not None:
            dth[2:] = gphi.detach().cpu().numpy().astype(np.float64)
        if gT is not None:
            dTl = gT.detach().cpu().numpy().astype(np.float64)
        _, dF = ctx.exo.flux_jvp(ctx.atmos, ctx.response, dth, dTl, want_flux=False)
        return dF
