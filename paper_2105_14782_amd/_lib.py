"""ctypes binding of libexohip.so (argument marshalling only).

The library must be built in-tree (``python -m paper_2105_14782_amd.build``).
Nothing here computes any part of the model: every step runs in the HIP
kernels behind the C ABI of ``include/exohip.h``.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("EXO_LIB_PATH") or os.path.join(_HERE, "libexohip.so")

EXO_OK, EXO_EINVAL, EXO_ENOMEM, EXO_ENOTSET, EXO_EDEVICE = 0, -1, -2, -3, -4
EXO_FP32_KAHAN, EXO_FP64, EXO_FP64_TILED = 0, 1, 2
EXO_QR_POWER, EXO_QR_TABLE = 0, 1
EXO_FB_PLANCK_BOTTOM, EXO_FB_ZERO = 0, 1
EXO_OPACITY_LPF, EXO_OPACITY_MODIT = 0, 1
EXO_MAX_SPECIES = 64

_c_dp = ctypes.POINTER(ctypes.c_double)
_c_ip = ctypes.POINTER(ctypes.c_int32)


class ExoAtmos(ctypes.Structure):
    _fields_ = [
        ("n_layers", ctypes.c_int32),
        ("P_bar", _c_dp),
        ("T0_K", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("n_species", ctypes.c_int32),
        ("species", _c_ip),
        ("log10_mmr", _c_dp),
        ("g_cgs", ctypes.c_double),
        ("mmw", ctypes.c_double),
        ("cia_alpha0", ctypes.c_double),
        ("cia_Tpow", ctypes.c_double),
        ("cia_slope", ctypes.c_double),
        ("cia_nu_c", ctypes.c_double),
        ("vmr_h2", ctypes.c_double),
        ("bottom", ctypes.c_int32),
        ("grid_begin", ctypes.c_int64),
        ("grid_len", ctypes.c_int64),
        ("T_layers", _c_dp),
        ("opacity", ctypes.c_int32),
        ("modit_dln_gamma", ctypes.c_double),
    ]


class ExoResponse(ctypes.Structure):
    _fields_ = [
        ("rv_kms", ctypes.c_double),
        ("vsini_kms", ctypes.c_double),
        ("u1", ctypes.c_double),
        ("u2", ctypes.c_double),
        ("R_inst", ctypes.c_double),
        ("out_begin", ctypes.c_int64),
        ("out_len", ctypes.c_int64),
    ]


class ExoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"exohip error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libexohip.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2105_14782_amd.build`")
    # PyTorch ships its own HIP runtime.  When this library (linked against the
    # system one) is loaded first and PyTorch then initialises the device, this
    # library's runtime no longer finds it; loading PyTorch first avoids that.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    V, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "exo_last_error": ([], ctypes.c_char_p),
        "exo_version": ([], ctypes.c_char_p),
        "exo_create": ([I, ctypes.POINTER(V)], I),
        "exo_destroy": ([V], I),
        "exo_set_lines": ([V, I, I64, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, D, I, _c_dp, I], I),
        "exo_set_grid": ([V, I64, _c_dp], I),
        "exo_cross_section": ([V, I, D, D, I, V, V], I),
        "exo_cross_section_noalloc": ([V, I, D, D, I, V, V], I),
        "exo_emission_flux": ([V, ctypes.POINTER(ExoAtmos), ctypes.POINTER(ExoResponse), I, V, V], I),
        "exo_flux_vjp": ([V, ctypes.POINTER(ExoAtmos), ctypes.POINTER(ExoResponse), I, V, _c_dp, _c_dp, V, V], I),
        "exo_broaden": ([V, I64, I64, ctypes.POINTER(ExoResponse), V, V, V], I),
        "exo_hjert_f32": ([I64, V, V, V, V, V], I),
        "exo_hjert_f64": ([I64, V, V, V, V], I),
        "exo_trans2e3": ([I64, V, V, V, V], I),
        "exo_profile_enable": ([V, I], I),
        "exo_profile_read": ([V, ctypes.POINTER(I64), ctypes.POINTER(D), ctypes.POINTER(D)], I),
        "exo_profile_read_near": ([V, ctypes.POINTER(D)], I),
        "exo_profile_read_far_cut": ([V, ctypes.POINTER(D)], I),
        "exo_profile_read_far_outer": ([V, ctypes.POINTER(D)], I),
        "exo_cross_section_modit": ([V, I, D, D, I, D, V, V], I),
        "exo_select_lines": ([V, I, D, ctypes.POINTER(ExoAtmos), D, _c_dp, I, I, V,
                              ctypes.POINTER(I64), V], I),
        "exo_flux_jvp": ([V, ctypes.POINTER(ExoAtmos), ctypes.POINTER(ExoResponse), I, _c_dp, _c_dp, V, V, V], I),
        "exo_loss_grad": ([V, ctypes.POINTER(ExoAtmos), ctypes.POINTER(ExoResponse), I, V, V,
                           ctypes.POINTER(D), _c_dp, _c_dp, V, V], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def check(rc: int):
    if rc != EXO_OK:
        msg = _lib.exo_last_error().decode() if _lib is not None else ""
        raise ExoError(rc, msg)


def dptr(a):
    """ctypes double* of a C-contiguous float64 numpy array (or None)."""
    if a is None:
        return None
    return a.ctypes.data_as(_c_dp)
