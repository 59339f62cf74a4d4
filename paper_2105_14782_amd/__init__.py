"""exohip: MI355X-native direct line-by-line emission spectrum model.

HIP kernels for gfx950 behind the C ABI of ``include/exohip.h``; this
package is the thin Python binding (ctypes + PyTorch device memory/streams).
"""
from ._lib import (  # noqa: F401
    load_library, ExoError, LIB_PATH, EXO_FP32_KAHAN, EXO_FP64, EXO_FB_PLANCK_BOTTOM, EXO_FB_ZERO,
    EXO_QR_POWER, EXO_QR_TABLE, EXO_EINVAL, EXO_ENOMEM, EXO_ENOTSET, EXO_EDEVICE,
)


def __getattr__(name):
    # the torch-dependent front end is imported lazily
    if name in ("Context", "Atmos", "Response", "EmissionFlux", "LayerEmissionFlux", "hjert_f32", "hjert_f64",
                "trans2e3"):
        from . import api
        return getattr(api, name)
    if name in ("Server", "ServeRequest"):
        from . import serve
        return getattr(serve, name)
    raise AttributeError(name)
