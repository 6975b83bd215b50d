"""ctypes loader for libsetd.so (the HIP library built by build.py).

The library must exist: nothing here falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsetd.so")

# status codes and enums (include/setd.h)
SETD_OK = 0
SETD_EINVAL = -1
SETD_ENOMEM = -2
SETD_EHIP = -3
SETD_ENONFINITE = -4
SETD_EUNSUPPORTED = -5

PREC_F64 = 0
PREC_F32 = 1
PREC_BF16X3 = 2
PREC_BF16X2 = 3
PREC_I8X4 = 4

G_NONE = 0
G_SCHNAKENBERG = 1
G_FHN = 2

STAGE_2 = 2
STAGE_3 = 3
STAGE_F = 4

# exported symbols with their C signatures
_c_int, _c_i64, _c_double, _vp, _c_size = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
SIGNATURES = {
    "setd_phi_matrices": (_c_int, [_vp, _c_i64, _c_double, _c_int, _vp, _vp]),
    "setd_tucker_apply": (_c_int, [_vp, _vp, _c_int, ctypes.POINTER(_c_i64), ctypes.POINTER(_vp), _c_double,
                                   _c_double, _c_int, _vp, _c_size, _vp]),
    "setd_tucker_workspace_bytes": (_c_size, [_c_int, ctypes.POINTER(_c_i64), _c_int]),
    "setd_tucker_apply_noalloc": (_c_int, [_vp, _vp, _c_int, ctypes.POINTER(_c_i64), ctypes.POINTER(_vp),
                                           _c_double, _c_double, _c_int, _vp]),
    "setd_release_workspace": (_c_int, []),
    "setd_ctx_create": (_c_int, [ctypes.POINTER(_vp), _c_int, ctypes.POINTER(_c_i64), _c_int, ctypes.POINTER(_vp),
                                 _c_double, _c_int, _vp]),
    "setd_ctx_destroy": (_c_int, [_vp]),
    "setd_split_phi_apply": (_c_int, [_vp, _c_int, _c_int, _c_int, _vp, _vp, _c_double, _c_double, _vp]),
    "setd_etd_step": (_c_int, [_vp, _vp, _c_int, _c_double, _c_int, ctypes.POINTER(_c_double), _c_int, _vp]),
    "setd_etd_step_record": (_c_int, [_vp, _vp, _c_double, _c_int, ctypes.POINTER(_c_double), _c_int, _vp, _vp]),
    "setd_etd_adjoint_step_recorded": (_c_int, [_vp, _vp, _vp, _vp, _c_int, ctypes.POINTER(_c_double), _c_int,
                                                _c_int, _vp, _vp]),
    "setd_etd2_step": (_c_int, [_vp, _vp, _c_int, _c_double, _c_int, ctypes.POINTER(_c_double), _c_int, _vp]),
    "setd_etd_cplx_step": (_c_int, [_vp, _vp, _c_int, _c_double, _c_int, ctypes.POINTER(_c_double), _c_int, _vp]),
    "setd_field_norms": (_c_int, [_vp, _vp, _c_i64, ctypes.POINTER(_c_double), _vp]),
    "setd_last_error": (ctypes.c_char_p, []),
    "setd_sync": (_c_int, [_vp]),
    "setd_version": (ctypes.c_char_p, []),
    "setd_profile_enable": (_c_int, [_c_int]),
    "setd_profile_read": (_c_int, [ctypes.POINTER(_c_double), _c_int]),
    "setd_etd_adjoint_step": (_c_int, [_vp, _vp, _vp, _c_int, ctypes.POINTER(_c_double), _c_int, _c_int, _vp,
                                       _vp]),
    "setd_batch_create": (_c_int, [ctypes.POINTER(_vp), _c_int, _c_int, ctypes.POINTER(_c_i64), _c_int,
                                   ctypes.POINTER(_vp), _c_double, _c_int, _vp]),
    "setd_batch_destroy": (_c_int, [_vp]),
    "setd_batch_layout": (_c_int, [_vp, ctypes.POINTER(_c_i64), ctypes.POINTER(_c_i64)]),
    "setd_batch_step": (_c_int, [_vp, _vp, _c_int, _c_int, ctypes.POINTER(_c_double), _c_int, _vp]),
    "setd_batch_tune": (_c_int, [_vp, _vp]),
    "setd_batch_set_tiles": (_c_int, [_vp, ctypes.POINTER(_c_int)]),
    "setd_batch_info": (_c_int, [_vp, ctypes.POINTER(_c_i64)]),
}

BATCH_INFO = 10
NOALLOC_SCRATCH_BYTES = 64 << 20   # SETD_NOALLOC_SCRATCH_BYTES

PROF_CLASSES = ("mode1_f64", "modeB_f64", "mode1_lp", "modeB_lp", "pointwise", "modeB_panel_f64")

_lib = None


class SetdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("setd error %d: %s" % (code, msg))
        self.code = code


def load(path: str = LIB_PATH):
    """Load libsetd.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libsetd.so not found at %s: build it with `python -m paper_2310_07551_amd.build` "
                           "(there is no fallback implementation)" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != SETD_OK:
        raise SetdError(rc, load().setd_last_error().decode())
    return rc
