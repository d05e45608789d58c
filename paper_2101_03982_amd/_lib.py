"""ctypes declarations of liblbm.so (the C ABI in include/lbm.h).

Argument marshalling only.  The library must have been built in-tree
(``python -m paper_2101_03982_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

SETS = ("D2Q9", "D2Q19", "D2Q25", "D3Q13", "D3Q21", "D3Q27", "D3V27", "D3Q45")
STORAGES = ("f64", "f32", "bf16", "f16")
BOUNDARIES = ("periodic", "extrapolate")
SUPPORTS = ("uniform", "glc")
ROUNDINGS = ("nearest", "stochastic")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EUNSUPPORTED, LBM_EDIVERGED = 0, -1, -2, -3, -4, -5


class Options(ctypes.Structure):
    _fields_ = [
        ("storage", ctypes.c_int32),
        ("stencil", ctypes.c_int32),
        ("compressible", ctypes.c_int32),
        ("boundary", ctypes.c_int32 * 3),
        ("energy_f64", ctypes.c_int32),
        ("support", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("cs", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("prandtl", ctypes.c_double),
        ("rounding", ctypes.c_int32),
        ("seed", ctypes.c_uint32),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double),
        ("momentum", ctypes.c_double * 3),
        ("ke", ctypes.c_double),
        ("energy", ctypes.c_double),
        ("min_rho", ctypes.c_double),
        ("min_theta", ctypes.c_double),
        ("nonfinite", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class LbmError(RuntimeError):
    def __init__(self, code, what, msg):
        super().__init__("%s: %s (%d): %s" % (what, _strerror(code), code, msg))
        self.code = code


_lib = None
_V, _P, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double

_SIGS = {
    "lbm_abi_version": (_I32, []),
    "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_default_options": (None, [ctypes.POINTER(Options)]),
    "lbm_create": (ctypes.c_int, [ctypes.POINTER(_V), _I32, ctypes.POINTER(_I64), _D, _I32, ctypes.POINTER(Options)]),
    "lbm_destroy": (ctypes.c_int, [_V]),
    "lbm_state_bytes": (ctypes.c_size_t, [_V]),
    "lbm_bind": (ctypes.c_int, [_V, _P, _P]),
    "lbm_state": (_P, [_V]),
    "lbm_init_equilibrium": (ctypes.c_int, [_V, _P, _P, _P]),
    "lbm_get_state": (ctypes.c_int, [_V, _P]),
    "lbm_set_state": (ctypes.c_int, [_V, _P]),
    "lbm_step": (ctypes.c_int, [_V, _I64]),
    "lbm_step_into": (ctypes.c_int, [_V, _P, _P]),
    "lbm_moments": (ctypes.c_int, [_V, _P, _P, _P, _P, ctypes.POINTER(Diag)]),
    "lbm_moments_noalloc": (ctypes.c_int, [_V, _P, _P, _P, _P, ctypes.POINTER(Diag)]),
    "lbm_enstrophy": (ctypes.c_int, [_V, _P, _I32, ctypes.POINTER(_D)]),
    "lbm_sync": (ctypes.c_int, [_V]),
    "lbm_set_stream": (ctypes.c_int, [_V, _P]),
    "lbm_stream": (ctypes.c_int, [_V, _P, _P]),
    "lbm_adjoint_collide": (ctypes.c_int, [_V, _P, _P, _P]),
    "lbm_adjoint_stream": (ctypes.c_int, [_V, _P, _P]),
    "lbm_adjoint_step": (ctypes.c_int, [_V, _P, _P, _P]),
    "lbm_ke_adjoint": (ctypes.c_int, [_V, _P, _P]),
    "lbm_init_equilibrium_adjoint": (ctypes.c_int, [_V, _P, _P, _P, _P]),
    "lbm_float_moment_defects": (ctypes.c_int, [_I32, ctypes.POINTER(_D)]),
    "lbm_stencil": (ctypes.c_int, [_I32, _D, _D, _D, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_D)]),
    "lbm_set_table": (ctypes.c_int, [_I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                     ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
}


def lib():
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm.so is not built (%s); run python -m paper_2101_03982_amd.build" % LIB_PATH)
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def _strerror(code):
    try:
        return lib().lbm_strerror(code).decode()
    except Exception:  # noqa: BLE001 - only used to format a message
        return "status"


def check(code, what):
    if code != LBM_OK:
        raise LbmError(code, what, lib().lbm_last_error().decode())
    return code
