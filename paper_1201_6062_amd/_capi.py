"""ctypes declarations of the C ABI in include/tdse.h (argument marshalling only).

The library must be built in-tree (python -m paper_1201_6062_amd.build); loading
fails loudly otherwise. torch is imported first so that the library binds to
the HIP runtime torch already loaded (both carry SONAME libamdhip64.so.7) and
device pointers and streams are shared.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdse.so")

TDSE_OK, TDSE_E_INVAL, TDSE_E_NOMEM, TDSE_E_HIP, TDSE_E_UNSUPPORTED, TDSE_E_UNSTABLE = range(6)
TDSE_RK4, TDSE_TAYLOR, TDSE_LANCZOS, TDSE_RKF45 = 0, 1, 2, 3
TDSE_LENGTH, TDSE_VELOCITY = 0, 1
STATUS_NAMES = {0: "TDSE_OK", 1: "TDSE_E_INVAL", 2: "TDSE_E_NOMEM", 3: "TDSE_E_HIP",
                4: "TDSE_E_UNSUPPORTED", 5: "TDSE_E_UNSTABLE"}

# Every function include/tdse.h declares, with (restype, argtypes).
_vp = ctypes.c_void_p
_i32, _i64, _d = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_st = ctypes.c_int
SIGNATURES = {
    "tdse_abi_version": (ctypes.c_int, []),
    "tdse_last_error": (ctypes.c_char_p, []),
    "tdse_create": (_st, [ctypes.POINTER(_vp), _vp, _vp, _i32, _i32, _i32, _vp]),
    "tdse_create_gauge": (_st, [ctypes.POINTER(_vp), _vp, _vp, _st, _i32, _i32, _i32, _vp]),
    "tdse_destroy": (_st, [_vp]),
    "tdse_plan_shape": (_st, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "tdse_hmul": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "tdse_propagate": (_st, [_vp, _st, _i32, _d, _i64, _vp, _vp, _vp, _vp, _i32, _vp]),
    "tdse_propagate_noalloc": (_st, [_vp, _st, _i32, _d, _i64, _vp, _vp, _vp, _vp, _i32, _vp]),
    "tdse_propagate_rkf45": (_st, [_vp, _d, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "tdse_propagate_adaptive": (_st, [_vp, _d, _d, _d, _d, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_i64), _vp]),
    "tdse_check_stability": (_st, [_vp, _st, _i32, _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "tdse_adjoint": (_st, [_vp, _st, _i32, _d, _i64, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "tdse_group_create": (_st, [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp), _vp]),
    "tdse_group_propagate": (_st, [_vp, _st, _i32, _d, ctypes.POINTER(_i64), ctypes.POINTER(_vp),
                                   ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
    "tdse_group_destroy": (_st, [_vp]),
    "tdse_tune": (_st, [_i32, _i32, _i32, ctypes.c_char_p]),
}

# void (*tdse_field_fn)(double t, double h, double *samples, void *ctx)
FIELD_FN = ctypes.CFUNCTYPE(None, _d, _d, ctypes.POINTER(_d), _vp)

_lib = None


class TdseError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load(require_torch: bool = True):
    """Load libtdse.so (built in-tree). Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if require_torch:
        import torch  # noqa: F401  (bind to torch's HIP runtime)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1201_6062_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != TDSE_OK:
        msg = load().tdse_last_error().decode(errors="replace")
        raise TdseError(status, msg)
