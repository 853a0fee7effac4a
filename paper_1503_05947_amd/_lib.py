"""ctypes view of the C ABI in include/rbd.h (no torch, no GPU needed to load)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbd.so")

# rbd_dtype
RBD_F32, RBD_BF16, RBD_F16, RBD_F64 = 0, 1, 2, 3
# rbd_tol_mode
RBD_TOL_ABS, RBD_TOL_REL = 0, 1
# status codes
RBD_OK, RBD_EINVAL, RBD_ENONFINITE, RBD_EWORKSPACE, RBD_EDEVICE = 0, -1, -2, -3, -4
# stop reasons
RBD_STOP_TOL, RBD_STOP_DMAX, RBD_STOP_BREAK = 1, 2, 3
RBD_MAX_D = 1024

# every symbol include/rbd.h declares, with its ctypes signature
_i64, _i32, _sz, _vp, _dp = ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double
SIGNATURES = {
    "rbd_fit_workspace_size": (ctypes.c_int, [_i64, _i64, _i32, ctypes.c_int, ctypes.POINTER(_sz)]),
    "rbd_fit": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _i64, _i64, _dp, ctypes.c_int, _i32, _i64,
                               _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "rbd_project_workspace_size": (ctypes.c_int, [_i64, _i32, _i64, ctypes.c_int, ctypes.POINTER(_sz)]),
    "rbd_project": (ctypes.c_int, [_vp, _i64, _i64, _i32, _vp, ctypes.c_int, _i64, _i64, _vp, _vp,
                                   _vp, _sz, _vp]),
    "rbd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rbd_version": (ctypes.c_char_p, []),
}

_lib = None


class LibraryMissing(ImportError):
    pass


def load(path: str = LIB_PATH):
    """Load librbd.so (built by ``_build.build_library``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} not found: build it with __graft_entry__.build() "
                             "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().rbd_status_string(int(code)).decode()


def check(code: int, what: str) -> None:
    if code != RBD_OK:
        raise RuntimeError(f"{what}: {status_string(code)} (code {code})")


def fit_workspace_size(m: int, n: int, d_max: int, dtype: int) -> int:
    out = ctypes.c_size_t(0)
    check(load().rbd_fit_workspace_size(m, n, d_max, dtype, ctypes.byref(out)), "rbd_fit_workspace_size")
    return out.value


def project_workspace_size(m: int, d: int, k: int, dtype: int) -> int:
    out = ctypes.c_size_t(0)
    check(load().rbd_project_workspace_size(m, d, k, dtype, ctypes.byref(out)), "rbd_project_workspace_size")
    return out.value
