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
# rbd_basis
RBD_BASIS_F64, RBD_BASIS_F32 = 0, 1
# status codes
RBD_OK, RBD_EINVAL, RBD_ENONFINITE, RBD_EWORKSPACE, RBD_EDEVICE, RBD_EMATRIX, RBD_ETOOLARGE = 0, -1, -2, -3, -4, -5, -6
RBD_NOALLOC_MAX_BYTES = 64 << 20
# stop reasons
RBD_STOP_TOL, RBD_STOP_DMAX, RBD_STOP_BREAK = 1, 2, 3
RBD_MAX_D = 1024
PHASES = ("colnorm", "init", "cgs1", "cgs2", "xscan", "update", "resid", "resid_finish", "epilogue", "loop")

# every symbol include/rbd.h declares, with its ctypes signature
_i64, _i32, _sz, _vp, _dp = ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double
SIGNATURES = {
    "rbd_fit_workspace_size": (ctypes.c_int, [_i64, _i64, _i32, ctypes.c_int, ctypes.POINTER(_sz)]),
    "rbd_fit": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _i64, _i64, _dp, ctypes.c_int, _i32, _i64,
                               _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "rbd_fit_basis_workspace_size": (ctypes.c_int, [_i64, _i64, _i32, ctypes.c_int, ctypes.c_int,
                                                    ctypes.POINTER(_sz)]),
    "rbd_fit_basis": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _i64, _i64, _dp, ctypes.c_int, _i32, _i64, ctypes.c_int,
                                     _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "rbd_fit_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _i64, _i64, _dp, ctypes.c_int, _i32, _i64,
                                       _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rbd_fit_weighted": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _i64, _i64, _vp, _dp, ctypes.c_int, _i32, _i64,
                                        _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "rbd_fit_graph_create": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _i64, _i64, _vp, _dp, ctypes.c_int, _i32,
                                            _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp,
                                            ctypes.POINTER(_vp)]),
    "rbd_fit_graph_launch": (ctypes.c_int, [_vp, _vp]),
    "rbd_fit_graph_destroy": (ctypes.c_int, [_vp]),
    "rbd_fit_spd_workspace_size": (ctypes.c_int, [_i64, _i64, _i32, ctypes.c_int, ctypes.POINTER(_sz)]),
    "rbd_fit_spd": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _i64, _i64, _vp, _vp, _vp, _i64, _dp, ctypes.c_int, _i32,
                                   _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "rbd_project_workspace_size": (ctypes.c_int, [_i64, _i32, _i64, ctypes.c_int, ctypes.POINTER(_sz)]),
    "rbd_project": (ctypes.c_int, [_vp, _i64, _i64, _i32, _vp, ctypes.c_int, _i64, _i64, _vp, _vp,
                                   _vp, _sz, _vp]),
    "rbd_batch_plan": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp, _vp, _vp]),
    "rbd_fit_batched": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _i32, _dp, ctypes.c_int, _i32, None,
                                       _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp]),
    "rbd_batched_autotune": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _i32, _dp, ctypes.c_int, _i32, _i32,
                                            _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp, _vp, _vp]),
    "rbd_reconstruct": (ctypes.c_int, [_vp, _i64, _i64, _i32, _vp, _i64, _i64, _vp, _i64, _vp]),
    "rbd_classify_workspace_size": (ctypes.c_int, [_i64, _i32, _i64, ctypes.POINTER(_sz)]),
    "rbd_classify": (ctypes.c_int, [_vp, _i64, _i64, _i32, _vp, _i64, _i64, _vp, _vp, ctypes.c_int, _i64, _i64,
                                    _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "rbd_reconstruct_backward_workspace_size": (ctypes.c_int, [_i64, _i64, _i32, ctypes.POINTER(_sz)]),
    "rbd_reconstruct_backward": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _vp, ctypes.c_int, _i64, _vp, _i64, _vp,
                                                _i64, _vp, _i64, _i64, _i32, _vp, _i64, _vp, _sz, _vp]),
    "rbd_profiler_begin": (ctypes.c_int, [ctypes.c_uint32]),
    "rbd_profiler_end": (ctypes.c_int, [_vp, _vp, _i32, _vp, _i64, _vp]),
    "rbd_read_stream": (ctypes.c_int, [_vp, _sz, ctypes.c_int, _vp, _vp]),
    "rbd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rbd_version": (ctypes.c_char_p, []),
}



class BatchSizes(ctypes.Structure):
    _fields_ = [("x_elems", ctypes.c_int64), ("y_elems", ctypes.c_int64), ("t_elems", ctypes.c_int64),
                ("c_elems", ctypes.c_int64), ("max_m", ctypes.c_int64), ("max_n", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_size_t)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32)]


# the by-value struct argument of rbd_fit_batched
SIGNATURES["rbd_fit_batched"][1][8] = BatchConfig

_lib = None


class LibraryMissing(ImportError):
    pass


def load(path: str = None):
    """Load librbd.so (built by ``_build.build_library``); raises if it is missing.
    RBD_LIBRARY in the environment names another build of the same library (the
    host-sanitized one of ``_build.build_host_sanitized``, for CPU tests)."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = os.environ.get("RBD_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} not found: build it with __graft_entry__.build() "
                             "(there is no fallback implementation)")
    # torch brings its own HIP runtime; it must be the one librbd binds to, or
    # torch's streams and memory are foreign to the library's launches
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
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


def fit_workspace_size(m: int, n: int, d_max: int, dtype: int, basis: int = RBD_BASIS_F64) -> int:
    out = ctypes.c_size_t(0)
    check(load().rbd_fit_basis_workspace_size(m, n, d_max, dtype, basis, ctypes.byref(out)),
          "rbd_fit_basis_workspace_size")
    return out.value


def project_workspace_size(m: int, d: int, k: int, dtype: int) -> int:
    out = ctypes.c_size_t(0)
    check(load().rbd_project_workspace_size(m, d, k, dtype, ctypes.byref(out)), "rbd_project_workspace_size")
    return out.value


def fit_spd_workspace_size(m: int, n: int, d_max: int, dtype: int) -> int:
    out = ctypes.c_size_t(0)
    check(load().rbd_fit_spd_workspace_size(m, n, d_max, dtype, ctypes.byref(out)), "rbd_fit_spd_workspace_size")
    return out.value


def classify_workspace_size(m: int, d: int, k: int) -> int:
    out = ctypes.c_size_t(0)
    check(load().rbd_classify_workspace_size(m, d, k, ctypes.byref(out)), "rbd_classify_workspace_size")
    return out.value


class Profiler:
    """Context manager around rbd_profiler_begin/end (HIP events on the fit's stream)."""

    def __init__(self, phases=PHASES, max_steps=RBD_MAX_D):
        self.mask = 0
        for p in phases:
            self.mask |= 1 << PHASES.index(p)
        self.max_steps = max_steps
        self.phase_ms = {}
        self.launches = {}
        self.step_end_ms = []

    def __enter__(self):
        check(load().rbd_profiler_begin(self.mask), "rbd_profiler_begin")
        return self

    def __exit__(self, *exc):
        n = len(PHASES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        steps = (ctypes.c_double * self.max_steps)()
        nout = ctypes.c_int64(0)
        rc = load().rbd_profiler_end(ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(cnt, ctypes.c_void_p), n,
                                     ctypes.cast(steps, ctypes.c_void_p), self.max_steps, ctypes.byref(nout))
        if exc[0] is None:
            check(rc, "rbd_profiler_end")
        self.phase_ms = {p: ms[i] for i, p in enumerate(PHASES)}
        self.launches = {p: cnt[i] for i, p in enumerate(PHASES)}
        self.step_end_ms = [steps[i] for i in range(min(nout.value, self.max_steps))]
        return False

    def avg_ms(self, phase):
        c = self.launches.get(phase, 0)
        return self.phase_ms[phase] / c if c else float("nan")
