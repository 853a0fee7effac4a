"""MI355X-native Reduced Basis Decomposition.

Reduced Basis Decomposition (Y. Chen, arXiv 1503.05947) compresses a data
matrix X (m x n, one sample per column) as Y T with an orthonormal Y built
greedily (Algorithm 1, section 3.1) and T = Y'X.  Every step of that loop runs
in the HIP kernels of ``librbd.so`` (C ABI in include/rbd.h); this module only
marshals torch tensors (device memory, streams) into that ABI.  There is no
fallback: without the built library every entry point raises.

    res = fit(X, tol=1e-4, d_max=256, rel=True)     # X: cuda tensor (m, n)
    res.Y, res.T, res.pivots, res.col_err, res.err_hist, res.d
    Tv, err = project(res.Y, V)                     # out-of-sample compression
"""
from __future__ import annotations

from dataclasses import dataclass

from . import _lib
from ._lib import (LibraryMissing, RBD_MAX_D, RBD_STOP_BREAK, RBD_STOP_DMAX, RBD_STOP_TOL, load,
                   status_string)

__all__ = ["fit", "fit_into", "FitBuffers", "FitResult", "project", "load", "status_string",
           "LibraryMissing", "RBD_MAX_D"]

STOP_NAMES = {0: "error", RBD_STOP_TOL: "tol", RBD_STOP_DMAX: "dmax", RBD_STOP_BREAK: "break"}


def _torch():
    import torch
    return torch


def dtype_code(dtype) -> int:
    torch = _torch()
    table = {torch.float32: _lib.RBD_F32, torch.bfloat16: _lib.RBD_BF16,
             torch.float16: _lib.RBD_F16, torch.float64: _lib.RBD_F64}
    if dtype not in table:
        raise TypeError(f"unsupported storage dtype {dtype}")
    return table[dtype]


def _check_matrix(A, name):
    torch = _torch()
    if not isinstance(A, torch.Tensor) or A.dim() != 2:
        raise TypeError(f"{name} must be a 2-D torch tensor")
    if A.device.type != "cuda":
        raise ValueError(f"{name} must live in GPU memory")
    if A.stride(1) != 1 or A.stride(0) < A.shape[1]:
        raise ValueError(f"{name} must be row-major with unit column stride")


@dataclass
class FitResult:
    Y: object          # (m, d) float64
    T: object          # (d, n) float64
    pivots: object     # (d,) int64
    col_err: object    # (n,) float64
    err_hist: object   # (d+1,) float64
    d: int
    stop: str


class FitBuffers:
    """Outputs and workspace of one rbd_fit configuration, reusable across calls."""

    def __init__(self, m: int, n: int, d_max: int, dtype, device):
        torch = _torch()
        self.m, self.n, self.d_max, self.dtype = int(m), int(n), int(d_max), dtype
        code = dtype_code(dtype)
        self.ws_bytes = _lib.fit_workspace_size(self.m, self.n, self.d_max, code)
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        self.Y = torch.empty((self.m, self.d_max), **f64)
        self.T = torch.empty((self.d_max, self.n), **f64)
        self.pivots = torch.empty(self.d_max, dtype=torch.int64, device=dev)
        self.col_err = torch.empty(self.n, **f64)
        self.err_hist = torch.empty(self.d_max + 1, **f64)
        self.ints = torch.empty(4, dtype=torch.int32, device=dev)     # d, status, stop reason
        self.workspace = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=dev)

    def result(self) -> FitResult:
        d, status, stop = (int(v) for v in self.ints[:3].tolist())
        if status != _lib.RBD_OK:
            raise FloatingPointError(f"rbd_fit: {status_string(status)}")
        return FitResult(Y=self.Y[:, :d], T=self.T[:d], pivots=self.pivots[:d], col_err=self.col_err,
                         err_hist=self.err_hist[: d + 1], d=d, stop=STOP_NAMES.get(stop, str(stop)))


def fit_into(bufs: FitBuffers, X, tol: float = 0.0, rel: bool = False, start: int = -1, stream=None) -> None:
    """Enqueue rbd_fit on ``stream`` (default: torch's current stream) without waiting."""
    torch = _torch()
    _check_matrix(X, "X")
    if tuple(X.shape) != (bufs.m, bufs.n) or X.dtype != bufs.dtype:
        raise ValueError("X does not match the buffers' shape/dtype")
    lib = load()
    with torch.cuda.device(X.device):
        s = stream if stream is not None else torch.cuda.current_stream(X.device)
        ints = bufs.ints.data_ptr()
        rc = lib.rbd_fit(X.data_ptr(), dtype_code(X.dtype), bufs.m, bufs.n, X.stride(0), float(tol),
                         _lib.RBD_TOL_REL if rel else _lib.RBD_TOL_ABS, bufs.d_max, int(start),
                         bufs.Y.data_ptr(), bufs.T.data_ptr(), bufs.pivots.data_ptr(), bufs.col_err.data_ptr(),
                         bufs.err_hist.data_ptr(), ints, ints + 4, ints + 8,
                         bufs.workspace.data_ptr(), bufs.workspace.numel(), s.cuda_stream)
    _lib.check(rc, "rbd_fit")


def fit(X, tol: float = 0.0, d_max: int = 64, rel: bool = False, start: int = -1, stream=None) -> FitResult:
    """Algorithm 1 on a device matrix X (m x n, f32/bf16/f16/f64 storage).

    ``tol`` is eps_R (absolute, or relative to max_j ||x_j|| when ``rel``);
    ``start < 0`` starts from the column of largest norm.  Waits for the
    device and returns views of the first d basis vectors / rows of T.
    """
    torch = _torch()
    bufs = FitBuffers(X.shape[0], X.shape[1], d_max, X.dtype, X.device)
    fit_into(bufs, X, tol=tol, rel=rel, start=start, stream=stream)
    (stream or torch.cuda.current_stream(X.device)).synchronize()
    return bufs.result()


def project(Y, V, stream=None):
    """Out-of-sample compression: returns (Y'V, ||v_q - Y Y'v_q|| per column)."""
    torch = _torch()
    _check_matrix(Y, "Y")
    _check_matrix(V, "V")
    if Y.dtype != torch.float64:
        raise TypeError("Y must be float64")
    m, d = Y.shape
    if V.shape[0] != m:
        raise ValueError("V must have as many rows as Y")
    k = V.shape[1]
    code = dtype_code(V.dtype)
    ws = _lib.project_workspace_size(m, d, k, code)
    dev = V.device
    Tv = torch.empty((d, k), dtype=torch.float64, device=dev)
    err = torch.empty(k, dtype=torch.float64, device=dev)
    work = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
    lib = load()
    with torch.cuda.device(dev):
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        rc = lib.rbd_project(Y.data_ptr(), Y.stride(0), m, d, V.data_ptr(), code, k, V.stride(0),
                             Tv.data_ptr(), err.data_ptr(), work.data_ptr(), work.numel(), s.cuda_stream)
        _lib.check(rc, "rbd_project")
        s.synchronize()
    return Tv, err
