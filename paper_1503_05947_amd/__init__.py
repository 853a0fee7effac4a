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

__all__ = ["fit", "fit_into", "FitBuffers", "FitResult", "project", "fit_batched", "BatchPlan", "BatchConfig",
           "reconstruct", "reconstruct_backward", "rbd_reconstruction",
           "load", "status_string",
           "LibraryMissing", "RBD_MAX_D"]

STOP_NAMES = {0: "error", RBD_STOP_TOL: "tol", RBD_STOP_DMAX: "dmax", RBD_STOP_BREAK: "break"}


def _torch():
    import torch
    return torch


def basis_code(basis) -> int:
    """'f64' (rbd_fit) or 'f32' (the basis stored in FP32 while the loop runs, rbd_fit_basis)."""
    codes = {"f64": _lib.RBD_BASIS_F64, "f32": _lib.RBD_BASIS_F32}
    if basis not in codes:
        raise ValueError(f"basis must be 'f64' or 'f32', not {basis!r}")
    return codes[basis]


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


@dataclass
class CsrMatrix:
    """A symmetric positive definite m x m matrix in CSR form, on the device:
    indptr (m + 1, int64), indices (nnz, int32), values (nnz, float64)."""
    indptr: "object"
    indices: "object"
    values: "object"

    @property
    def m(self) -> int:
        return int(self.indptr.numel()) - 1

    @property
    def nnz(self) -> int:
        return int(self.values.numel())

    def check(self, m: int, device) -> None:
        torch = _torch()
        ok = (self.indptr.dtype == torch.int64 and self.indices.dtype == torch.int32
              and self.values.dtype == torch.float64 and self.m == m and self.indices.numel() == self.nnz
              and all(t.device == device and t.is_contiguous() and t.dim() == 1
                      for t in (self.indptr, self.indices, self.values)))
        if not ok:
            raise ValueError("A must be CSR on X's device: indptr int64 (m + 1), indices int32, values float64")


class FitBuffers:
    """Outputs and workspace of one rbd_fit configuration, reusable across calls
    (``spd``: sized for rbd_fit_spd as well)."""

    def __init__(self, m: int, n: int, d_max: int, dtype, device, spd: bool = False, workspace: bool = True,
                 basis: str = "f64"):
        torch = _torch()
        self.m, self.n, self.d_max, self.dtype = int(m), int(n), int(d_max), dtype
        code = dtype_code(dtype)
        self.spd = bool(spd)
        self.basis = basis_code(basis)
        if spd and self.basis != _lib.RBD_BASIS_F64:
            raise ValueError("the FP32 basis is for A = I fits only")
        if not workspace:
            self.ws_bytes = 0
        elif spd:
            self.ws_bytes = _lib.fit_spd_workspace_size(self.m, self.n, self.d_max, code)
        else:
            self.ws_bytes = _lib.fit_workspace_size(self.m, self.n, self.d_max, code, self.basis)
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        self.Y = torch.empty((self.m, self.d_max), **f64)
        self.T = torch.empty((self.d_max, self.n), **f64)
        self.pivots = torch.empty(self.d_max, dtype=torch.int64, device=dev)
        self.col_err = torch.empty(self.n, **f64)
        self.err_hist = torch.empty(self.d_max + 1, **f64)
        self.ints = torch.empty(4, dtype=torch.int32, device=dev)     # d, status, stop reason
        self.workspace = (torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=dev) if workspace
                          else None)

    def result(self) -> FitResult:
        d, status, stop = (int(v) for v in self.ints[:3].tolist())
        if status == _lib.RBD_EMATRIX:
            raise ValueError(f"rbd_fit_spd: {status_string(status)}")
        if status == _lib.RBD_EDEVICE:
            raise RuntimeError(f"rbd_fit: {status_string(status)} (the persistent loop's workgroups were not all resident)")
        if status != _lib.RBD_OK:
            raise FloatingPointError(f"rbd_fit: {status_string(status)}")
        return FitResult(Y=self.Y[:, :d], T=self.T[:d], pivots=self.pivots[:d], col_err=self.col_err,
                         err_hist=self.err_hist[: d + 1], d=d, stop=STOP_NAMES.get(stop, str(stop)))


def fit_into(bufs: FitBuffers, X, tol: float = 0.0, rel: bool = False, start: int = -1, stream=None,
             weights=None, A: "CsrMatrix | None" = None) -> None:
    """Enqueue rbd_fit (rbd_fit_weighted when ``weights`` is given: A = diag(weights);
    rbd_fit_spd when a CsrMatrix ``A`` is given) on ``stream`` (default: torch's
    current stream).  None of the variants waits for the device."""
    torch = _torch()
    _check_matrix(X, "X")
    if tuple(X.shape) != (bufs.m, bufs.n) or X.dtype != bufs.dtype:
        raise ValueError("X does not match the buffers' shape/dtype")
    if weights is not None:
        if (weights.dtype != torch.float64 or weights.dim() != 1 or weights.numel() != bufs.m
                or weights.device != X.device or not weights.is_contiguous()):
            raise ValueError("weights must be a contiguous float64 vector of m values on X's device")
    lib = load()
    with torch.cuda.device(X.device):
        s = stream if stream is not None else torch.cuda.current_stream(X.device)
        ints = bufs.ints.data_ptr()
        mode = _lib.RBD_TOL_REL if rel else _lib.RBD_TOL_ABS
        outs = (bufs.Y.data_ptr(), bufs.T.data_ptr(), bufs.pivots.data_ptr(), bufs.col_err.data_ptr(),
                bufs.err_hist.data_ptr(), ints, ints + 4, ints + 8, bufs.workspace.data_ptr(),
                bufs.workspace.numel(), s.cuda_stream)
        if A is not None:
            if weights is not None:
                raise ValueError("give weights or A, not both")
            if not bufs.spd:
                raise ValueError("buffers were not sized for a sparse A (FitBuffers(..., spd=True))")
            A.check(bufs.m, X.device)
            rc = lib.rbd_fit_spd(X.data_ptr(), dtype_code(X.dtype), bufs.m, bufs.n, X.stride(0), A.indptr.data_ptr(),
                                 A.indices.data_ptr(), A.values.data_ptr(), A.nnz, float(tol), mode, bufs.d_max,
                                 int(start), *outs)
        elif weights is None:
            rc = lib.rbd_fit_basis(X.data_ptr(), dtype_code(X.dtype), bufs.m, bufs.n, X.stride(0), float(tol), mode,
                                   bufs.d_max, int(start), bufs.basis, *outs)
        else:
            if bufs.basis != _lib.RBD_BASIS_F64:
                raise ValueError("the FP32 basis is for A = I fits only")
            rc = lib.rbd_fit_weighted(X.data_ptr(), dtype_code(X.dtype), bufs.m, bufs.n, X.stride(0),
                                      weights.data_ptr(), float(tol), mode, bufs.d_max, int(start), *outs)
    _lib.check(rc, "rbd_fit")


def fit_noalloc_into(bufs: FitBuffers, X, tol: float = 0.0, rel: bool = False, start: int = -1,
                     stream=None) -> None:
    """Enqueue rbd_fit_noalloc (A = I) on ``stream``: rbd_fit with the library's fixed
    per-device scratch in place of a workspace (``bufs`` may be created with
    ``workspace=False``).  Calls that overlap on one GPU share that scratch."""
    torch = _torch()
    _check_matrix(X, "X")
    if tuple(X.shape) != (bufs.m, bufs.n) or X.dtype != bufs.dtype:
        raise ValueError("X does not match the buffers' shape/dtype")
    lib = load()
    with torch.cuda.device(X.device):
        s = stream if stream is not None else torch.cuda.current_stream(X.device)
        ints = bufs.ints.data_ptr()
        rc = lib.rbd_fit_noalloc(X.data_ptr(), dtype_code(X.dtype), bufs.m, bufs.n, X.stride(0), float(tol),
                                 _lib.RBD_TOL_REL if rel else _lib.RBD_TOL_ABS, bufs.d_max, int(start),
                                 bufs.Y.data_ptr(), bufs.T.data_ptr(), bufs.pivots.data_ptr(),
                                 bufs.col_err.data_ptr(), bufs.err_hist.data_ptr(), ints, ints + 4, ints + 8,
                                 s.cuda_stream)
    _lib.check(rc, "rbd_fit_noalloc")


class FitGraph:
    """A captured fit (rbd_fit_graph_create): all D greedy steps recorded once as a
    HIP graph; ``replay`` refits whatever X (and weights) hold, into ``bufs``, with a
    single graph launch.  X, weights and bufs must stay alive and keep their storage."""

    def __init__(self, bufs: FitBuffers, X, tol: float = 0.0, rel: bool = False, start: int = -1, weights=None):
        import ctypes
        torch = _torch()
        _check_matrix(X, "X")
        if tuple(X.shape) != (bufs.m, bufs.n) or X.dtype != bufs.dtype:
            raise ValueError("X does not match the buffers' shape/dtype")
        if bufs.basis != _lib.RBD_BASIS_F64:
            raise ValueError("the captured fit keeps the basis in FP64")
        if weights is not None and (weights.dtype != torch.float64 or weights.dim() != 1
                                    or weights.numel() != bufs.m or weights.device != X.device
                                    or not weights.is_contiguous()):
            raise ValueError("weights must be a contiguous float64 vector of m values on X's device")
        self._keep = (bufs, X, weights)
        self.bufs = bufs
        self.device = X.device
        lib = load()
        handle = ctypes.c_void_p()
        with torch.cuda.device(X.device):
            cap = torch.cuda.Stream(device=X.device)      # capture needs a created stream
            torch.cuda.current_stream(X.device).synchronize()
            ints = bufs.ints.data_ptr()
            rc = lib.rbd_fit_graph_create(
                X.data_ptr(), dtype_code(X.dtype), bufs.m, bufs.n, X.stride(0),
                weights.data_ptr() if weights is not None else None, float(tol),
                _lib.RBD_TOL_REL if rel else _lib.RBD_TOL_ABS, bufs.d_max, int(start), bufs.Y.data_ptr(),
                bufs.T.data_ptr(), bufs.pivots.data_ptr(), bufs.col_err.data_ptr(), bufs.err_hist.data_ptr(),
                ints, ints + 4, ints + 8, bufs.workspace.data_ptr(), bufs.workspace.numel(), cap.cuda_stream,
                ctypes.byref(handle))
        _lib.check(rc, "rbd_fit_graph_create")
        self._h = handle

    def replay(self, stream=None) -> None:
        """Enqueue one replay on ``stream`` (default: torch's current stream)."""
        torch = _torch()
        if self._h is None:
            raise RuntimeError("graph destroyed")
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            _lib.check(load().rbd_fit_graph_launch(self._h, s.cuda_stream), "rbd_fit_graph_launch")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            load().rbd_fit_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit(X, tol: float = 0.0, d_max: int = 64, rel: bool = False, start: int = -1, stream=None,
        weights=None, A: "CsrMatrix | None" = None, basis: str = "f64") -> FitResult:
    """Algorithm 1 on a device matrix X (m x n, f32/bf16/f16/f64 storage).

    ``tol`` is eps_R (absolute, or relative to max_j ||x_j|| when ``rel``);
    ``start < 0`` starts from the column of largest norm; ``weights`` (float64,
    m values > 0) selects the diagonal A-norm of section 3.2, ``A`` (CsrMatrix)
    a general SPD A-norm; ``basis='f32'`` keeps the basis in FP32 while the
    loop runs (rbd_fit_basis, for BF16-stored data).  Waits for the
    device and returns views of the first d basis vectors / rows of T.
    """
    torch = _torch()
    bufs = FitBuffers(X.shape[0], X.shape[1], d_max, X.dtype, X.device, spd=A is not None, basis=basis)
    fit_into(bufs, X, tol=tol, rel=rel, start=start, stream=stream, weights=weights, A=A)
    (stream or torch.cuda.current_stream(X.device)).synchronize()
    return bufs.result()


def read_stream(t, nontemporal: bool = True, stream=None) -> None:
    """Enqueue rbd_read_stream over a contiguous device tensor (a measurement tool:
    one read of every byte, the values discarded)."""
    torch = _torch()
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("read_stream needs a contiguous device tensor")
    sink = torch.empty(1, dtype=torch.int32, device=t.device)
    with torch.cuda.device(t.device):
        s = stream if stream is not None else torch.cuda.current_stream(t.device)
        rc = load().rbd_read_stream(t.data_ptr(), t.numel() * t.element_size(), int(bool(nontemporal)),
                                    sink.data_ptr(), s.cuda_stream)
    _lib.check(rc, "rbd_read_stream")


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


@dataclass
class Classification:
    index: "object"       # (k,) int64 nearest training column
    label: "object"       # (k,) int32 its label
    dist2: "object"       # (k,) float64 squared distance in the compressed coordinates
    C: "object"           # (d, k) float64 coordinates Y'V of the queries


def classify(Y, T, V, labels=None, stream=None, sync: bool = True, workspace=None) -> Classification:
    """Nearest training sample in compressed coordinates (rbd_classify): c = Y'v
    for every column v of V, then argmin_j ||c - T(:, j)||^2 (lowest index on ties).

    Y (m, d) and T (d, n) are float64 (typically a fit's basis and T); labels
    is an int32 vector of n class labels or None.  With ``sync`` False the
    call only enqueues on ``stream``; ``workspace`` may pass a reusable uint8
    buffer of at least ``_lib.classify_workspace_size`` bytes."""
    torch = _torch()
    _check_matrix(Y, "Y")
    _check_matrix(T, "T")
    _check_matrix(V, "V")
    if Y.dtype != torch.float64 or T.dtype != torch.float64:
        raise TypeError("Y and T must be float64")
    m, d = Y.shape
    if T.shape[0] != d or V.shape[0] != m:
        raise ValueError("shapes: Y (m, d), T (d, n), V (m, k)")
    n, k = T.shape[1], V.shape[1]
    dev = V.device
    if labels is not None:
        if labels.dtype != torch.int32 or labels.numel() != n or labels.device != dev or not labels.is_contiguous():
            raise ValueError("labels must be a contiguous int32 vector of n values on V's device")
    ws = _lib.classify_workspace_size(m, d, k)
    if workspace is None or workspace.numel() < ws:
        workspace = torch.empty(ws, dtype=torch.uint8, device=dev)
    C = torch.empty((d, k), dtype=torch.float64, device=dev)
    index = torch.empty(k, dtype=torch.int64, device=dev)
    label = torch.empty(k, dtype=torch.int32, device=dev)
    dist2 = torch.empty(k, dtype=torch.float64, device=dev)
    lib = load()
    with torch.cuda.device(dev):
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        rc = lib.rbd_classify(Y.data_ptr(), Y.stride(0), m, d, T.data_ptr(), T.stride(0), n,
                              labels.data_ptr() if labels is not None else None, V.data_ptr(), dtype_code(V.dtype),
                              k, V.stride(0), C.data_ptr(), index.data_ptr(), label.data_ptr(), dist2.data_ptr(),
                              workspace.data_ptr(), workspace.numel(), s.cuda_stream)
        _lib.check(rc, "rbd_classify")
        if sync:
            s.synchronize()
    return Classification(index, label, dist2, C)


# ---------------------------------------------------------------------------
# batched fits
# ---------------------------------------------------------------------------
@dataclass
class BatchConfig:
    threads: int
    wg_per_cu: int


class BatchPlan:
    """Sizes, packed device buffers and workspace of one batch of matrices.

    ``ms``/``ns`` give every matrix's shape; X_b is stored row-major with
    leading dimension n_b, back to back in batch order (``pack`` does this).
    """

    def __init__(self, ms, ns, d_max: int, dtype, device):
        import ctypes

        import numpy as np
        torch = _torch()
        self.ms = np.asarray(ms, dtype=np.int64)
        self.ns = np.asarray(ns, dtype=np.int64)
        self.batch = len(self.ms)
        self.d_max, self.dtype = int(d_max), dtype
        self.device = torch.device(device)
        desc = np.zeros((self.batch, 8), dtype=np.int64)
        order = np.zeros(self.batch, dtype=np.int32)
        sizes = _lib.BatchSizes()
        rc = load().rbd_batch_plan(self.ms.ctypes.data, self.ns.ctypes.data, self.batch, self.d_max,
                                   desc.ctypes.data, order.ctypes.data, ctypes.byref(sizes))
        _lib.check(rc, "rbd_batch_plan")
        self.desc_host, self.order_host, self.sizes = desc, order, sizes
        dev = self.device
        self.desc = torch.from_numpy(desc).to(dev)
        self.order = torch.from_numpy(order).to(dev)
        f64 = dict(dtype=torch.float64, device=dev)
        self.Y = torch.empty(sizes.y_elems, **f64)
        self.T = torch.empty(sizes.t_elems, **f64)
        self.col_err = torch.empty(sizes.c_elems, **f64)
        self.pivots = torch.empty((self.batch, self.d_max), dtype=torch.int64, device=dev)
        self.err_hist = torch.empty((self.batch, self.d_max + 1), **f64)
        self.ints = torch.empty((2, self.batch), dtype=torch.int32, device=dev)   # d, status
        self.workspace = torch.empty(max(int(sizes.workspace_bytes), 256), dtype=torch.uint8, device=dev)
        self.config = None

    def pack(self, mats):
        """Concatenate row-major matrices (device tensors of the plan's dtype) in batch order."""
        torch = _torch()
        for b, A in enumerate(mats):
            if tuple(A.shape) != (int(self.ms[b]), int(self.ns[b])) or A.dtype != self.dtype:
                raise ValueError(f"matrix {b} does not match the plan")
        return torch.cat([A.contiguous().reshape(-1) for A in mats]).to(self.device)

    def _args(self, Xp, tol, rel):
        if Xp.dim() != 1 or Xp.numel() != self.sizes.x_elems or Xp.dtype != self.dtype:
            raise ValueError("packed X does not match the plan")
        ints = self.ints.data_ptr()
        return (Xp.data_ptr(), dtype_code(self.dtype), self.desc.data_ptr(), self.order.data_ptr(), self.batch,
                float(tol), _lib.RBD_TOL_REL if rel else _lib.RBD_TOL_ABS, self.d_max)

    def _outs(self):
        ints = self.ints.data_ptr()
        return (self.Y.data_ptr(), self.T.data_ptr(), self.pivots.data_ptr(), self.col_err.data_ptr(),
                self.err_hist.data_ptr(), ints, ints + 4 * self.batch, int(self.sizes.max_m),
                self.workspace.data_ptr(), self.workspace.numel())

    def autotune(self, Xp, tol=0.0, rel=False, sample_stride=None, stream=None):
        """Pick the workgroup shape by timing every candidate on a sub-batch (waits for the device).

        The default stride keeps at least 4 matrices per workgroup at the largest
        candidate grid (8 workgroups per compute unit), so that the trials time
        throughput, not the latency of the largest matrix."""
        import ctypes
        torch = _torch()
        if sample_stride is None:
            cus = torch.cuda.get_device_properties(self.device).multi_processor_count
            sample_stride = max(1, self.batch // (4 * 8 * cus))
        best = _lib.BatchConfig()
        times = (ctypes.c_double * 16)()
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            rc = load().rbd_batched_autotune(*self._args(Xp, tol, rel), int(sample_stride), *self._outs(),
                                             s.cuda_stream, ctypes.byref(best), ctypes.cast(times, ctypes.c_void_p))
        _lib.check(rc, "rbd_batched_autotune")
        self.config = BatchConfig(best.threads, best.wg_per_cu)
        self.trials = {(t, w): times[i * 4 + k] for i, t in enumerate((128, 256, 512, 1024))
                       for k, w in enumerate((1, 2, 4, 8))}
        return self.config

    def run(self, Xp, tol=0.0, rel=False, config=None, stream=None):
        """Enqueue the batched fit (no wait)."""
        torch = _torch()
        cfg = config or self.config or BatchConfig(256, 2)
        c = _lib.BatchConfig(int(cfg.threads), int(cfg.wg_per_cu))
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            a = self._args(Xp, tol, rel)
            rc = load().rbd_fit_batched(*a, c, *self._outs(), s.cuda_stream)
        _lib.check(rc, "rbd_fit_batched")

    def results(self):
        """Per-matrix FitResult views (waits for the device)."""
        torch = _torch()
        torch.cuda.current_stream(self.device).synchronize()
        ds, sts = (v.tolist() for v in self.ints.cpu())
        out = []
        for b in range(self.batch):
            if sts[b] != _lib.RBD_OK:
                out.append(None)
                continue
            dsc = self.desc_host[b]
            m, n, d = int(dsc[0]), int(dsc[1]), int(ds[b])
            Y = self.Y[dsc[3]: dsc[3] + m * self.d_max].view(m, self.d_max)[:, :d]
            T = self.T[dsc[4]: dsc[4] + self.d_max * n].view(self.d_max, n)[:d]
            out.append(FitResult(Y=Y, T=T, pivots=self.pivots[b, :d], col_err=self.col_err[dsc[5]: dsc[5] + n],
                                 err_hist=self.err_hist[b, : d + 1], d=d, stop=""))
        return out


def fit_batched(mats, tol: float = 0.0, d_max: int = 64, rel: bool = False, config=None, autotune: bool = False):
    """Fit every matrix in ``mats`` (device tensors, one dtype) in one persistent launch.

    Returns (list of FitResult or None for matrices with non-finite data, BatchPlan)."""
    plan = BatchPlan([A.shape[0] for A in mats], [A.shape[1] for A in mats], d_max, mats[0].dtype, mats[0].device)
    Xp = plan.pack(mats)
    if autotune and config is None:
        plan.autotune(Xp, tol=tol, rel=rel)
    plan.run(Xp, tol=tol, rel=rel, config=config)
    return plan.results(), plan


# ---------------------------------------------------------------------------
# reconstruction and its backward (pivots fixed)
# ---------------------------------------------------------------------------
def reconstruct(Y, T, stream=None):
    """Uncompress: Z = Y T (FP64), section 3.1."""
    torch = _torch()
    _check_matrix(Y, "Y")
    _check_matrix(T, "T")
    m, d = Y.shape
    n = T.shape[1]
    if T.shape[0] != d or Y.dtype != torch.float64 or T.dtype != torch.float64:
        raise ValueError("Y (m x d) and T (d x n) must be float64")
    Z = torch.empty((m, n), dtype=torch.float64, device=Y.device)
    with torch.cuda.device(Y.device):
        s = stream if stream is not None else torch.cuda.current_stream(Y.device)
        rc = load().rbd_reconstruct(Y.data_ptr(), Y.stride(0), m, d, T.data_ptr(), T.stride(0), n, Z.data_ptr(),
                                    Z.stride(0), s.cuda_stream)
    _lib.check(rc, "rbd_reconstruct")
    return Z


def reconstruct_backward(X, G, Y, T, pivots, stream=None):
    """dL/dX (FP64) for L = <G, Y Y' X> with the pivots held fixed."""
    import ctypes
    torch = _torch()
    for A, nm in ((X, "X"), (G, "G"), (Y, "Y"), (T, "T")):
        _check_matrix(A, nm)
    m, n = X.shape
    d = Y.shape[1]
    if G.shape != X.shape or Y.shape[0] != m or T.shape != (d, n) or pivots.numel() != d:
        raise ValueError("shape mismatch")
    if G.dtype not in (torch.float64, torch.float32):
        raise TypeError("G must be float64 or float32")
    piv = pivots.to(torch.int64).contiguous()
    ws = ctypes.c_size_t(0)
    _lib.check(load().rbd_reconstruct_backward_workspace_size(m, n, d, ctypes.byref(ws)),
               "rbd_reconstruct_backward_workspace_size")
    dX = torch.empty((m, n), dtype=torch.float64, device=X.device)
    work = torch.empty(max(ws.value, 256), dtype=torch.uint8, device=X.device)
    with torch.cuda.device(X.device):
        s = stream if stream is not None else torch.cuda.current_stream(X.device)
        rc = load().rbd_reconstruct_backward(X.data_ptr(), dtype_code(X.dtype), X.stride(0), G.data_ptr(),
                                             dtype_code(G.dtype), G.stride(0), Y.data_ptr(), Y.stride(0),
                                             T.data_ptr(), T.stride(0), piv.data_ptr(), m, n, d, dX.data_ptr(),
                                             dX.stride(0), work.data_ptr(), work.numel(), s.cuda_stream)
    _lib.check(rc, "rbd_reconstruct_backward")
    return dX


def _autograd_function():
    torch = _torch()

    class RBDReconstruct(torch.autograd.Function):
        """Z = Y Y' X where (Y, T) = RBD(X): the forward runs the greedy fit and the
        reconstruction; the backward differentiates with the pivots held fixed."""

        @staticmethod
        def forward(ctx, X, tol, d_max, rel):
            res = fit(X.detach(), tol=tol, d_max=d_max, rel=rel)
            ctx.save_for_backward(X.detach(), res.Y, res.T, res.pivots)
            return reconstruct(res.Y, res.T)

        @staticmethod
        def backward(ctx, G):
            X, Y, T, piv = ctx.saved_tensors
            dX = reconstruct_backward(X, G.contiguous(), Y, T, piv)
            return dX.to(X.dtype), None, None, None

    return RBDReconstruct


_RBDReconstruct = None


def rbd_reconstruction(X, tol: float = 0.0, d_max: int = 64, rel: bool = False):
    """Differentiable Z = Y Y' X (torch.autograd); gradients hold the pivots fixed."""
    global _RBDReconstruct
    if _RBDReconstruct is None:
        _RBDReconstruct = _autograd_function()
    return _RBDReconstruct.apply(X, tol, d_max, rel)
