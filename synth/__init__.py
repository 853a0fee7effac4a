"""Seeded synthetic inputs for the reduced-basis-decomposition hot path.

This module is shared by the FP64 oracle (``oracle/``), the tests and the
benchmark.  It holds input generators and storage-precision rounding only:
none of the decomposition's own arithmetic (no Gram-Schmidt, no projection,
no error evaluation, no pivot search) lives here.

Every generator draws from ``numpy.random.default_rng(SeedSequence([cfg,
seed, stream]))`` with a fixed stream id per quantity, so a workload is a
pure function of ``(cfg, seed)``:

    stream 0  left orthonormal factor U     stream 4  decay rates mu
    stream 1  right orthonormal factor V    stream 5  fixed centres c_k
    stream 2  additive noise                stream 6  cotangent G
    stream 3  bump parameters               stream 7  batch sizes

Workloads (the data model is X in R^{m x n}, columns are the samples, as in
eq. (1) of the paper):

* ``lowrank_spectrum``   -- X = U diag(sigma) V^T + noise, sigma_i = 10^(-i/4)
  for i < 32 (512 x 256, the small parity case).
* ``bump_field``         -- a sum of 50 random 2-D Gaussian bumps sampled on a
  grid; column j is the slice at s2 = j/(n-1) (image-like stand-in for the
  paper's 512 x 512 test images, whose pixels are not available).
* ``parametric_field``   -- x(s; mu) = sum_{k<8} exp(-mu_k |s - c_k|^2) on a
  g x g grid, one column per parameter draw (the parametric-snapshot workload
  that motivates the method in section 2 of the paper).
* ``table3``             -- the three separable functions of Table 3.
* ``approx_field``       -- f = 0.6 f1 + 0.1 f2 + 0.01 f3 of section 4.2.2.
* ``batched_spectra``    -- many small matrices with a 10^(-i/8) spectrum.

Storage rounding (``quantize``) defines the exact values a reduced-precision
X holds: FP64 -> FP32 round-to-nearest-even, then (for BF16) FP32 -> BF16
round-to-nearest-even on the bit pattern, or FP64 -> FP16 round-to-nearest-
even.  Both the oracle and the device path consume these stored values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# seeding
# ----------------------------------------------------------------------------

S_U, S_V, S_NOISE, S_BUMPS, S_MU, S_CENTRES, S_G, S_SIZES = range(8)


def rng(cfg: int, seed: int, stream: int) -> np.random.Generator:
    """Counter-free, platform-independent generator for one (cfg, seed, stream)."""
    return np.random.default_rng(np.random.SeedSequence([int(cfg), int(seed), int(stream)]))


def haar(g: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Random matrix with orthonormal columns (QR of a Gaussian, diag(R) > 0)."""
    a = g.standard_normal((rows, cols))
    q, r = np.linalg.qr(a)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


@dataclass
class Workload:
    """An input matrix plus the fit settings it is quoted with."""

    name: str
    X: np.ndarray                 # FP64 values before storage rounding
    tol: float
    rel: bool                     # tau = tol * max_j ||x_j|| when True
    d_max: int
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# storage precision
# ----------------------------------------------------------------------------

DTYPES = ("f64", "f32", "bf16", "f16")


def bf16_bits_from_f32(a32: np.ndarray) -> np.ndarray:
    """Round FP32 values to BF16 (nearest, ties to even); returns uint16 bit patterns."""
    u = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return r.astype(np.uint16)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    u = bits.astype(np.uint32) << np.uint32(16)
    return u.view(np.float32).astype(np.float64)


def quantize(X: np.ndarray, dtype: str):
    """Round X to a storage dtype.

    Returns ``(stored, values)``: ``stored`` is the array in its storage form
    (float64 / float32 / uint16 BF16 bit patterns / float16), ``values`` the
    exact stored values as FP64 (what every consumer must treat as the data).
    """
    X = np.asarray(X, dtype=np.float64)
    if dtype == "f64":
        s = np.ascontiguousarray(X)
        return s, s
    if dtype == "f32":
        s = np.ascontiguousarray(X.astype(np.float32))
        return s, s.astype(np.float64)
    if dtype == "bf16":
        s = bf16_bits_from_f32(X.astype(np.float32))
        return s, bf16_bits_to_f64(s)
    if dtype == "f16":
        s = np.ascontiguousarray(X.astype(np.float16))
        return s, s.astype(np.float64)
    raise ValueError(f"unknown storage dtype {dtype!r}")


# ----------------------------------------------------------------------------
# 1. low-rank spectrum (512 x 256, rank 32 + 1e-10 noise)
# ----------------------------------------------------------------------------

def lowrank_spectrum(seed: int = 0, m: int = 512, n: int = 256, r: int = 32,
                     decade: float = 4.0, noise: float = 1e-10) -> Workload:
    """X = U diag(10^(-i/decade)) V^T + noise * N(0,1); noise is a standard deviation."""
    U = haar(rng(1, seed, S_U), m, r)
    V = haar(rng(1, seed, S_V), n, r)
    sig = 10.0 ** (-np.arange(r) / decade)
    X = (U * sig[None, :]) @ V.T
    if noise:
        X = X + noise * rng(1, seed, S_NOISE).standard_normal((m, n))
    return Workload("lowrank_spectrum", X, tol=1e-8, rel=False, d_max=64,
                    meta=dict(m=m, n=n, rank=r, sigma=sig))


def random_rank(seed: int, m: int, n: int, r: int) -> np.ndarray:
    """Random exactly-rank-r matrix (Gaussian factors, no noise)."""
    g = rng(90, seed, S_U)
    return g.standard_normal((m, r)) @ g.standard_normal((r, n))


# ----------------------------------------------------------------------------
# 2. bump field (image-like, 2048 x 2048)
# ----------------------------------------------------------------------------

def bump_params(seed: int, count: int = 50, cfg: int = 2):
    g = rng(cfg, seed, S_BUMPS)
    centres = g.uniform(0.0, 1.0, size=(count, 2))
    widths = g.uniform(0.02, 0.2, size=count)
    amps = g.standard_normal(count)
    return centres, widths, amps


def bump_field(seed: int = 0, m: int = 2048, n: int = 2048, noise: float = 1e-4,
               cfg: int = 2, tol: float = 1e-4, d_max: int = 256) -> Workload:
    """F(s1, s2) = sum_b a_b exp(-|s - c_b|^2 / (2 w_b^2)) + noise, s1 = i/(m-1), s2 = j/(n-1).

    Each bump is separable, so X is accumulated as rank-1 terms in a fixed
    order (elementwise IEEE arithmetic: identical on every host).
    """
    centres, widths, amps = bump_params(seed, cfg=cfg)
    s1 = np.arange(m, dtype=np.float64) / max(m - 1, 1)
    s2 = np.arange(n, dtype=np.float64) / max(n - 1, 1)
    X = np.zeros((m, n))
    for (c1, c2), w, a in zip(centres, widths, amps):
        g1 = np.exp(-((s1 - c1) ** 2) / (2.0 * w * w))
        g2 = np.exp(-((s2 - c2) ** 2) / (2.0 * w * w))
        X += (a * g1)[:, None] * g2[None, :]
    if noise:
        X += noise * rng(cfg, seed, S_NOISE).standard_normal((m, n))
    return Workload("bump_field", X, tol=tol, rel=True, d_max=d_max,
                    meta=dict(m=m, n=n, bumps=len(amps)))


def bump_fill(seed: int, out, noise: float = 1e-4, cfg: int = 2, rows_per_chunk: int = 8192) -> None:
    """Write the stored values of ``bump_field(seed, m, n, noise)`` into a torch tensor
    ``out`` (m x n, float64/float32/bfloat16, any device).

    The same FP64 products and sums in the same order as ``bump_field`` (so the
    values are bit-identical to the host's), then one rounding to the storage
    type; the noise is drawn on the host from the same stream.  This is input
    generation, not part of the decomposition.
    """
    import torch

    m, n = out.shape
    centres, widths, amps = bump_params(seed, cfg=cfg)
    s1 = np.arange(m, dtype=np.float64) / max(m - 1, 1)
    s2 = np.arange(n, dtype=np.float64) / max(n - 1, 1)
    ag1 = np.stack([a * np.exp(-((s1 - c1) ** 2) / (2.0 * w * w)) for (c1, _), w, a in zip(centres, widths, amps)])
    g2 = np.stack([np.exp(-((s2 - c2) ** 2) / (2.0 * w * w)) for (_, c2), w in zip(centres, widths)])
    dev = out.device
    A = torch.from_numpy(ag1).to(dev)
    B = torch.from_numpy(g2).to(dev)
    g = rng(cfg, seed, S_NOISE) if noise else None
    for r0 in range(0, m, rows_per_chunk):
        r1 = min(m, r0 + rows_per_chunk)
        acc = torch.zeros((r1 - r0, n), dtype=torch.float64, device=dev)
        for b in range(A.shape[0]):
            acc += A[b, r0:r1, None] * B[b, None, :]
        if g is not None:
            acc += noise * torch.from_numpy(g.standard_normal((r1 - r0, n))).to(dev)
        if out.dtype == torch.float64:
            out[r0:r1] = acc
        elif out.dtype == torch.float32:
            out[r0:r1] = acc.to(torch.float32)
        else:
            out[r0:r1] = acc.to(torch.float32).to(out.dtype)
        del acc


# ----------------------------------------------------------------------------
# 3. parametric field (1,048,576 x 4096 at full size)
# ----------------------------------------------------------------------------

@dataclass
class ParametricField:
    """x_j(s) = sum_{k<8} exp(-mu_{j,k} |s - c_k|^2), s = (a/(g-1), b/(g-1)), row = g*a + b."""

    mu: np.ndarray        # (n, K) decay rates, U[1, 100]
    centres: np.ndarray   # (K, 2) fixed centres, U[0.1, 0.9]^2
    grid: int             # g: the grid is g x g, m = g*g

    @property
    def m(self) -> int:
        return self.grid * self.grid

    @property
    def n(self) -> int:
        return self.mu.shape[0]

    def factors(self, cols=None):
        """Separable factors A[k, a, j] = exp(-mu_jk (a/(g-1) - c_k1)^2), B likewise with c_k2."""
        mu = self.mu if cols is None else self.mu[cols]
        s = np.arange(self.grid, dtype=np.float64) / (self.grid - 1)
        K = mu.shape[1]
        A = np.empty((K, self.grid, mu.shape[0]))
        B = np.empty((K, self.grid, mu.shape[0]))
        for k in range(K):
            A[k] = np.exp(-mu[None, :, k] * ((s[:, None] - self.centres[k, 0]) ** 2))
            B[k] = np.exp(-mu[None, :, k] * ((s[:, None] - self.centres[k, 1]) ** 2))
        return A, B

    def rows(self, idx, A=None, B=None) -> np.ndarray:
        """FP64 values of the given rows (all columns), same operation order as ``fill_device``."""
        idx = np.asarray(idx, dtype=np.int64)
        if A is None:
            A, B = self.factors()
        a, b = idx // self.grid, idx % self.grid
        out = A[0][a] * B[0][b]
        for k in range(1, A.shape[0]):
            out = out + A[k][a] * B[k][b]
        return out

    def columns(self, cols) -> np.ndarray:
        """FP64 values of the given columns (all rows), same operation order as ``rows``."""
        cols = np.asarray(cols, dtype=np.int64)
        A, B = self.factors(cols=cols)
        idx = np.arange(self.m)
        a, b = idx // self.grid, idx % self.grid
        out = A[0][a] * B[0][b]
        for k in range(1, A.shape[0]):
            out = out + A[k][a] * B[k][b]
        return out

    def full(self) -> np.ndarray:
        A, B = self.factors()
        return self.rows(np.arange(self.m), A, B)

    def fill_device(self, out, rows_per_chunk: int = 16 * 1024):
        """Write the stored values into a device tensor ``out`` (m x n, f32/bf16/f16/f64).

        Elementwise FP64 multiplies and adds in the same order as ``rows`` (so the
        values are bit-identical to the host's), then one rounding to FP32 and,
        for BF16/F16, a second rounding from FP32 as torch defines it.  This is
        input generation, not part of the decomposition.
        """
        import torch

        dev = out.device
        A, B = self.factors()
        At = torch.from_numpy(A).to(dev)
        Bt = torch.from_numpy(B).to(dev)
        g = self.grid
        per = max(1, rows_per_chunk // g)
        for a0 in range(0, g, per):
            a1 = min(g, a0 + per)
            acc = At[0, a0:a1, None, :] * Bt[0, None, :, :]
            for k in range(1, At.shape[0]):
                acc = acc + At[k, a0:a1, None, :] * Bt[k, None, :, :]
            acc = acc.reshape((a1 - a0) * g, -1)
            if out.dtype == torch.float64:
                out[a0 * g:a1 * g] = acc
            elif out.dtype == torch.float32:
                out[a0 * g:a1 * g] = acc.to(torch.float32)
            else:
                out[a0 * g:a1 * g] = acc.to(torch.float32).to(out.dtype)
            del acc
        del At, Bt


def parametric_field(seed: int = 0, grid: int = 1024, n: int = 4096, K: int = 8) -> ParametricField:
    mu = rng(3, seed, S_MU).uniform(1.0, 100.0, size=(n, K))
    centres = rng(3, 0, S_CENTRES).uniform(0.1, 0.9, size=(K, 2))   # fixed across seeds
    return ParametricField(mu=mu, centres=centres, grid=grid)


# ----------------------------------------------------------------------------
# Table 3 and section 4.2.2 functions (uniform grid on [-1, 1]^2)
# ----------------------------------------------------------------------------

def grid_11(n: int) -> np.ndarray:
    return -1.0 + 2.0 * np.arange(n, dtype=np.float64) / (n - 1)


def table3(which: int, n: int = 512) -> np.ndarray:
    """The separable functions of Table 3; rows follow x, columns follow y."""
    x = grid_11(n)[:, None]
    y = grid_11(n)[None, :]
    f = np.sin(np.pi * x) * np.cos(np.pi * y)
    if which >= 2:
        f = f + 0.1 * np.sin(10 * np.pi * x) * np.cos(10 * np.pi * y)
    if which >= 3:
        f = f + 0.01 * np.sin(100 * np.pi * x) * np.cos(100 * np.pi * y)
    return f


def approx_field(n: int = 5001) -> np.ndarray:
    """f = 0.6 f1 + 0.1 f2 + 0.01 f3 on an n x n grid over [-1, 1]^2 (section 4.2.2)."""
    x = grid_11(n)[:, None]
    y = grid_11(n)[None, :]
    f1 = np.sin(np.pi * (x + 2 * y)) * np.cos(np.pi * (2 * x - y))
    f2 = np.sin(10 * np.pi * (x - 3 * y)) * np.cos(10 * np.pi * (3 * x + y))
    f3 = np.sin(3 * np.pi * x * x * y) * np.cos(6 * np.pi * np.sqrt(np.abs(x)) / (y + 2))
    return 0.6 * f1 + 0.1 * f2 + 0.01 * f3


# ----------------------------------------------------------------------------
# batched small matrices (4096 matrices, m, n log-uniform in [64, 1024])
# ----------------------------------------------------------------------------

def batched_sizes(seed: int = 0, count: int = 4096, lo: int = 64, hi: int = 1024):
    g = rng(4, seed, S_SIZES)
    m = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    n = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    return m, n


def batched_matrix(seed: int, index: int, m: int, n: int, decade: float = 8.0) -> np.ndarray:
    """X_b = U diag(10^(-i/decade)) V^T with orthonormal U, V of rank min(m, n, 17 decade).

    Singular values beyond i = 17 decade are below 1e-17 of the largest, under
    the resolution of FP64 (and far under FP32) storage, so they are omitted.
    """
    r = min(m, n, int(17 * decade))
    U = haar(rng(4, seed * 1_000_003 + index, S_U), m, r)
    V = haar(rng(4, seed * 1_000_003 + index, S_V), n, r)
    sig = 10.0 ** (-np.arange(r) / decade)
    return (U * sig[None, :]) @ V.T


# ----------------------------------------------------------------------------
# differentiation workload (bump field at 65536 x 2048 plus a cotangent)
# ----------------------------------------------------------------------------

def cotangent(seed: int, m: int, n: int) -> np.ndarray:
    return rng(5, seed, S_G).standard_normal((m, n))


# ----------------------------------------------------------------------------
# diagonal A-norm weights (section 3.2, "general diagonal matrix")
# ----------------------------------------------------------------------------

def band_weights(m: int, start: float = 0.25, stop: float = 0.5, hi: float = 100.0, lo: float = 1.0) -> np.ndarray:
    """Rows start*m .. stop*m (a band of the spatial grid) weighted hi, the rest lo."""
    w = np.full(m, float(lo))
    w[int(start * m):int(stop * m)] = float(hi)
    return w


def random_weights(seed: int, m: int, lo: float = 0.1, hi: float = 10.0) -> np.ndarray:
    """Log-uniform weights in [lo, hi]."""
    g = rng(6, seed, S_G)
    return np.exp(g.uniform(math.log(lo), math.log(hi), size=m))


def disc_weights(grid: int, centre=(0.5, 0.5), radius: float = 0.25, hi: float = 100.0) -> np.ndarray:
    """Rows of a grid x grid field (row = grid*a + b) inside a disc weighted hi, the rest 1."""
    s = np.arange(grid, dtype=np.float64) / max(grid - 1, 1)
    inside = ((s[:, None] - centre[0]) ** 2 + (s[None, :] - centre[1]) ** 2) <= radius * radius
    return np.where(inside, float(hi), 1.0).reshape(-1)


# ----------------------------------------------------------------------------
# recognition workload: synthetic classes of smooth "views" on an image grid
# (stands in for a face data set: 20 subjects, 19-48 views each, 112 x 92)
# ----------------------------------------------------------------------------

@dataclass
class ViewClasses:
    """Class c's views are template_c + sum_i a_i mode_{c,i} + noise on a
    rows x cols grid (flattened row-major).  Templates and modes are sums of
    Gaussian bumps; a_i ~ N(0, pose), noise ~ N(0, noise)."""
    templates: np.ndarray     # (classes, m)
    modes: np.ndarray         # (classes, nmodes, m)
    counts: np.ndarray        # views per class
    pose: float
    noise: float
    seed: int

    @property
    def m(self) -> int:
        return self.templates.shape[1]

    def views(self, c: int, count: int, stream: int) -> np.ndarray:
        g = rng(7, self.seed * 1009 + c, stream)
        a = self.pose * g.standard_normal((count, self.modes.shape[1]))
        V = self.templates[c][None, :] + a @ self.modes[c]
        V = V + self.noise * g.standard_normal(V.shape)
        return V.T.copy()     # (m, count)

    def split(self, train_per_class: int = 10):
        """Each class's views; the first train_per_class of a seeded shuffle
        are training samples, the rest test samples.  Returns
        (Xtrain, ytrain, Xtest, ytest), samples as columns."""
        tr, ytr, te, yte = [], [], [], []
        for c, cnt in enumerate(self.counts):
            V = self.views(c, int(cnt), S_NOISE)
            order = rng(7, self.seed * 1009 + c, S_SIZES).permutation(int(cnt))
            tr.append(V[:, order[:train_per_class]])
            te.append(V[:, order[train_per_class:]])
            ytr += [c] * train_per_class
            yte += [c] * (int(cnt) - train_per_class)
        return (np.concatenate(tr, axis=1), np.array(ytr, dtype=np.int32),
                np.concatenate(te, axis=1), np.array(yte, dtype=np.int32))

    def fill_queries(self, out, labels, coeff_seed: int = 0):
        """Device generation of many query views: out[:, q] = a view of class
        labels[q] (torch tensors on one device; out is (m, k), any float dtype)."""
        import torch
        dev = out.device
        Tm = torch.from_numpy(self.templates).to(dev)
        Md = torch.from_numpy(self.modes).to(dev)
        gen = torch.Generator(device=dev)
        gen.manual_seed(int(coeff_seed))
        k = out.shape[1]
        step = 4096
        for q0 in range(0, k, step):
            lab = labels[q0:q0 + step].long()
            a = self.pose * torch.randn((lab.numel(), Md.shape[1]), generator=gen, device=dev,
                                        dtype=torch.float64)
            V = Tm[lab] + torch.bmm(a[:, None, :].contiguous(), Md[lab].contiguous())[:, 0, :]
            V += self.noise * torch.randn(V.shape, generator=gen, device=dev, dtype=torch.float64)
            out[:, q0:q0 + lab.numel()] = V.T.to(out.dtype)


def view_classes(seed: int = 0, classes: int = 20, rows: int = 112, cols: int = 92, lo: int = 19, hi: int = 48,
                 nmodes: int = 3, bumps: int = 12, pose: float = 0.3, noise: float = 0.02) -> ViewClasses:
    g = rng(7, seed, S_BUMPS)
    s1 = np.arange(rows, dtype=np.float64) / max(rows - 1, 1)
    s2 = np.arange(cols, dtype=np.float64) / max(cols - 1, 1)

    def field():
        F = np.zeros((rows, cols))
        c1 = g.uniform(0.1, 0.9, bumps)
        c2 = g.uniform(0.1, 0.9, bumps)
        w = g.uniform(0.05, 0.25, bumps)
        a = g.standard_normal(bumps)
        for i in range(bumps):
            F += a[i] * np.exp(-((s1[:, None] - c1[i]) ** 2 + (s2[None, :] - c2[i]) ** 2) / (2.0 * w[i] ** 2))
        return F.reshape(-1)

    templates = np.stack([field() for _ in range(classes)])
    modes = np.stack([np.stack([field() for _ in range(nmodes)]) for _ in range(classes)])
    counts = g.integers(lo, hi + 1, size=classes)
    return ViewClasses(templates, modes, counts, pose, noise, seed)


def grid_laplacian_spd(rows: int, cols: int, c: float = 1.0):
    """A = I + c L, L the 5-point graph Laplacian of a rows x cols grid
    (row-major numbering): symmetric positive definite, an energy-type norm
    for fields on the grid.  Returned as CSR arrays (indptr int64, indices
    int32, data float64), sorted column indices per row."""
    m = rows * cols
    idx = np.arange(m).reshape(rows, cols)
    deg = np.zeros((rows, cols))
    pairs = []
    if rows > 1:
        pairs.append((idx[:-1, :].ravel(), idx[1:, :].ravel()))
        deg[:-1, :] += 1
        deg[1:, :] += 1
    if cols > 1:
        pairs.append((idx[:, :-1].ravel(), idx[:, 1:].ravel()))
        deg[:, :-1] += 1
        deg[:, 1:] += 1
    r = [np.arange(m)]
    cidx = [np.arange(m)]
    v = [1.0 + c * deg.ravel()]
    for a, b in pairs:
        r += [a, b]
        cidx += [b, a]
        v += [np.full(a.size, -c), np.full(a.size, -c)]
    r = np.concatenate(r)
    cidx = np.concatenate(cidx)
    v = np.concatenate(v)
    order = np.lexsort((cidx, r))
    r, cidx, v = r[order], cidx[order], v[order]
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(indptr, r + 1, 1)
    indptr = np.cumsum(indptr)
    return indptr, cidx.astype(np.int32), v.astype(np.float64)
