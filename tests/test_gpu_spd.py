"""Parity of rbd_fit_spd (a general SPD A-norm in CSR form, section 3.2 and
eq. (3)) with the FP64 oracle, which evaluates sqrt(r'Ar) on the explicit
residual with scipy.sparse.  Every case prints its name and sizes before
touching the GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from parity import compare_fit
from test_gpu_fit import to_device

pytestmark = pytest.mark.gpu


def _norms_A(R, A):
    return np.sqrt(np.maximum(np.einsum("ij,ij->j", R, np.asarray(A @ R)), 0.0))


def device_csr(indptr, indices, values):
    import torch
    import paper_1503_05947_amd as rbd
    dev = "cuda:0"
    return rbd.CsrMatrix(torch.from_numpy(np.ascontiguousarray(indptr, dtype=np.int64)).to(dev),
                         torch.from_numpy(np.ascontiguousarray(indices, dtype=np.int32)).to(dev),
                         torch.from_numpy(np.ascontiguousarray(values, dtype=np.float64)).to(dev))


def run(stored, dtype, csr, tol, d_max, rel=False, start=-1, pad_cols=0):
    import paper_1503_05947_amd as rbd
    X = to_device(stored, dtype, pad_cols)
    res = rbd.fit(X, tol=tol, d_max=d_max, rel=rel, start=start, A=device_csr(*csr))
    return dict(Y=res.Y.cpu().numpy(), T=res.T.cpu().numpy(), pivots=res.pivots.cpu().numpy(),
                col_err=res.col_err.cpu().numpy(), err_hist=res.err_hist.cpu().numpy(), d=res.d, stop=res.stop)


def check(name, stored, vals, dtype, csr, tol, d_max, rel=False, start=-1, pad_cols=0, gap=1e-8):
    m = vals.shape[0]
    print(f"[gpu] spd {name} dtype={dtype} shape={vals.shape} nnz={len(csr[2])} tol={tol} d_max={d_max}",
          flush=True)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(m, m))
    dev = run(stored, dtype, csr, tol, d_max, rel=rel, start=start, pad_cols=pad_cols)
    ref = oracle.rbd_fit(vals, tol, d_max, rel=rel, start=start, A=A)
    msgs = compare_fit(dev, ref, vals, gap=gap, weights=None, norms=lambda R: _norms_A(R, A))
    assert msgs == [], f"{name}: " + "; ".join(msgs)
    return dev, ref


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_lowrank_laplacian_norm(dtype):
    """512 rows as a 32 x 16 grid, A = I + L; the errors fall to 1e-8, so
    exact refreshes (in residual chunks) run."""
    wl = synth.lowrank_spectrum(0)
    stored, vals = synth.quantize(wl.X, dtype)
    csr = synth.grid_laplacian_spd(32, 16, 1.0)
    dev, ref = check("lowrank", stored, vals, dtype, csr, wl.tol, wl.d_max)
    if dtype == "f64":
        assert dev["d"] == ref.d and np.array_equal(dev["pivots"], ref.pivots)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_bump_field_chain_laplacian(dtype):
    """The 2048-point grid of the bump field with a chain Laplacian, relative tol 1e-4."""
    wl = synth.bump_field(0)
    stored, vals = synth.quantize(wl.X, dtype)
    check("bump", stored, vals, dtype, synth.grid_laplacian_spd(2048, 1, 50.0), wl.tol, wl.d_max, rel=True)


def test_random_sparse_spd_ragged():
    g = synth.rng(97, 0, 0)
    m, n = 1000, 777
    nz = 6 * m
    r = g.integers(0, m, nz)
    c = g.integers(0, m, nz)
    v = g.standard_normal(nz) * 0.1
    B = sp.coo_matrix((v, (r, c)), shape=(m, m)).tocsr()
    A = (B + B.T).tocsr()
    A = (A + sp.diags(np.abs(A).sum(axis=1).A1 + 0.5)).tocsr()      # diagonally dominant: SPD
    A.sort_indices()
    X = synth.random_rank(5, m, n, 60)
    stored, vals = synth.quantize(X, "f32")
    check("random", stored, vals, "f32", (A.indptr, A.indices, A.data), 0.0, 50, pad_cols=3)


def test_diagonal_csr_matches_the_weighted_path():
    import torch
    import paper_1503_05947_amd as rbd
    wl = synth.lowrank_spectrum(1)
    stored, vals = synth.quantize(wl.X, "f32")
    w = synth.random_weights(1, vals.shape[0])
    m = vals.shape[0]
    print("[gpu] spd diagonal vs weighted", flush=True)
    a = run(stored, "f32", (np.arange(m + 1), np.arange(m), w), wl.tol, wl.d_max)
    X = to_device(stored, "f32")
    b = rbd.fit(X, tol=wl.tol, d_max=wl.d_max, weights=torch.from_numpy(w).to("cuda:0"))
    assert a["d"] == b.d and np.array_equal(a["pivots"], b.pivots.cpu().numpy())
    E0 = a["err_hist"][0]
    assert np.max(np.abs(a["err_hist"] - b.err_hist.cpu().numpy())) < 1e-9 * E0


def test_identity_csr_matches_the_plain_fit():
    import paper_1503_05947_amd as rbd
    wl = synth.lowrank_spectrum(2)
    stored, vals = synth.quantize(wl.X, "f32")
    m = vals.shape[0]
    print("[gpu] spd identity vs plain", flush=True)
    a = run(stored, "f32", (np.arange(m + 1), np.arange(m), np.ones(m)), wl.tol, wl.d_max)
    b = rbd.fit(to_device(stored, "f32"), tol=wl.tol, d_max=wl.d_max)
    assert a["d"] == b.d and np.array_equal(a["pivots"], b.pivots.cpu().numpy())
    assert np.max(np.abs(a["err_hist"] - b.err_hist.cpu().numpy())) < 1e-9 * a["err_hist"][0]


def test_index_out_of_range_is_reported():
    import paper_1503_05947_amd as rbd
    print("[gpu] spd bad index", flush=True)
    m = 64
    indptr = np.arange(m + 1)
    indices = np.arange(m)
    indices[10] = m + 5                     # outside the matrix: skipped by the kernels, reported
    X = to_device(np.ones((m, 8), dtype=np.float32), "f32")
    with pytest.raises(ValueError):
        rbd.fit(X, tol=0.0, d_max=4, A=device_csr(indptr, indices, np.ones(m)))


def test_decreasing_indptr_is_reported():
    import paper_1503_05947_amd as rbd
    print("[gpu] spd decreasing indptr", flush=True)
    m = 64
    indptr = np.arange(m + 1)
    indptr[20] = 25                          # row 19 ends after row 20 ends: not a CSR layout
    X = to_device(np.ones((m, 8), dtype=np.float32), "f32")
    with pytest.raises(ValueError):
        rbd.fit(X, tol=0.0, d_max=4, A=device_csr(indptr, np.arange(m), np.ones(m)))
