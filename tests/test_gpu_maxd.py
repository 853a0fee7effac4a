"""Fits at the largest basis size the library accepts (RBD_MAX_D = 1024), so the
Gram-Schmidt passes run with their widest register tiles (16 chunks of 64
columns of Y) and the staging of basis columns cycles through 128 blocks.
A = I, a diagonal A and a sparse SPD A, each against the FP64 oracle.  Every
case prints its name before touching the GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from parity import compare_fit
from test_gpu_fit import to_device

pytestmark = pytest.mark.gpu

M, N, D = 1100, 1030, 1024


def _host(res):
    return dict(Y=res.Y.cpu().numpy(), T=res.T.cpu().numpy(), pivots=res.pivots.cpu().numpy(),
                col_err=res.col_err.cpu().numpy(), err_hist=res.err_hist.cpu().numpy(), d=res.d, stop=res.stop)


@pytest.fixture(scope="module")
def gauss():
    g = synth.rng(96, 0, 0)
    return synth.quantize(g.standard_normal((M, N)), "f32")


@pytest.mark.parametrize("loop", ["0", "1"])
def test_identity_at_max_d(gauss, loop, monkeypatch):
    """loop = 0: one launch per kernel of a step; 1: the persistent loop."""
    import paper_1503_05947_amd as rbd
    monkeypatch.setenv("RBD_LOOP", loop)
    stored, vals = gauss
    print(f"[gpu] max d identity {M}x{N} d_max={D} RBD_LOOP={loop}", flush=True)
    dev = _host(rbd.fit(to_device(stored, "f32"), tol=0.0, d_max=D))
    ref = oracle.rbd_fit(vals, 0.0, D)
    assert dev["d"] == D == ref.d
    msgs = compare_fit(dev, ref, vals)
    assert msgs == [], "; ".join(msgs)


def test_diagonal_at_max_d(gauss):
    import torch
    import paper_1503_05947_amd as rbd
    stored, vals = gauss
    w = synth.random_weights(4, M)
    print(f"[gpu] max d diagonal {M}x{N} d_max={D}", flush=True)
    dev = _host(rbd.fit(to_device(stored, "f32"), tol=0.0, d_max=D, weights=torch.from_numpy(w).to("cuda:0")))
    ref = oracle.rbd_fit(vals, 0.0, D, weights=w)
    msgs = compare_fit(dev, ref, vals, weights=w)
    assert msgs == [], "; ".join(msgs)


def test_spd_at_max_d(gauss):
    from test_gpu_spd import _norms_A, device_csr
    import paper_1503_05947_amd as rbd
    stored, vals = gauss
    ip, ix, av = synth.grid_laplacian_spd(44, 25, 1.0)
    A = sp.csr_matrix((av, ix, ip), shape=(M, M))
    print(f"[gpu] max d spd {M}x{N} d_max={D}", flush=True)
    dev = _host(rbd.fit(to_device(stored, "f32"), tol=0.0, d_max=D, A=device_csr(ip, ix, av)))
    ref = oracle.rbd_fit(vals, 0.0, D, A=A)
    msgs = compare_fit(dev, ref, vals, norms=lambda R: _norms_A(R, A))
    assert msgs == [], "; ".join(msgs)


@pytest.mark.parametrize("m,n,d_max", [(100, 250_000, 24), (2_000_000, 8, 8)])
def test_extreme_shapes(m, n, d_max):
    """Very wide (many column blocks in the update and argmax, a long refresh
    queue) and very tall and skinny (two 16-byte vectors per row of X)."""
    import paper_1503_05947_amd as rbd
    g = synth.rng(98, m % 1000, n % 1000)
    r = min(m, n, 12)
    X = (g.standard_normal((m, r)) * (10.0 ** -np.arange(r) / 2)) @ g.standard_normal((r, n)) \
        + 1e-6 * g.standard_normal((m, n))
    stored, vals = synth.quantize(X, "f32")
    print(f"[gpu] extreme shape {m}x{n} d_max={d_max}", flush=True)
    dev = _host(rbd.fit(to_device(stored, "f32"), tol=0.0, d_max=d_max))
    ref = oracle.rbd_fit(vals, 0.0, d_max)
    msgs = compare_fit(dev, ref, vals)
    assert msgs == [], "; ".join(msgs)
