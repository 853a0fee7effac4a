"""Basis columns reach Y in blocks of 8 (the columns of an unfinished block are
kept in a staging buffer and copied into Y before exact refreshes and after the
loop).  These fits stop at every residue of d modulo 8, through each of the
three step sequences (A = I, diagonal A, sparse SPD A), and compare Y, T and
the errors with the FP64 oracle.  Every case prints its name before touching
the GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from parity import compare_fit
from test_gpu_fit import to_device

pytestmark = pytest.mark.gpu


def _host(res):
    return dict(Y=res.Y.cpu().numpy(), T=res.T.cpu().numpy(), pivots=res.pivots.cpu().numpy(),
                col_err=res.col_err.cpu().numpy(), err_hist=res.err_hist.cpu().numpy(), d=res.d, stop=res.stop)


@pytest.fixture(autouse=True)
def multi_launch_driver(monkeypatch):
    """These cases check the staged basis columns of the one-launch-per-kernel
    driver; the persistent loop would otherwise take shapes this small."""
    monkeypatch.setenv("RBD_LOOP", "0")


@pytest.fixture(scope="module")
def field():
    g = synth.rng(95, 0, 0)
    m, n = 300, 40
    X = synth.random_rank(7, m, n, 30) + 1e-3 * g.standard_normal((m, n))
    return synth.quantize(X, "f32")


@pytest.mark.parametrize("d_max", list(range(1, 21)))
def test_identity_every_final_block_residue(field, d_max):
    import paper_1503_05947_amd as rbd
    stored, vals = field
    print(f"[gpu] stage identity d_max={d_max}", flush=True)
    dev = _host(rbd.fit(to_device(stored, "f32"), tol=0.0, d_max=d_max))
    ref = oracle.rbd_fit(vals, 0.0, d_max)
    assert dev["d"] == d_max
    msgs = compare_fit(dev, ref, vals)
    assert msgs == [], "; ".join(msgs)


@pytest.mark.parametrize("d_max", [1, 7, 8, 9, 15, 16, 17])
def test_diagonal_every_final_block_residue(field, d_max):
    import torch
    import paper_1503_05947_amd as rbd
    stored, vals = field
    w = synth.random_weights(3, vals.shape[0])
    print(f"[gpu] stage diagonal d_max={d_max}", flush=True)
    dev = _host(rbd.fit(to_device(stored, "f32"), tol=0.0, d_max=d_max, weights=torch.from_numpy(w).to("cuda:0")))
    ref = oracle.rbd_fit(vals, 0.0, d_max, weights=w)
    msgs = compare_fit(dev, ref, vals, weights=w)
    assert msgs == [], "; ".join(msgs)


@pytest.mark.parametrize("d_max", [1, 7, 8, 9, 15, 16, 17])
def test_spd_every_final_block_residue(field, d_max):
    from test_gpu_spd import _norms_A, device_csr
    import paper_1503_05947_amd as rbd
    stored, vals = field
    ip, ix, av = synth.grid_laplacian_spd(20, 15, 1.0)
    A = sp.csr_matrix((av, ix, ip), shape=(300, 300))
    print(f"[gpu] stage spd d_max={d_max}", flush=True)
    dev = _host(rbd.fit(to_device(stored, "f32"), tol=0.0, d_max=d_max, A=device_csr(ip, ix, av)))
    ref = oracle.rbd_fit(vals, 0.0, d_max, A=A)
    msgs = compare_fit(dev, ref, vals, norms=lambda R: _norms_A(R, A))
    assert msgs == [], "; ".join(msgs)


def test_refresh_inside_a_block_then_more_steps():
    """Errors fall by many orders within a few steps, so exact refreshes run at
    steps whose staged block is incomplete, and the loop continues past them."""
    import paper_1503_05947_amd as rbd
    wl = synth.lowrank_spectrum(3)
    stored, vals = synth.quantize(wl.X, "f32")
    print("[gpu] stage refresh inside a block", flush=True)
    dev = _host(rbd.fit(to_device(stored, "f32"), tol=wl.tol, d_max=wl.d_max))
    ref = oracle.rbd_fit(vals, wl.tol, wl.d_max)
    msgs = compare_fit(dev, ref, vals)
    assert msgs == [], "; ".join(msgs)
    Y = dev["Y"]
    assert np.max(np.abs(Y.T @ Y - np.eye(dev["d"]))) < 1e-12
