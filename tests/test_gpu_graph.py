"""Captured fits (rbd_fit_graph_*): every replay must equal an eager fit of the
same data bit for bit -- replays are checked one by one, with eager work on the
device in between, and after X is overwritten in place."""
import numpy as np
import pytest

import synth
from test_gpu_fit import to_device

pytestmark = pytest.mark.gpu


def _snap(res):
    return [res.Y.cpu().numpy(), res.T.cpu().numpy(), res.pivots.cpu().numpy(), res.col_err.cpu().numpy(),
            res.err_hist.cpu().numpy(), res.d, res.stop]


def _same(a, b):
    for u, v in zip(a, b):
        if isinstance(u, np.ndarray):
            if u.shape != v.shape or not np.array_equal(u, v):
                return False
        elif u != v:
            return False
    return True


@pytest.fixture(params=["auto", "0"])
def driver(request, monkeypatch):
    """auto: the persistent loop takes these cache-resident shapes; 0: one launch per kernel."""
    if request.param == "0":
        monkeypatch.setenv("RBD_LOOP", "0")
    return request.param


@pytest.mark.parametrize("dtype,weighted", [("f32", False), ("bf16", False), ("f32", True)])
def test_replays_equal_eager_fits(dtype, weighted, driver):
    import torch
    import paper_1503_05947_amd as rbd
    print(f"[gpu] graph replay dtype={dtype} weighted={weighted} driver={driver}", flush=True)
    wl = synth.lowrank_spectrum(0)
    stored, _ = synth.quantize(wl.X, dtype)
    X = to_device(stored, dtype)
    w = torch.from_numpy(synth.random_weights(0, X.shape[0])).to("cuda:0") if weighted else None
    eager = _snap(rbd.fit(X, tol=wl.tol, d_max=wl.d_max, weights=w))
    bufs = rbd.FitBuffers(X.shape[0], X.shape[1], wl.d_max, X.dtype, X.device)
    g = rbd.FitGraph(bufs, X, tol=wl.tol, weights=w)
    for rep in range(3):
        g.replay()
        got = _snap(bufs.result())
        assert _same(got, eager), f"replay {rep} differs"
        # eager work between replays: another fit and torch kernels on the same device
        rbd.fit(X, tol=0.0, d_max=5, weights=w)
        torch.cuda.synchronize()
        _ = (X.float() * 2.0).sum().item()
    # new contents of the same X buffer: the replay fits them
    X2s, _ = synth.quantize(synth.lowrank_spectrum(3).X, dtype)
    X.copy_(to_device(X2s, dtype))
    eager2 = _snap(rbd.fit(X, tol=wl.tol, d_max=wl.d_max, weights=w))
    g.replay()
    assert _same(_snap(bufs.result()), eager2)
    g.close()


def test_fixed_steps_bump_field_replay(driver):
    import paper_1503_05947_amd as rbd
    print(f"[gpu] graph replay bump field 2048 x 2048 fixed 256 steps driver={driver}", flush=True)
    wl = synth.bump_field(0)
    X = to_device(synth.quantize(wl.X, "f32")[0], "f32")
    eager = _snap(rbd.fit(X, tol=0.0, d_max=256))
    bufs = rbd.FitBuffers(2048, 2048, 256, X.dtype, X.device)
    g = rbd.FitGraph(bufs, X, tol=0.0)
    g.replay()
    g.replay()
    assert _same(_snap(bufs.result()), eager)
    g.close()


def test_null_stream_rejected():
    import ctypes
    import torch
    from paper_1503_05947_amd import _lib
    print("[gpu] graph null stream", flush=True)
    lib = _lib.load()
    X = torch.zeros((16, 8), dtype=torch.float32, device="cuda:0")
    h = ctypes.c_void_p()
    rc = lib.rbd_fit_graph_create(X.data_ptr(), 0, 16, 8, 8, None, 0.0, 0, 4, -1, 4096, 4096, 4096, 4096, 4096,
                                  4096, 4096, None, 1 << 20, 1 << 30, None, ctypes.byref(h))
    assert rc == _lib.RBD_EINVAL
