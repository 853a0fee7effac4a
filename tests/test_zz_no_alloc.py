"""rbd_fit_noalloc (for callers that cannot allocate device memory) against
rbd_fit and the FP64 oracle: two calls in a row on one device, the second with
a smaller input, so the second call runs in scratch the first one left behind."""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_fit
from test_gpu_fit import to_device

pytestmark = pytest.mark.gpu

CASES = [
    ("bump_field 1500x1200 f32 rel 1e-5", lambda: synth.bump_field(7, m=1500, n=1200).X, "f32", 1e-5, True, 96),
    ("lowrank 512x256 f32", lambda: synth.lowrank_spectrum(2).X, "f32", 1e-8, False, 64),
]


def _host(r):
    return dict(Y=r.Y.cpu().numpy(), T=r.T.cpu().numpy(), pivots=r.pivots.cpu().numpy(),
                col_err=r.col_err.cpu().numpy(), err_hist=r.err_hist.cpu().numpy(), d=r.d, stop=r.stop)


def test_noalloc_matches_fit_on_two_calls_in_a_row():
    import torch

    import paper_1503_05947_amd as rbd
    for name, make, dt, tol, rel, d_max in CASES:
        stored, vals = synth.quantize(make(), dt)
        print(f"[gpu] noalloc {name} shape={vals.shape} d_max={d_max}", flush=True)
        X = to_device(stored, dt)
        m, n = X.shape
        ref_bufs = rbd.FitBuffers(m, n, d_max, X.dtype, X.device)
        rbd.fit_into(ref_bufs, X, tol=tol, rel=rel)
        nb = rbd.FitBuffers(m, n, d_max, X.dtype, X.device, workspace=False)
        assert nb.workspace is None
        rbd.fit_noalloc_into(nb, X, tol=tol, rel=rel)
        torch.cuda.synchronize()
        a, b = _host(ref_bufs.result()), _host(nb.result())
        assert a["d"] == b["d"] and a["stop"] == b["stop"]
        for key in ("Y", "T", "pivots", "col_err", "err_hist"):
            assert np.array_equal(a[key], b[key]), (name, key)
        ref = oracle.rbd_fit(vals, tol, d_max, rel=rel)
        rep = compare_fit(b, ref, vals)
        print(f"[gpu] noalloc {name}: {rep.summary()}", flush=True)
        assert rep == [], "; ".join(rep)


def test_noalloc_rejects_a_fit_beyond_its_scratch():
    import torch

    import paper_1503_05947_amd as rbd
    from paper_1503_05947_amd import _lib
    X = torch.zeros((1 << 20, 64), dtype=torch.float32, device="cuda:0")
    nb = rbd.FitBuffers(1 << 20, 64, 64, X.dtype, X.device, workspace=False)
    assert _lib.fit_workspace_size(1 << 20, 64, 64, _lib.RBD_F32) > _lib.RBD_NOALLOC_MAX_BYTES
    with pytest.raises(RuntimeError, match="scratch"):
        rbd.fit_noalloc_into(nb, X)
