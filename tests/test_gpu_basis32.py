"""rbd_fit_basis with the basis kept in FP32 while the loop runs (meant for
BF16-stored data) against the FP64 oracle.

The stored basis is the FP64 one rounded to FP32 (orthonormal to about 1e-7),
and the downdated errors carry an absolute error of order
2^-24 ||x_j||^2 / e_j between exact refreshes; the checks use that accuracy:
basis vectors orthonormal to 1e-6, errors to max(1e-5, 2^-22 E_0 / E_d) E_0,
pivots compared where the oracle's top two errors differ by more than 1e-5 E_0.
Every case prints its name before touching the GPU."""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_fit
from test_gpu_fit import to_device

pytestmark = pytest.mark.gpu


def run(stored, dtype, tol, d_max, rel=False, basis="f32"):
    import paper_1503_05947_amd as rbd
    res = rbd.fit(to_device(stored, dtype), tol=tol, d_max=d_max, rel=rel, basis=basis)
    return dict(Y=res.Y.cpu().numpy(), T=res.T.cpu().numpy(), pivots=res.pivots.cpu().numpy(),
                col_err=res.col_err.cpu().numpy(), err_hist=res.err_hist.cpu().numpy(), d=res.d, stop=res.stop)


def check32(name, stored, vals, dtype, tol, d_max, rel=False, exact_d=True):
    print(f"[gpu] basis f32 {name} dtype={dtype} shape={vals.shape} tol={tol} rel={rel} d_max={d_max}", flush=True)
    dev = run(stored, dtype, tol, d_max, rel=rel)
    ref = oracle.rbd_fit(vals, tol, d_max, rel=rel)
    E0 = ref.err_hist[0]
    rtol = max(1e-5, 2.0 ** -22 * E0 / max(ref.err_hist[-1], 1e-300))
    rep = compare_fit(dev, ref, vals, rtol=rtol, gap=1e-5, exact_d=exact_d, basis_tol=1e-6)
    print(f"[gpu]   rtol {rtol:.2e}: {rep.summary()}", flush=True)
    assert rep == [], f"{name}: " + "; ".join(rep)
    return dev, ref


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_lowrank(dtype):
    w = synth.lowrank_spectrum(2)
    stored, vals = synth.quantize(w.X, dtype)
    dev, ref = check32("lowrank rel 1e-2", stored, vals, dtype, 1e-2, 64, rel=True)
    assert dev["stop"] == "tol"


def test_bump_field_bf16():
    w = synth.bump_field(0)
    stored, vals = synth.quantize(w.X, "bf16")
    check32("bump 2048^2 rel 1e-3", stored, vals, "bf16", 1e-3, 256, rel=True)


def test_ragged_fixed_steps_to_the_bf16_floor():
    w = synth.bump_field(2, m=1111, n=777)
    stored, vals = synth.quantize(w.X, "bf16")
    dev, ref = check32("ragged 1111x777 fixed 60", stored, vals, "bf16", 0.0, 60, exact_d=False)
    assert dev["d"] == 60


def test_parametric_small_grid_bf16():
    pf = synth.parametric_field(0, grid=48, n=300)
    stored, vals = synth.quantize(pf.full(), "bf16")
    check32("parametric 48^2 fixed 40", stored, vals, "bf16", 0.0, 40, exact_d=False)


def test_f64_basis_entry_point_equals_rbd_fit():
    import paper_1503_05947_amd as rbd
    w = synth.bump_field(4, m=700, n=900)
    stored, vals = synth.quantize(w.X, "bf16")
    print("[gpu] rbd_fit_basis(F64) vs rbd_fit", flush=True)
    X = to_device(stored, "bf16")
    a = rbd.fit(X, tol=0.0, d_max=40)
    b = rbd.fit(X, tol=0.0, d_max=40, basis="f64")
    for k in ("Y", "T", "pivots", "col_err", "err_hist"):
        assert np.array_equal(getattr(a, k).cpu().numpy(), getattr(b, k).cpu().numpy()), k


def test_weighted_rejects_the_f32_basis():
    import torch
    import paper_1503_05947_amd as rbd
    X = torch.ones((8, 8), dtype=torch.float32, device="cuda:0")
    w = torch.ones(8, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError):
        rbd.fit(X, tol=0.0, d_max=4, weights=w, basis="f32")
