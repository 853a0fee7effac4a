"""rbd_fit_basis with the basis kept in FP32 once the fit passes 128 columns
(meant for BF16-stored data) against the FP64 oracle, and against rbd_fit for
fits that end within 128 columns (those run rbd_fit's steps exactly).  The
test inputs are small, so they run with RBD_LOOP=0: inputs of at most 64 MB
otherwise take the single-launch loop, which keeps the FP64 basis.

Past 128 columns the stored basis is the FP64 one rounded to FP32
(orthonormal to about 1e-7), and the downdated errors carry an absolute error
of order 2^-24 ||x_j||^2 / e_j between exact refreshes; the checks use that
accuracy: basis vectors orthonormal to 1e-6, errors to
max(1e-5, 2^-22 E_0 / E_d) E_0, pivots compared where the oracle's top two
errors differ by more than 1e-5 E_0.  Every case prints its name before
touching the GPU."""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_fit
from test_gpu_fit import to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def per_kernel_driver(monkeypatch, request):
    if "loop" not in request.fixturenames:
        monkeypatch.setenv("RBD_LOOP", "0")


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


def test_bump_field_bf16_256_steps():
    w = synth.bump_field(0)
    stored, vals = synth.quantize(w.X, "bf16")
    dev, _ = check32("bump 2048^2 fixed 256", stored, vals, "bf16", 0.0, 256, exact_d=False)
    assert dev["d"] == 256


def test_ragged_fixed_steps_past_the_switch():
    w = synth.bump_field(2, m=1111, n=777, noise=1e-2)
    stored, vals = synth.quantize(w.X, "bf16")
    dev, _ = check32("ragged 1111x777 fixed 200", stored, vals, "bf16", 0.0, 200, exact_d=False)
    assert dev["d"] == 200


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_parametric_small_grid_past_the_switch(dtype):
    pf = synth.parametric_field(0, grid=48, n=300)
    stored, vals = synth.quantize(pf.full(), dtype)
    dev, _ = check32("parametric 48^2 fixed 160", stored, vals, dtype, 0.0, 160, exact_d=False)
    assert dev["d"] == 160


@pytest.mark.parametrize("d_max", [128, 129, 136])
def test_switch_boundaries(d_max):
    """Fits that end exactly at, one past and one block past the switch column."""
    w = synth.bump_field(5, m=900, n=700, noise=1e-2)
    stored, vals = synth.quantize(w.X, "bf16")
    dev, _ = check32(f"bump 900x700 fixed {d_max}", stored, vals, "bf16", 0.0, d_max, exact_d=False)
    assert dev["d"] == d_max


@pytest.mark.parametrize("loop", ["0", "auto"])
@pytest.mark.parametrize("case", ["lowrank", "bump_rel_1e-2", "bump_128"])
def test_within_128_columns_equals_rbd_fit(case, loop, monkeypatch):
    """A fit that ends within 128 columns runs rbd_fit's steps (and an input the
    single-launch loop takes runs rbd_fit itself): identical results."""
    import paper_1503_05947_amd as rbd
    if loop == "0":
        monkeypatch.setenv("RBD_LOOP", "0")
    else:
        monkeypatch.delenv("RBD_LOOP", raising=False)
    if case == "lowrank":
        stored, _ = synth.quantize(synth.lowrank_spectrum(2).X, "bf16")
        tol, rel, d_max = 1e-2, True, 64
    elif case == "bump_rel_1e-2":
        stored, _ = synth.quantize(synth.bump_field(0).X, "bf16")
        tol, rel, d_max = 1e-2, True, 512
    else:
        stored, _ = synth.quantize(synth.bump_field(3, m=1500, n=1300).X, "bf16")
        tol, rel, d_max = 0.0, False, 128
    print(f"[gpu] basis f32 = f64 within 128 columns: {case}, RBD_LOOP={loop}", flush=True)
    X = to_device(stored, "bf16")
    a = rbd.fit(X, tol=tol, d_max=d_max, rel=rel, basis="f64")
    b = rbd.fit(X, tol=tol, d_max=d_max, rel=rel, basis="f32")
    assert a.d <= 128 and a.d == b.d
    for k in ("Y", "T", "pivots", "col_err", "err_hist"):
        assert np.array_equal(getattr(a, k).cpu().numpy(), getattr(b, k).cpu().numpy()), k


def test_small_input_past_128_columns_keeps_the_loop(monkeypatch):
    """Inputs the single-launch loop takes keep the FP64 basis in every mode."""
    import paper_1503_05947_amd as rbd
    monkeypatch.delenv("RBD_LOOP", raising=False)
    stored, _ = synth.quantize(synth.bump_field(6, m=1200, n=900, noise=1e-2).X, "bf16")
    print("[gpu] basis f32 on a cache-resident input, 200 steps", flush=True)
    X = to_device(stored, "bf16")
    a = rbd.fit(X, tol=0.0, d_max=200, basis="f64")
    b = rbd.fit(X, tol=0.0, d_max=200, basis="f32")
    for k in ("Y", "T", "pivots", "col_err", "err_hist"):
        assert np.array_equal(getattr(a, k).cpu().numpy(), getattr(b, k).cpu().numpy()), k


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
