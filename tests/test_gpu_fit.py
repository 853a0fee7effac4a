"""Parity of the HIP rbd_fit / rbd_project path with the FP64 oracle (needs a gfx950 GPU).

Every case prints its name, shape and seed before touching the GPU.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_fit, invariant_msgs

pytestmark = pytest.mark.gpu

TORCH_DT = {}


def _torch():
    import torch
    if not TORCH_DT:
        TORCH_DT.update(f64=torch.float64, f32=torch.float32, bf16=torch.bfloat16, f16=torch.float16)
    return torch


def to_device(stored, dtype, pad_cols=0):
    """Upload stored values; BF16 arrives as uint16 bit patterns.  pad_cols > 0 gives ldx > n."""
    torch = _torch()
    if dtype == "bf16":
        t = torch.from_numpy(stored.view(np.int16)).view(torch.bfloat16)
    else:
        t = torch.from_numpy(stored)
    if pad_cols:
        m, n = t.shape
        big = torch.zeros((m, n + pad_cols), dtype=t.dtype)
        big[:, :n] = t
        return big.to("cuda:0")[:, :n]
    return t.to("cuda:0")


def run_fit(stored, dtype, tol, d_max, rel=False, start=-1, pad_cols=0):
    import paper_1503_05947_amd as rbd
    X = to_device(stored, dtype, pad_cols)
    res = rbd.fit(X, tol=tol, d_max=d_max, rel=rel, start=start)
    return dict(Y=res.Y.cpu().numpy(), T=res.T.cpu().numpy(), pivots=res.pivots.cpu().numpy(),
                col_err=res.col_err.cpu().numpy(), err_hist=res.err_hist.cpu().numpy(), d=res.d,
                stop=res.stop)


def check(name, stored, vals, dtype, tol, d_max, rel=False, start=-1, pad_cols=0, gap=1e-8, exact_d=True):
    print(f"[gpu] {name} dtype={dtype} shape={vals.shape} tol={tol} rel={rel} d_max={d_max}", flush=True)
    dev = run_fit(stored, dtype, tol, d_max, rel=rel, start=start, pad_cols=pad_cols)
    ref = oracle.rbd_fit(vals, tol, d_max, rel=rel, start=start)
    msgs = compare_fit(dev, ref, vals, gap=gap, exact_d=exact_d)
    print(f"[gpu] {name}: {msgs.summary()}", flush=True)
    assert msgs == [], f"{name}: " + "; ".join(msgs)
    return dev, ref


# ---------------------------------------------------------------------------
# the 512 x 256 low-rank workload in every storage type, several seeds
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lowrank_parity(dtype, seed):
    w = synth.lowrank_spectrum(seed)
    stored, vals = synth.quantize(w.X, dtype)
    dev, ref = check(f"lowrank seed={seed}", stored, vals, dtype, w.tol, w.d_max)
    if dtype == "f64":
        assert dev["d"] == ref.d and np.array_equal(dev["pivots"], ref.pivots)


def test_lowrank_fp32_stop_near_tolerance():
    """FP32 rounding leaves E_d within 0.4% of tau: the stop needs certified errors."""
    w = synth.lowrank_spectrum(0)
    stored, vals = synth.quantize(w.X, "f32")
    dev, ref = check("lowrank stop", stored, vals, "f32", w.tol, w.d_max)
    assert dev["d"] == ref.d and dev["stop"] == ref.stop


# ---------------------------------------------------------------------------
# the 2048 x 2048 bump field (relative tol 1e-4, d_max 256)
# ---------------------------------------------------------------------------
def test_bump_field_full_size_f32():
    w = synth.bump_field(0)
    stored, vals = synth.quantize(w.X, "f32")
    dev, ref = check("bump_field 2048^2", stored, vals, "f32", w.tol, w.d_max, rel=True)
    assert dev["stop"] == "tol"


def test_bump_field_full_size_f64_exact_pivots():
    """FP64 storage: the device must reproduce the oracle's pivots and d exactly."""
    w = synth.bump_field(0)
    stored, vals = synth.quantize(w.X, "f64")
    dev, ref = check("bump_field 2048^2 f64", stored, vals, "f64", w.tol, w.d_max, rel=True)
    assert dev["d"] == ref.d and np.array_equal(dev["pivots"], ref.pivots)


def test_bump_field_f64_exact_pivots():
    w = synth.bump_field(1, m=1024, n=1536)
    stored, vals = synth.quantize(w.X, "f64")
    dev, ref = check("bump_field f64", stored, vals, "f64", w.tol, w.d_max, rel=True)
    assert dev["d"] == ref.d and np.array_equal(dev["pivots"], ref.pivots)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_bump_field_fixed_steps_ragged(dtype):
    """tol = 0: runs to d_max; ragged shape (not a multiple of any tile)."""
    w = synth.bump_field(2, m=1111, n=777)
    stored, vals = synth.quantize(w.X, dtype)
    dev, ref = check("bump_field fixed", stored, vals, dtype, 0.0, 100, exact_d=False)
    assert dev["d"] == 100 and dev["stop"] == "dmax"


def test_parametric_field_small_grid():
    pf = synth.parametric_field(0, grid=48, n=300)
    stored, vals = synth.quantize(pf.full(), "f32")
    check("parametric 48^2", stored, vals, "f32", 0.0, 120, exact_d=False)


# ---------------------------------------------------------------------------
# exact recovery (Table 3, random rank r)
# ---------------------------------------------------------------------------
def test_table3_exact_dimensions(golden):
    for which, want in zip((1, 2, 3), golden["table3"]["intrinsic_dimension"]):
        X = synth.table3(which, 512)
        stored, vals = synth.quantize(X, "f64")
        dev, ref = check(f"table3 f{which}", stored, vals, "f64", 1e-10, 20, rel=True)
        assert dev["d"] == want and dev["stop"] == "tol"


@pytest.mark.parametrize("r", [1, 5, 17])
def test_random_rank_exact_recovery(r):
    X = synth.random_rank(r, 640, 300, r)
    dev, ref = check(f"rank {r}", X, X, "f64", 1e-10, 64, rel=True)
    assert dev["d"] == r and dev["stop"] == "tol"
    assert dev["err_hist"][-1] < 1e-12 * dev["err_hist"][0]


def test_approx_field_paper_example(golden):
    g = golden["approx_field"]
    X = synth.approx_field(g["grid"])
    dev, ref = check("approx_field 5001^2", X, X, "f64", 0.0, g["d"], exact_d=True)
    assert dev["d"] == g["d"]
    err = np.max(np.abs(X - dev["Y"] @ dev["T"]))
    assert err < g["max_pointwise_error_below"], err


# ---------------------------------------------------------------------------
# layouts and edge cases
# ---------------------------------------------------------------------------
def test_strided_rows_and_unaligned_leading_dimension():
    w = synth.bump_field(3, m=300, n=257)
    stored, vals = synth.quantize(w.X, "f32")
    check("ldx = n + 64", stored, vals, "f32", 1e-3, 60, rel=True, pad_cols=64)
    check("ldx = n + 3 (unaligned)", stored, vals, "f32", 1e-3, 60, rel=True, pad_cols=3)
    stored, vals = synth.quantize(w.X, "bf16")
    check("bf16 ldx = n + 5", stored, vals, "bf16", 1e-2, 40, rel=True, pad_cols=5)


def test_zero_matrix():
    print("[gpu] zero matrix", flush=True)
    dev = run_fit(np.zeros((33, 17), np.float32), "f32", 0.0, 5)
    assert dev["d"] == 0 and dev["stop"] == "break"
    assert np.all(dev["col_err"] == 0) and dev["err_hist"].tolist() == [0.0]


def test_tolerance_at_and_above_largest_norm():
    X = synth.rng(97, 0, 0).standard_normal((30, 20))
    E0 = np.linalg.norm(X, axis=0).max()
    print("[gpu] tol above E0", flush=True)
    dev = run_fit(X, "f64", E0 * 1.001, 10)
    assert dev["d"] == 0 and dev["stop"] == "break"
    dev = run_fit(X, "f64", E0, 10)
    assert dev["d"] == 1 and dev["stop"] == "tol"


def test_duplicate_columns_tie_lowest_index():
    X = synth.rng(97, 1, 0).standard_normal((20, 8))
    X[:, 5] = X[:, 2] = X[:, 2] * 10.0
    dev, ref = check("ties", X, X, "f64", 1e-12, 8)
    assert dev["pivots"][0] == 2 and 5 not in dev["pivots"].tolist() and dev["d"] == 7


def test_single_row_single_column_and_clamp():
    print("[gpu] 1 x 3 / 2 x 1 / clamp", flush=True)
    dev = run_fit(np.array([[3.0, -4.0, 1.0]]), "f64", 0.0, 3)
    assert dev["d"] == 1 and dev["pivots"].tolist() == [1] and abs(dev["T"][0, 1] - 4.0) < 1e-15
    dev = run_fit(np.array([[3.0], [4.0]]), "f64", 0.0, 3)
    assert dev["d"] == 1 and abs(dev["err_hist"][0] - 5.0) < 1e-15 and dev["err_hist"][1] == 0.0
    X = synth.rng(97, 2, 0).standard_normal((9, 14))
    dev, ref = check("clamp 9x14", X, X, "f64", 0.0, 50)
    assert dev["d"] == 9


def test_user_start_column():
    X = synth.rng(97, 4, 0).standard_normal((25, 12))
    dev, ref = check("start=7", X, X, "f64", 0.0, 5, start=7)
    assert dev["pivots"][0] == 7


def test_nonfinite_input_reports_status():
    import paper_1503_05947_amd as rbd
    torch = _torch()
    print("[gpu] nonfinite", flush=True)
    X = torch.ones((40, 30), dtype=torch.float32)
    X[7, 3] = float("nan")
    with pytest.raises(FloatingPointError):
        rbd.fit(X.cuda(), tol=0.0, d_max=4)
    X[7, 3] = float("inf")
    with pytest.raises(FloatingPointError):
        rbd.fit(X.cuda(), tol=0.0, d_max=4)


def test_invalid_arguments_rejected_before_launch():
    import paper_1503_05947_amd as rbd
    torch = _torch()
    X = torch.ones((8, 8), dtype=torch.float32, device="cuda:0")
    with pytest.raises(RuntimeError):
        rbd.fit(X, tol=-1.0, d_max=4)
    with pytest.raises(RuntimeError):
        rbd.fit(X, tol=0.0, d_max=0)
    with pytest.raises(RuntimeError):
        rbd.fit(X, tol=0.0, d_max=4, start=8)
    with pytest.raises((TypeError, ValueError)):
        rbd.fit(X.t(), tol=0.0, d_max=4)


def test_bitwise_deterministic():
    w = synth.bump_field(4, m=700, n=900)
    stored, vals = synth.quantize(w.X, "f32")
    print("[gpu] determinism", flush=True)
    a = run_fit(stored, "f32", 0.0, 64)
    b = run_fit(stored, "f32", 0.0, 64)
    for key in ("Y", "T", "pivots", "col_err", "err_hist"):
        assert np.array_equal(a[key], b[key]), key


# ---------------------------------------------------------------------------
# out-of-sample compression
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("vdtype", ["f64", "f32", "bf16"])
def test_project_parity(vdtype):
    import paper_1503_05947_amd as rbd
    torch = _torch()
    w = synth.bump_field(5, m=900, n=400)
    stored, vals = synth.quantize(w.X, "f32")
    print(f"[gpu] project {vdtype}", flush=True)
    dev = run_fit(stored, "f32", 0.0, 50)
    Y = dev["Y"]
    V64 = synth.bump_field(6, m=900, n=130).X
    V64[:, :5] = Y @ synth.rng(95, 0, 0).standard_normal((Y.shape[1], 5))   # in span(Y)
    Vs, Vv = synth.quantize(V64, vdtype)
    Tv, err = rbd.project(torch.from_numpy(Y).cuda(), to_device(Vs, vdtype))
    C, e = oracle.rbd_project(Y, Vv)
    Tv, err = Tv.cpu().numpy(), err.cpu().numpy()
    scale = np.linalg.norm(Vv, axis=0)
    assert np.max(np.linalg.norm(Tv - C, axis=0) / scale) < 1e-12
    assert np.max(np.abs(err - e) / scale) < 1e-12
    if vdtype == "f64":
        assert np.max(err[:5] / scale[:5]) < 1e-13


def test_project_reproduces_fit_columns():
    import paper_1503_05947_amd as rbd
    torch = _torch()
    w = synth.lowrank_spectrum(3)
    stored, vals = synth.quantize(w.X, "f32")
    print("[gpu] project = fit columns", flush=True)
    dev = run_fit(stored, "f32", w.tol, w.d_max)
    Tv, err = rbd.project(torch.from_numpy(dev["Y"]).cuda(), to_device(stored, "f32"))
    Tv, err = Tv.cpu().numpy(), err.cpu().numpy()
    assert np.max(np.abs(Tv - dev["T"])) < 1e-14
    mask = np.ones(vals.shape[1], bool)
    mask[dev["pivots"]] = False
    assert np.max(np.abs(err[mask] - dev["col_err"][mask])) < 1e-9 * np.linalg.norm(vals, axis=0).max()


@pytest.mark.parametrize("m,d,k,vdtype", [(300000, 70, 7, "f16"), (300000, 64, 1, "f32"), (40000, 200, 300, "f32"),
                                          (131072, 1024, 65, "bf16")])
def test_project_many_row_splits(m, d, k, vdtype):
    """Enough rows that the product is split over rows and the residual partials
    are summed in two levels; ragged d and k, several storage types."""
    import paper_1503_05947_amd as rbd
    torch = _torch()
    print(f"[gpu] project m={m} d={d} k={k} {vdtype}", flush=True)
    Y = synth.haar(synth.rng(97, m, d), m, d)
    V64 = synth.rng(98, m, k).standard_normal((m, k))
    V64[:, : min(k, 3)] += Y[:, :3] @ np.ones((3, min(k, 3)))     # components inside span(Y)
    Vs, Vv = synth.quantize(V64, vdtype)
    Tv, err = rbd.project(torch.from_numpy(Y).cuda(), to_device(Vs, vdtype))
    C, e = oracle.rbd_project(Y, Vv)
    Tv, err = Tv.cpu().numpy(), err.cpu().numpy()
    scale = np.linalg.norm(Vv, axis=0)
    assert np.max(np.linalg.norm(Tv - C, axis=0) / scale) < 1e-12
    assert np.max(np.abs(err - e) / scale) < 1e-12
