"""Batched fits (one persistent launch over many uneven matrices) vs the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from parity import compare_fit

pytestmark = pytest.mark.gpu


def make_batch(count, seed, lo=8, hi=300, dtype="f32"):
    g = synth.rng(77, seed, 0)
    mats, vals = [], []
    for b in range(count):
        m = int(np.exp(g.uniform(np.log(lo), np.log(hi))))
        n = int(np.exp(g.uniform(np.log(lo), np.log(hi))))
        X = synth.batched_matrix(seed, b, m, n)
        st, v = synth.quantize(X, dtype)
        mats.append(st)
        vals.append(v)
    return mats, vals


def to_dev(stored, dtype):
    import torch
    if dtype == "bf16":
        return torch.from_numpy(stored.view(np.int16)).view(torch.bfloat16).cuda()
    return torch.from_numpy(stored).cuda()


def host(res):
    return dict(Y=res.Y.cpu().numpy(), T=res.T.cpu().numpy(), pivots=res.pivots.cpu().numpy(),
                col_err=res.col_err.cpu().numpy(), err_hist=res.err_hist.cpu().numpy(), d=res.d)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_batched_parity_uneven(dtype):
    import paper_1503_05947_amd as rbd
    mats, vals = make_batch(40, seed=1, dtype=dtype)
    print(f"[gpu] batched 40 uneven matrices dtype={dtype}", flush=True)
    tol = 1e-6 if dtype != "bf16" else 1e-2
    res, plan = rbd.fit_batched([to_dev(s, dtype) for s in mats], tol=tol, d_max=64, rel=True)
    for b, (r, v) in enumerate(zip(res, vals)):
        ref = oracle.rbd_fit(v, tol, 64, rel=True)
        msgs = compare_fit(host(r), ref, v)
        assert msgs == [], f"matrix {b} {v.shape}: " + "; ".join(msgs)


@pytest.mark.parametrize("threads,wg", [(64, 1), (128, 4), (512, 2), (1024, 1)])
def test_batched_every_workgroup_shape(threads, wg):
    import paper_1503_05947_amd as rbd
    mats, vals = make_batch(24, seed=2)
    print(f"[gpu] batched shape threads={threads} wg_per_cu={wg}", flush=True)
    res, _ = rbd.fit_batched([to_dev(s, "f32") for s in mats], tol=1e-6, d_max=48, rel=True,
                             config=rbd.BatchConfig(threads, wg))
    for r, v in zip(res, vals):
        ref = oracle.rbd_fit(v, 1e-6, 48, rel=True)
        assert compare_fit(host(r), ref, v) == []


def test_batched_edge_cases():
    import paper_1503_05947_amd as rbd
    print("[gpu] batched edge cases", flush=True)
    g = synth.rng(78, 0, 0)
    mats = [np.zeros((20, 9)),                       # all zero: breaks at once
            g.standard_normal((1, 7)),               # one row
            g.standard_normal((9, 1)),               # one column
            g.standard_normal((300, 13)),            # tall, full rank
            synth.table3(3, 128),                    # rank 3
            g.standard_normal((33, 50))]
    bad = g.standard_normal((10, 10))
    bad[3, 4] = np.nan
    mats.insert(3, bad)
    res, plan = rbd.fit_batched([to_dev(np.ascontiguousarray(A), "f64") for A in mats], tol=1e-10, d_max=40,
                                rel=True)
    assert res[3] is None                            # the non-finite matrix reports its own status
    others = [i for i in range(len(mats)) if i != 3]
    for i in others:
        ref = oracle.rbd_fit(mats[i], 1e-10, 40, rel=True)
        assert compare_fit(host(res[i]), ref, mats[i]) == [], i
    assert res[0].d == 0 and res[1].d == 1 and res[2].d == 1
    assert res[5].d == 3


def test_batched_deterministic_and_autotune():
    import paper_1503_05947_amd as rbd
    mats, vals = make_batch(64, seed=3, hi=400)
    print("[gpu] batched autotune + determinism", flush=True)
    dev = [to_dev(s, "f32") for s in mats]
    plan = rbd.BatchPlan([A.shape[0] for A in dev], [A.shape[1] for A in dev], 64, dev[0].dtype, dev[0].device)
    Xp = plan.pack(dev)
    cfg = plan.autotune(Xp, tol=1e-6, rel=True, sample_stride=4)
    assert cfg.threads in (128, 256, 512, 1024) and cfg.wg_per_cu in (1, 2, 4, 8)
    assert plan.trials[(cfg.threads, cfg.wg_per_cu)] == min(t for t in plan.trials.values() if t > 0)
    plan.run(Xp, tol=1e-6, rel=True)
    a = [host(r) for r in plan.results()]
    plan.run(Xp, tol=1e-6, rel=True)
    b = [host(r) for r in plan.results()]
    for x, y, v in zip(a, b, vals):
        for k in ("Y", "T", "pivots", "col_err", "err_hist"):
            assert np.array_equal(x[k], y[k])
        ref = oracle.rbd_fit(v, 1e-6, 64, rel=True)
        assert compare_fit(x, ref, v) == []


def config4_subbatch(count=12):
    """Matrices of the 4096-matrix workload itself (sizes log-uniform in [64, 1024],
    spectrum 10^(-i/8)): its four largest by m*n and eight spread over the rest."""
    ms, ns = synth.batched_sizes(0, count=4096)
    order = np.argsort(-(ms * ns), kind="stable")
    idx = list(order[:4]) + list(order[np.linspace(4, len(order) - 1, count - 4).astype(int)])
    mats, vals = [], []
    for b in idx:
        st, v = synth.quantize(synth.batched_matrix(0, int(b), int(ms[b]), int(ns[b])), "f32")
        mats.append(st)
        vals.append(v)
    return idx, mats, vals


@pytest.mark.parametrize("threads,wg", [(512, 1), (1024, 1)])
def test_batched_parity_at_workload_sizes(threads, wg):
    """m, n up to 1024, d_max 128, relative tol 1e-6, FP32: the batched workload's
    own matrices (including its largest) against the oracle, under the autotuned
    shape (512 threads, one workgroup per CU) and the widest one."""
    import paper_1503_05947_amd as rbd
    idx, mats, vals = config4_subbatch()
    print(f"[gpu] batched workload sizes threads={threads} wg_per_cu={wg}: "
          + ", ".join(f"{v.shape[0]}x{v.shape[1]}" for v in vals), flush=True)
    res, _ = rbd.fit_batched([to_dev(s, "f32") for s in mats], tol=1e-6, d_max=128, rel=True,
                             config=rbd.BatchConfig(threads, wg))
    for b, r, v in zip(idx, res, vals):
        ref = oracle.rbd_fit(v, 1e-6, 128, rel=True)
        rep = compare_fit(host(r), ref, v)
        print(f"[gpu]   matrix {b} {v.shape}: d={r.d} {rep.summary()}", flush=True)
        assert rep == [], f"matrix {b} {v.shape}: " + "; ".join(rep)
