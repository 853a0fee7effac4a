"""Parity of rbd_classify (compression c = Y'v, section 3.1, then the nearest
training sample in compressed coordinates) with the FP64 oracle.

The oracle and the device use the same Y, T (from an oracle fit) and the same
stored query values.  Indices must match except where the oracle's two best
distances are equal to a relative 1e-10 (then either is correct and the
device's distance must equal the oracle's distance to its choice).
Every case prints its name and sizes before touching the GPU.
"""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_fit import to_device

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def check(name, Y, T, labels, Vs, Vv, dtype, pad_t=0):
    import torch
    import paper_1503_05947_amd as rbd
    m, d = Y.shape
    n, k = T.shape[1], Vv.shape[1]
    print(f"[gpu] classify {name} m={m} d={d} n={n} k={k} dtype={dtype}", flush=True)
    Yd = _dev(Y)
    if pad_t:
        Tbig = torch.zeros((d, n + pad_t), dtype=torch.float64)
        Tbig[:, :n] = torch.from_numpy(T)
        Td = Tbig.to("cuda:0")[:, :n]
    else:
        Td = _dev(T)
    Ld = None if labels is None else _dev(labels.astype(np.int32))
    Vd = to_device(Vs, dtype)
    res = rbd.classify(Yd, Td, Vd, labels=Ld)
    idx = res.index.cpu().numpy()
    lab = res.label.cpu().numpy()
    d2 = res.dist2.cpu().numpy()
    C = res.C.cpu().numpy()
    ridx, rlab, rd2, rC = oracle.rbd_classify(Y, T, labels if labels is not None else np.arange(n), Vv)
    scale = np.maximum(np.linalg.norm(Vv, axis=0), 1e-300)
    assert np.max(np.abs(C - rC) / scale) <= 1e-12, "C = Y'V differs"
    D = None
    for q in np.flatnonzero(idx != ridx):
        if D is None:
            diff = T[:, None, :] - rC[:, :, None]     # d x k x n
            D = np.einsum("dkn,dkn->kn", diff, diff)
        row = D[q]
        best = row.min()
        second = np.partition(row, 1)[1] if n > 1 else np.inf
        assert second - best <= 1e-10 * max(best, 1e-300), f"query {q}: index {idx[q]} vs {ridx[q]}"
        assert abs(row[idx[q]] - best) <= 1e-10 * max(best, 1e-300)
    assert np.array_equal(lab, (labels[idx] if labels is not None else idx).astype(np.int32))
    same = idx == ridx
    tol = 1e-9 * rd2 + 1e-10 * np.sqrt(rd2) * scale + 1e-300
    assert np.all(np.abs(d2 - rd2)[same] <= tol[same]), "distances differ"
    return idx, ridx


@pytest.fixture(scope="module")
def views():
    vc = synth.view_classes(0)
    Xtr, ytr, Xte, yte = vc.split()
    fit = oracle.rbd_fit(synth.quantize(Xtr, "f32")[1], 1e-3, 40, rel=True)
    return Xtr, ytr, Xte, yte, fit


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_view_classes(views, dtype):
    Xtr, ytr, Xte, yte, fit = views
    Vs, Vv = synth.quantize(Xte, dtype)
    idx, ridx = check("views", fit.Y, fit.T, ytr, Vs, Vv, dtype)
    acc = (ytr[idx] == yte).mean()
    assert acc > 0.9, acc


def test_training_columns_find_themselves(views):
    Xtr, ytr, _, _, fit = views
    Vs, Vv = synth.quantize(Xtr, "f32")
    idx, _ = check("own", fit.Y, fit.T, ytr, Vs, Vv, "f32")
    assert np.array_equal(idx, np.arange(Xtr.shape[1]))


@pytest.mark.parametrize("m,d,n,k", [(50, 1, 1, 1), (300, 7, 17, 257), (1000, 64, 16, 33), (777, 130, 33, 1000),
                                     (200000, 16, 40, 8)])
def test_ragged_shapes(m, d, n, k):
    g = synth.rng(91, m + d + n + k, 0)
    Y = np.linalg.qr(g.standard_normal((m, d)))[0]
    T = g.standard_normal((d, n))
    V = g.standard_normal((m, k))
    Vs, Vv = synth.quantize(V, "f32")
    labels = g.integers(0, 5, n).astype(np.int32)
    check("ragged", Y, T, labels, Vs, Vv, "f32", pad_t=3)


def test_without_labels_reports_indices():
    g = synth.rng(92, 0, 0)
    Y = np.linalg.qr(g.standard_normal((400, 10)))[0]
    T = g.standard_normal((10, 50))
    V = g.standard_normal((400, 70))
    idx, _ = check("no labels", Y, T, None, V, V, "f64")


def test_duplicate_training_columns_tie_to_lowest_index():
    g = synth.rng(93, 0, 0)
    Y = np.linalg.qr(g.standard_normal((128, 6)))[0]
    base = g.standard_normal((6, 5))
    T = np.concatenate([base, base, base], axis=1)        # columns j, j + 5, j + 10 identical
    V = Y @ base[:, [3, 1, 4]]
    idx, _ = check("ties", Y, T, np.arange(15).astype(np.int32), V, V, "f64")
    assert idx.tolist() == [3, 1, 4]


def test_many_queries_sampled(views):
    """100k generated queries; sampled queries checked against the oracle one by one."""
    import torch
    import paper_1503_05947_amd as rbd
    Xtr, ytr, _, _, fit = views
    vc = synth.view_classes(0)
    k = 100_000
    print(f"[gpu] classify many queries k={k}", flush=True)
    lab_q = torch.arange(k, dtype=torch.int32, device="cuda:0") % len(vc.counts)
    V = torch.empty((vc.m, k), dtype=torch.float32, device="cuda:0")
    vc.fill_queries(V, lab_q, coeff_seed=5)
    res = rbd.classify(_dev(fit.Y), _dev(fit.T), V, labels=_dev(ytr.astype(np.int32)))
    acc = (res.label == lab_q).double().mean().item()
    assert acc > 0.9, acc
    sample = np.linspace(0, k - 1, 64).astype(int)
    Vs = V[:, torch.from_numpy(sample).to("cuda:0")].cpu().numpy().astype(np.float64)
    ridx, rlab, rd2, _ = oracle.rbd_classify(fit.Y, fit.T, ytr, Vs)
    idx = res.index.cpu().numpy()[sample]
    assert np.mean(idx == ridx) >= 63 / 64
    assert np.allclose(res.dist2.cpu().numpy()[sample][idx == ridx], rd2[idx == ridx], rtol=1e-9)


def test_argument_validation():
    import torch
    import paper_1503_05947_amd as rbd
    print("[gpu] classify argument checks", flush=True)
    Y = torch.zeros((10, 3), dtype=torch.float64, device="cuda:0")
    T = torch.zeros((3, 4), dtype=torch.float64, device="cuda:0")
    V = torch.zeros((10, 2), dtype=torch.float32, device="cuda:0")
    with pytest.raises(TypeError):
        rbd.classify(Y.float(), T, V)
    with pytest.raises(ValueError):
        rbd.classify(Y, T[:2], V)
    with pytest.raises(ValueError):
        rbd.classify(Y, T, V, labels=torch.zeros(4, dtype=torch.int64, device="cuda:0"))
