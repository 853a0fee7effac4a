"""Reconstruction Y T and its backward (pivots fixed) vs the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype="f64"):
    import torch
    if dtype == "bf16":
        return torch.from_numpy(a.view(np.int16)).view(torch.bfloat16).cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("m,d,n", [(300, 37, 211), (1, 1, 1), (129, 128, 130), (64, 5, 4000)])
def test_reconstruct_gemm(m, d, n):
    import paper_1503_05947_amd as rbd
    print(f"[gpu] reconstruct {m}x{d} @ {d}x{n}", flush=True)
    g = synth.rng(70, m, d)
    Y = g.standard_normal((m, d))
    T = g.standard_normal((d, n))
    Z = rbd.reconstruct(dev(Y), dev(T)).cpu().numpy()
    assert np.max(np.abs(Z - Y @ T)) <= 1e-12 * np.sqrt(d) * max(1.0, np.abs(Y @ T).max())


@pytest.mark.parametrize("xdt,gdt", [("f64", "f64"), ("f32", "f64"), ("f32", "f32"), ("bf16", "f64")])
def test_backward_matches_oracle(xdt, gdt):
    import paper_1503_05947_amd as rbd
    print(f"[gpu] backward X={xdt} G={gdt}", flush=True)
    w = synth.bump_field(7, m=700, n=333)
    Xs, Xv = synth.quantize(w.X, xdt)
    res = rbd.fit(dev(Xs, xdt), tol=0.0, d_max=40)
    P = res.pivots.cpu().numpy()
    G = synth.cotangent(0, 700, 333)
    if gdt == "f32":
        G = G.astype(np.float32)
    grad = rbd.reconstruct_backward(dev(Xs, xdt), dev(G), res.Y, res.T, res.pivots).cpu().numpy()
    ref = oracle.reconstruction_grad(Xv, P, G.astype(np.float64))
    scale = np.abs(ref).max()
    assert np.max(np.abs(grad - ref)) <= 1e-9 * scale


@pytest.mark.parametrize("m,n,d", [(1111, 777, 200), (517, 300, 128), (333, 129, 129), (2000, 3, 3)])
def test_backward_ragged_shapes_and_both_inverses(m, n, d):
    """Shapes off the 128 x 128 tiles, d on both sides of the LDS inverse's limit
    (128), pivots reaching the last columns: the pivot columns are added inside
    the tiles of dX that hold them."""
    import paper_1503_05947_amd as rbd
    print(f"[gpu] backward ragged m={m} n={n} d={d}", flush=True)
    w = synth.bump_field(9, m=m, n=n, noise=1e-2)
    Xs, Xv = synth.quantize(w.X, "f32")
    res = rbd.fit(dev(Xs, "f32"), tol=0.0, d_max=d)
    assert res.d == d
    P = res.pivots.cpu().numpy()
    G = synth.cotangent(3, m, n)
    grad = rbd.reconstruct_backward(dev(Xs, "f32"), dev(G), res.Y, res.T, res.pivots).cpu().numpy()
    ref = oracle.reconstruction_grad(Xv, P, G)
    assert np.max(np.abs(grad - ref)) <= 1e-9 * np.abs(ref).max()


def test_backward_finite_differences_on_device_gradient():
    import paper_1503_05947_amd as rbd
    print("[gpu] backward vs central differences", flush=True)
    g = synth.rng(71, 0, 0)
    X = g.standard_normal((90, 60))
    res = rbd.fit(dev(X), tol=0.0, d_max=12)
    P = res.pivots.cpu().numpy()
    G = g.standard_normal((90, 60))
    grad = rbd.reconstruct_backward(dev(X), dev(G), res.Y, res.T, res.pivots).cpu().numpy()
    for t in range(4):
        D = g.standard_normal(X.shape)
        if t == 0:
            D[:, np.setdiff1d(np.arange(60), P)] = 0.0
        h = 1e-6
        fd = (oracle.reconstruction_loss(X + h * D, P, G) - oracle.reconstruction_loss(X - h * D, P, G)) / (2 * h)
        assert abs(fd - np.sum(grad * D)) <= 1e-6 * max(1.0, abs(fd))


def test_full_basis_backward_is_the_cotangent():
    import paper_1503_05947_amd as rbd
    print("[gpu] backward d = n", flush=True)
    g = synth.rng(72, 0, 0)
    X = g.standard_normal((50, 16))
    G = g.standard_normal((50, 16))
    res = rbd.fit(dev(X), tol=0.0, d_max=16)
    assert res.d == 16
    grad = rbd.reconstruct_backward(dev(X), dev(G), res.Y, res.T, res.pivots).cpu().numpy()
    assert np.max(np.abs(grad - G)) < 1e-11


def test_autograd_function():
    import torch

    import paper_1503_05947_amd as rbd
    print("[gpu] autograd", flush=True)
    w = synth.bump_field(8, m=200, n=120)
    X = dev(w.X).requires_grad_(True)
    Z = rbd.rbd_reconstruction(X, tol=0.0, d_max=20)
    G = torch.from_numpy(synth.cotangent(1, 200, 120)).cuda()
    (gx,) = torch.autograd.grad((Z * G).sum(), X)
    res = rbd.fit(X.detach(), tol=0.0, d_max=20)
    ref = oracle.reconstruction_grad(w.X, res.pivots.cpu().numpy(), G.cpu().numpy())
    assert np.max(np.abs(gx.cpu().numpy() - ref)) <= 1e-9 * np.abs(ref).max()
    assert np.max(np.abs(Z.detach().cpu().numpy() - res.Y.cpu().numpy() @ res.T.cpu().numpy())) < 1e-10


def test_backward_full_size():
    """65536 x 2048 FP32 bump field, d = 128 pivots fixed from a tol-0 fit, G ~ N(0,1)."""
    import paper_1503_05947_amd as rbd
    print("[gpu] backward 65536 x 2048, d = 128", flush=True)
    w = synth.bump_field(0, m=65536, n=2048, d_max=128)
    Xs, Xv = synth.quantize(w.X, "f32")
    del w
    Xd = dev(Xs, "f32")
    res = rbd.fit(Xd, tol=0.0, d_max=128)
    assert res.d == 128
    G = synth.cotangent(0, 65536, 2048)
    grad = rbd.reconstruct_backward(Xd, dev(G), res.Y, res.T, res.pivots).cpu().numpy()
    ref = oracle.reconstruction_grad(Xv, res.pivots.cpu().numpy(), G)
    err = np.max(np.abs(grad - ref)) / np.abs(ref).max()
    print(f"[gpu] backward full size: max |grad - ref| / max |ref| = {err:.3e}", flush=True)
    assert err <= 1e-8
