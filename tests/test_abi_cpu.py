"""CPU-side checks of the C-ABI library: it loads without a GPU, exports every
function include/rbd.h declares, sizes workspaces, and rejects bad arguments
before any device call.  Also checks the separation between the product
package and the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbd.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1503_05947_amd import _build, _lib
    if not os.path.exists(_lib.LIB_PATH):
        _build.build_library()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rbd_fit", "rbd_fit_workspace_size", "rbd_project", "rbd_project_workspace_size",
                 "rbd_status_string"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1503_05947_amd import _lib
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def test_version_and_status_strings(lib):
    assert lib.rbd_version().decode().startswith("rbd-gfx950")
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.rbd_status_string(code)
    assert lib.rbd_status_string(123) == b"unknown status"


def test_workspace_size_queries(lib):
    from paper_1503_05947_amd import _lib
    small = _lib.fit_workspace_size(512, 256, 64, _lib.RBD_F32)
    big = _lib.fit_workspace_size(1 << 20, 4096, 512, _lib.RBD_F32)
    assert 0 < small < big < (1 << 30)
    assert _lib.fit_workspace_size(512, 256, 64, _lib.RBD_BF16) > 0
    assert _lib.project_workspace_size(1000, 20, 7, _lib.RBD_F64) > 0
    out = ctypes.c_size_t(0)
    assert lib.rbd_fit_workspace_size(0, 10, 5, 0, ctypes.byref(out)) == _lib.RBD_EINVAL
    assert lib.rbd_fit_workspace_size(10, 10, 0, 0, ctypes.byref(out)) == _lib.RBD_EINVAL
    assert lib.rbd_fit_workspace_size(10, 10, 5, 9, ctypes.byref(out)) == _lib.RBD_EINVAL
    assert lib.rbd_fit_workspace_size(5000, 5000, 2000, 0, ctypes.byref(out)) == _lib.RBD_EINVAL
    assert lib.rbd_fit_workspace_size(10, 10, 5, 0, None) == _lib.RBD_EINVAL


def test_fit_argument_validation_without_device(lib):
    from paper_1503_05947_amd import _lib
    fake = ctypes.c_void_p(4096)           # never dereferenced: validation fails first
    ws = ctypes.c_void_p(1 << 20)

    def call(**kw):
        a = dict(X=fake, xt=0, m=10, n=10, ldx=10, tol=0.0, mode=0, d_max=5, start=-1, Y=fake, T=fake,
                 piv=fake, ce=fake, eh=fake, dout=fake, st=fake, sr=None, ws=ws, wsb=0, stream=None)
        a.update(kw)
        return lib.rbd_fit(a["X"], a["xt"], a["m"], a["n"], a["ldx"], a["tol"], a["mode"], a["d_max"],
                           a["start"], a["Y"], a["T"], a["piv"], a["ce"], a["eh"], a["dout"], a["st"], a["sr"],
                           a["ws"], a["wsb"], a["stream"])

    assert call(X=None) == _lib.RBD_EINVAL
    assert call(ldx=9) == _lib.RBD_EINVAL
    assert call(tol=-1.0) == _lib.RBD_EINVAL
    assert call(tol=float("nan")) == _lib.RBD_EINVAL
    assert call(tol=float("inf")) == _lib.RBD_EINVAL
    assert call(mode=5) == _lib.RBD_EINVAL
    assert call(start=10) == _lib.RBD_EINVAL
    assert call(d_max=0) == _lib.RBD_EINVAL
    assert call(ws=ctypes.c_void_p((1 << 20) + 8)) == _lib.RBD_EINVAL     # misaligned workspace
    assert call(wsb=16) == _lib.RBD_EWORKSPACE


def test_project_argument_validation_without_device(lib):
    from paper_1503_05947_amd import _lib
    fake = ctypes.c_void_p(4096)
    rc = lib.rbd_project(fake, 3, 10, 5, fake, 0, 4, 4, fake, fake, ctypes.c_void_p(1 << 20), 1 << 30, None)
    assert rc == _lib.RBD_EINVAL     # ldy < d
    rc = lib.rbd_project(fake, 5, 10, 5, fake, 0, 4, 4, fake, fake, ctypes.c_void_p(1 << 20), 8, None)
    assert rc == _lib.RBD_EWORKSPACE
    rc = lib.rbd_project(fake, 5, 10, 0, fake, 0, 4, 4, fake, fake, ctypes.c_void_p(1 << 20), 1 << 30, None)
    assert rc == _lib.RBD_EINVAL


def test_product_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1503_05947_amd")
    for dirpath, _dirs, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text, f"{f} mentions the oracle"
                assert "import synth" not in text and "from synth" not in text, f


def test_oracle_shares_no_code_with_the_product():
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith(".py"):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1503_05947_amd" not in text


def test_missing_library_fails_loudly(tmp_path):
    from paper_1503_05947_amd import _lib
    with pytest.raises(_lib.LibraryMissing):
        _lib._lib_saved = _lib._lib
        try:
            _lib._lib = None
            _lib.load(str(tmp_path / "nope.so"))
        finally:
            _lib._lib = _lib._lib_saved


def test_batch_plan_offsets_and_order(lib):
    import numpy as np
    from paper_1503_05947_amd import _lib
    ms = np.array([5, 300, 40, 7], dtype=np.int64)
    ns = np.array([9, 20, 40, 1], dtype=np.int64)
    desc = np.zeros((4, 8), dtype=np.int64)
    order = np.zeros(4, dtype=np.int32)
    sizes = _lib.BatchSizes()
    import ctypes
    rc = lib.rbd_batch_plan(ms.ctypes.data, ns.ctypes.data, 4, 16, desc.ctypes.data, order.ctypes.data,
                            ctypes.byref(sizes))
    assert rc == _lib.RBD_OK
    D = np.minimum(16, np.minimum(ms, ns))
    assert desc[:, 0].tolist() == ms.tolist() and desc[:, 1].tolist() == ns.tolist()
    assert desc[:, 7].tolist() == D.tolist()
    assert desc[:, 2].tolist() == [0, 45, 45 + 6000, 45 + 6000 + 1600]              # X offsets
    assert desc[:, 3].tolist() == [0, 5 * 16, 305 * 16, 345 * 16]                  # Y offsets
    assert desc[:, 4].tolist() == [0, 16 * 9, 16 * 29, 16 * 69]                    # T offsets
    assert sizes.x_elems == 45 + 6000 + 1600 + 7 and sizes.max_m == 300 and sizes.max_n == 40
    cost = ms * ns * D
    assert order.tolist() == sorted(range(4), key=lambda b: -cost[b])
    assert sizes.workspace_bytes >= 256 + 8 * int((D * ms + 2 * ns).sum())
    bad = np.array([5000, 3], dtype=np.int64)
    assert lib.rbd_batch_plan(bad.ctypes.data, bad.ctypes.data, 2, 16, desc.ctypes.data, order.ctypes.data,
                              ctypes.byref(sizes)) == _lib.RBD_EINVAL
    assert lib.rbd_batch_plan(ms.ctypes.data, ns.ctypes.data, 4, 300, desc.ctypes.data, order.ctypes.data,
                              ctypes.byref(sizes)) == _lib.RBD_EINVAL


def test_weighted_fit_rejects_missing_weights(lib):
    from paper_1503_05947_amd import _lib
    fake = ctypes.c_void_p(4096)
    rc = lib.rbd_fit_weighted(fake, 0, 10, 10, 10, None, 0.0, 0, 5, -1, fake, fake, fake, fake, fake, fake, fake,
                              None, ctypes.c_void_p(1 << 20), 1 << 30, None)
    assert rc == _lib.RBD_EINVAL
    rc = lib.rbd_fit_weighted(fake, 0, 10, 10, 9, fake, 0.0, 0, 5, -1, fake, fake, fake, fake, fake, fake, fake,
                              None, ctypes.c_void_p(1 << 20), 1 << 30, None)
    assert rc == _lib.RBD_EINVAL      # ldx < n


def test_fit_graph_rejects_the_null_stream(lib):
    from paper_1503_05947_amd import _lib
    fake = ctypes.c_void_p(4096)
    h = ctypes.c_void_p()
    rc = lib.rbd_fit_graph_create(fake, 0, 16, 8, 8, None, 0.0, 0, 4, -1, fake, fake, fake, fake, fake, fake, fake,
                                  None, ctypes.c_void_p(1 << 20), 1 << 30, None, ctypes.byref(h))
    assert rc == _lib.RBD_EINVAL
    assert lib.rbd_fit_graph_launch(None, None) == _lib.RBD_EINVAL
    assert lib.rbd_fit_graph_destroy(None) == _lib.RBD_OK


def test_noalloc_rejects_before_any_device_call(lib):
    """rbd_fit_noalloc: argument errors and sizes beyond its fixed scratch are
    reported before the device is touched (this container has no GPU)."""
    from paper_1503_05947_amd import _lib
    fake = ctypes.c_void_p(4096)

    def call(m, n, d_max, X=fake, ldx=None):
        return lib.rbd_fit_noalloc(X, 0, m, n, n if ldx is None else ldx, 0.0, 0, d_max, -1, fake, fake, fake,
                                   fake, fake, fake, fake, None, None)

    assert call(1 << 20, 4096, 512) == _lib.RBD_ETOOLARGE
    assert _lib.fit_workspace_size(1 << 20, 4096, 512, _lib.RBD_F32) > _lib.RBD_NOALLOC_MAX_BYTES
    assert _lib.fit_workspace_size(2048, 2048, 256, _lib.RBD_F32) <= _lib.RBD_NOALLOC_MAX_BYTES
    assert call(100, 100, 10, X=None) == _lib.RBD_EINVAL
    assert call(100, 100, 10, ldx=99) == _lib.RBD_EINVAL
    assert call(0, 100, 10) == _lib.RBD_EINVAL
    assert lib.rbd_status_string(_lib.RBD_ETOOLARGE)


@pytest.mark.parametrize("loop", ["0", "1"])
def test_workspace_queries_over_many_shapes(lib, loop, monkeypatch):
    """Every size query over shapes from tiny to the largest accepted, with the
    persistent loop's plan on and off: the host's plan arithmetic (run under the
    sanitizers by test_host_sanitized.py)."""
    from paper_1503_05947_amd import _lib
    monkeypatch.setenv("RBD_LOOP", loop)
    out = ctypes.c_size_t(0)
    shapes = [(1, 1, 1), (1, 7, 3), (9, 1, 4), (33, 17, 5), (512, 256, 64), (2048, 2048, 256), (1111, 777, 1024),
              (70000, 40, 40), (262144, 1024, 256), (300, 250000, 24), (1 << 20, 4096, 512), (2000000, 8, 8),
              (1 << 22, 64, 64)]
    for m, n, dm in shapes:
        for dt in (_lib.RBD_F32, _lib.RBD_BF16, _lib.RBD_F16, _lib.RBD_F64):
            assert lib.rbd_fit_workspace_size(m, n, dm, dt, ctypes.byref(out)) == _lib.RBD_OK, (m, n, dm, dt)
            assert out.value > 0
            assert lib.rbd_fit_spd_workspace_size(m, n, dm, dt, ctypes.byref(out)) == _lib.RBD_OK
            d = min(dm, m, n, _lib.RBD_MAX_D)
            assert lib.rbd_project_workspace_size(m, d, n, dt, ctypes.byref(out)) == _lib.RBD_OK
        d = min(dm, m, n, _lib.RBD_MAX_D)
        assert lib.rbd_classify_workspace_size(m, d, n, ctypes.byref(out)) == _lib.RBD_OK
        if d <= min(m, n):
            assert lib.rbd_reconstruct_backward_workspace_size(m, n, d, ctypes.byref(out)) == _lib.RBD_OK


def test_fit_basis_queries_and_validation_without_device(lib, monkeypatch):
    from paper_1503_05947_amd import _lib
    monkeypatch.setenv("RBD_LOOP", "0")      # the FP32-basis plan never holds the persistent loop's buffers
    out = ctypes.c_size_t(0)
    for m, n, d in ((512, 256, 64), (1111, 777, 60), (1 << 20, 4096, 512)):
        s64 = _lib.fit_workspace_size(m, n, d, _lib.RBD_BF16, _lib.RBD_BASIS_F64)
        assert s64 == _lib.fit_workspace_size(m, n, d, _lib.RBD_BF16)
        s32 = _lib.fit_workspace_size(m, n, d, _lib.RBD_BF16, _lib.RBD_BASIS_F32)
        assert s32 >= s64 + 4 * m * d - 4096      # room for the FP32 basis (plan alignment aside)
    assert lib.rbd_fit_basis_workspace_size(10, 10, 5, 0, 2, ctypes.byref(out)) == _lib.RBD_EINVAL
    assert lib.rbd_fit_basis_workspace_size(10, 10, 5, 0, -1, ctypes.byref(out)) == _lib.RBD_EINVAL
    fake = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)

    def call(basis, wsb=1 << 30, **kw):
        a = dict(X=fake, xt=0, m=10, n=10, ldx=10, tol=0.0, mode=0, d_max=5, start=-1)
        a.update(kw)
        return lib.rbd_fit_basis(a["X"], a["xt"], a["m"], a["n"], a["ldx"], a["tol"], a["mode"], a["d_max"],
                                 a["start"], basis, fake, fake, fake, fake, fake, fake, fake, None, ws, wsb, None)

    assert call(2) == _lib.RBD_EINVAL
    assert call(_lib.RBD_BASIS_F32, X=None) == _lib.RBD_EINVAL
    assert call(_lib.RBD_BASIS_F32, ldx=9) == _lib.RBD_EINVAL
    assert call(_lib.RBD_BASIS_F32, wsb=16) == _lib.RBD_EWORKSPACE


def test_binding_rejects_bad_basis_choices():
    import paper_1503_05947_amd as rbd
    with pytest.raises(ValueError):
        rbd.basis_code("f16")
    with pytest.raises(ValueError):
        import torch
        rbd.FitBuffers(16, 16, 4, torch.float32, "cpu", spd=True, workspace=False, basis="f32")
