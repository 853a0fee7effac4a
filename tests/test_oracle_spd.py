"""Pins for the oracle with a general symmetric positive definite A-norm
(section 3.2, "general SPD matrix", and eq. (3))."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth


def _csr(indptr, indices, data, m):
    return sp.csr_matrix((data, indices, indptr), shape=(m, m))


def test_diagonal_A_matches_the_weights_path():
    X = synth.bump_field(0, m=180, n=120).X
    w = synth.random_weights(4, 180)
    a = oracle.rbd_fit(X, 0.0, 25, weights=w)
    b = oracle.rbd_fit(X, 0.0, 25, A=sp.diags(w).tocsr())
    assert np.array_equal(a.pivots, b.pivots)
    assert np.max(np.abs(a.err_hist - b.err_hist)) < 1e-12 * a.err_hist[0]


def test_identity_A_matches_the_plain_fit():
    X = synth.quantize(synth.lowrank_spectrum(0).X, "f32")[1]
    a = oracle.rbd_fit(X, 1e-8, 64)
    b = oracle.rbd_fit(X, 1e-8, 64, A=sp.identity(X.shape[0], format="csr"))
    assert a.d == b.d and np.array_equal(a.pivots, b.pivots)
    assert np.max(np.abs(a.err_hist - b.err_hist)) < 1e-14


@pytest.mark.parametrize("seed", range(5))
def test_brute_force_through_the_cholesky_factor(seed):
    """||r||_A = ||L' r|| with A = L L' (an independent route to the A-norm);
    pivots are the greedy choice under it."""
    g = synth.rng(95, seed, 0)
    m, n = 9, 7
    X = g.standard_normal((m, n))
    B = g.standard_normal((m, m))
    A = B @ B.T + 0.5 * np.eye(m)
    L = np.linalg.cholesky(A)
    fit = oracle.rbd_fit(X, 0.0, 6, A=A)
    piv = []
    nxt = int(np.argmax(np.linalg.norm(L.T @ X, axis=0)))
    for _ in range(fit.d):
        piv.append(nxt)
        Q = np.linalg.qr(X[:, piv])[0]
        R = X - Q @ (Q.T @ X)
        e = np.linalg.norm(L.T @ R, axis=0)
        e[piv] = 0.0
        nxt = int(np.flatnonzero(e == e.max())[0])
    assert fit.pivots.tolist() == piv
    Rf = X - fit.Y @ fit.T
    ef = np.linalg.norm(L.T @ Rf, axis=0)
    ef[fit.pivots] = 0.0
    assert np.max(np.abs(ef - fit.col_err)) < 1e-12 * max(1.0, ef.max())


def test_eq3_matches_the_definition_for_a_laplacian_norm():
    ip, ix, v = synth.grid_laplacian_spd(12, 10, 3.0)
    A = _csr(ip, ix, v, 120)
    g = synth.rng(96, 0, 0)
    X = g.standard_normal((120, 30))
    fit = oracle.rbd_fit(X, 0.0, 12, A=A)
    for j in range(30):
        r = X[:, j] - fit.Y @ fit.T[:, j]
        direct = float(r @ (A @ r))
        assert abs(oracle.eq3_error(X[:, j], fit.Y, fit.T[:, j], A=A) - direct) < 1e-9 * max(1.0, direct)
        want = 0.0 if j in fit.pivots else np.sqrt(direct)
        assert abs(fit.col_err[j] - want) < 1e-12 * max(1.0, want)


def test_laplacian_generator_is_spd_and_symmetric():
    ip, ix, v = synth.grid_laplacian_spd(7, 5, 2.0)
    A = _csr(ip, ix, v, 35).toarray()
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0.99
    assert np.allclose(A.sum(axis=1), 1.0)          # I + c L: rows of L sum to zero
    assert np.all(np.diff(ip) >= 3) and np.all(np.diff(ip) <= 5)


def test_bad_A_rejected():
    with pytest.raises(ValueError):
        oracle.rbd_fit(np.ones((4, 3)), 0.0, 2, A=np.eye(5))
