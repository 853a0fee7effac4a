"""Pins for the oracle's gradient of the reconstruction (pivots fixed): central
finite differences of the loss by its definition, and exact special cases."""
import numpy as np
import pytest

import oracle
import synth


def _case(seed, m=40, n=25, d=8):
    g = synth.rng(60, seed, 0)
    X = g.standard_normal((m, n))
    fit = oracle.rbd_fit(X, 0.0, d)
    G = g.standard_normal((m, n))
    return X, fit.pivots, G


@pytest.mark.parametrize("seed", range(4))
def test_gradient_matches_central_differences(seed):
    X, P, G = _case(seed)
    grad = oracle.reconstruction_grad(X, P, G)
    g = synth.rng(61, seed, 0)
    for trial in range(6):
        D = g.standard_normal(X.shape)
        if trial == 0:
            D[:, np.setdiff1d(np.arange(X.shape[1]), P)] = 0.0    # pivot columns only
        if trial == 1:
            D[:, P] = 0.0                                           # non-pivot columns only
        h = 1e-6
        fd = (oracle.reconstruction_loss(X + h * D, P, G) - oracle.reconstruction_loss(X - h * D, P, G)) / (2 * h)
        an = float(np.sum(grad * D))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (trial, fd, an)


def test_full_basis_gradient_is_the_cotangent():
    """d = n: Y Y' X = X, so dL/dX = G exactly."""
    g = synth.rng(62, 0, 0)
    X = g.standard_normal((30, 12))
    G = g.standard_normal((30, 12))
    fit = oracle.rbd_fit(X, 0.0, 12)
    assert fit.d == 12
    grad = oracle.reconstruction_grad(X, fit.pivots, G)
    assert np.max(np.abs(grad - G)) < 1e-12


def test_non_pivot_columns_see_only_the_projection():
    """Columns outside the pivots do not move Y: their gradient is (Y Y' G)(:, j)."""
    X, P, G = _case(5)
    Y, _ = oracle.basis_from_pivots(X, P)
    grad = oracle.reconstruction_grad(X, P, G)
    rest = np.setdiff1d(np.arange(X.shape[1]), P)
    assert np.max(np.abs(grad[:, rest] - (Y @ (Y.T @ G))[:, rest])) < 1e-12


def test_homogeneity():
    """L(cX) = c L(X) (Y is scale invariant), so <dL/dX, X> = L."""
    X, P, G = _case(6)
    grad = oracle.reconstruction_grad(X, P, G)
    assert abs(np.sum(grad * X) - oracle.reconstruction_loss(X, P, G)) < 1e-10 * max(1, abs(np.sum(grad * X)))


def test_basis_matches_the_fit():
    X, P, G = _case(7)
    fit = oracle.rbd_fit(X, 0.0, len(P))
    Y, R = oracle.basis_from_pivots(X, P)
    assert np.max(np.abs(Y - fit.Y)) < 1e-12
    assert np.max(np.abs(R - fit.T[:, P])) < 1e-12


def test_planted_sign_error_in_the_adjoint_is_caught(monkeypatch):
    X, P, G = _case(8)
    good = oracle.reconstruction_grad(X, P, G)
    D = synth.rng(63, 0, 0).standard_normal(X.shape)
    D[:, np.setdiff1d(np.arange(X.shape[1]), P)] = 0.0
    h = 1e-6
    fd = (oracle.reconstruction_loss(X + h * D, P, G) - oracle.reconstruction_loss(X - h * D, P, G)) / (2 * h)
    assert abs(fd - np.sum(good * D)) < 1e-6 * abs(fd)
    real_tril = np.tril
    monkeypatch.setattr(np, "tril", lambda a, k=0: -real_tril(a, k))   # copyltu with the wrong sign
    bad = oracle.reconstruction_grad(X, P, G)
    monkeypatch.setattr(np, "tril", real_tril)
    assert abs(fd - np.sum(bad * D)) > 1e-4 * abs(fd)
