"""Pins for the oracle with a diagonal A-norm (section 3.2, eq. (3))."""
import numpy as np
import pytest

import oracle
import synth


def test_unit_weights_reduce_to_identity():
    X = synth.quantize(synth.lowrank_spectrum(0).X, "f32")[1]
    a = oracle.rbd_fit(X, 1e-8, 64)
    b = oracle.rbd_fit(X, 1e-8, 64, weights=np.ones(X.shape[0]))
    assert a.d == b.d and np.array_equal(a.pivots, b.pivots)
    assert np.max(np.abs(a.err_hist - b.err_hist)) == 0.0


def test_constant_weights_scale_errors():
    X = synth.bump_field(0, m=200, n=150).X
    a = oracle.rbd_fit(X, 0.0, 30)
    b = oracle.rbd_fit(X, 0.0, 30, weights=np.full(200, 9.0))
    assert np.array_equal(a.pivots, b.pivots)
    assert np.max(np.abs(3.0 * a.err_hist - b.err_hist)) < 1e-12 * b.err_hist[0]


def test_eq3_matches_the_definition():
    g = synth.rng(80, 0, 0)
    X = g.standard_normal((60, 30))
    w = g.uniform(0.1, 5.0, 60)
    fit = oracle.rbd_fit(X, 0.0, 10, weights=w)
    for j in range(30):
        direct = float(w @ (X[:, j] - fit.Y @ fit.T[:, j]) ** 2)
        assert abs(oracle.eq3_error(X[:, j], fit.Y, fit.T[:, j], w) - direct) < 1e-10 * max(1.0, direct)
        want = 0.0 if j in fit.pivots else np.sqrt(direct)
        assert abs(fit.col_err[j] - want) < 1e-12 * max(1.0, want)


@pytest.mark.parametrize("seed", range(6))
def test_weighted_brute_force(seed):
    """Each step picks the column of largest A-norm projection error (brute force)."""
    g = synth.rng(81, seed, 0)
    X = g.standard_normal((9, 7))
    w = g.uniform(0.05, 3.0, 9)
    fit = oracle.rbd_fit(X, 0.0, 6, weights=w)
    piv = []
    nxt = int(np.argmax([np.sqrt(w @ X[:, j] ** 2) for j in range(7)]))
    for _ in range(fit.d):
        piv.append(nxt)
        Q, _r = np.linalg.qr(X[:, piv])
        e = [0.0 if j in piv else float(np.sqrt(w @ (X[:, j] - Q @ (Q.T @ X[:, j])) ** 2)) for j in range(7)]
        nxt = min(j for j in range(7) if e[j] == max(e))
    assert fit.pivots.tolist() == piv


def test_weights_change_the_greedy_choice():
    """Weight on the rows where column 3 lives makes it the first pick."""
    X = np.zeros((6, 4))
    X[:, 0] = [3, 3, 0, 0, 0, 0]
    X[:, 3] = [0, 0, 0, 0, 1, 1]
    X[:, 1] = [1, 0, 1, 0, 0, 0]
    X[:, 2] = [0, 1, 0, 1, 0, 0]
    assert oracle.rbd_fit(X, 0.0, 2).pivots[0] == 0
    w = np.array([1, 1, 1, 1, 100, 100.0])
    assert oracle.rbd_fit(X, 0.0, 2, weights=w).pivots[0] == 3


def test_bad_weights_rejected():
    X = np.ones((4, 3))
    with pytest.raises(ValueError):
        oracle.rbd_fit(X, 0.0, 2, weights=np.array([1.0, 0.0, 1.0, 1.0]))
