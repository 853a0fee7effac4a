"""Pins for the classification oracle: out-of-sample compression c = Y'v
(section 3.1) and the nearest training sample in compressed coordinates."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
import synth


@pytest.fixture(scope="module")
def small():
    vc = synth.view_classes(1, classes=6, rows=24, cols=20, lo=12, hi=16, bumps=6)
    Xtr, ytr, Xte, yte = vc.split(train_per_class=5)
    fit = oracle.rbd_fit(Xtr, 1e-6, 25, rel=True)
    return Xtr, ytr, Xte, yte, fit


def test_nearest_matches_cdist(small):
    """Brute force with an independent distance routine on the coordinates."""
    Xtr, ytr, Xte, yte, fit = small
    idx, lab, d2, C = oracle.rbd_classify(fit.Y, fit.T, ytr, Xte)
    D = cdist(C.T, fit.T.T, "sqeuclidean")
    for q in range(Xte.shape[1]):
        row = D[q]
        best = row.min()
        # the oracle's choice attains the minimum (up to rounding of the two routines)
        assert abs(row[idx[q]] - best) <= 1e-12 * max(1.0, best)
        assert abs(d2[q] - row[idx[q]]) <= 1e-12 * max(1.0, best)
        second = np.partition(row, 1)[1]
        if second - best > 1e-9 * max(1.0, best):
            assert idx[q] == int(np.argmin(row))
    assert np.array_equal(lab, ytr[idx])


def test_training_column_is_its_own_neighbour(small):
    Xtr, ytr, _, _, fit = small
    idx, lab, d2, _ = oracle.rbd_classify(fit.Y, fit.T, ytr, Xtr)
    assert np.array_equal(idx, np.arange(Xtr.shape[1]))
    assert np.max(d2) < 1e-20 * np.max(np.sum(Xtr * Xtr, axis=0))


def test_isometry_in_the_span():
    """If every query minus every training column lies in span(Y), distances in
    coordinates equal the distances in R^m, so the neighbour is the full-space one."""
    g = synth.rng(90, 0, 0)
    m, r = 300, 12
    B = np.linalg.qr(g.standard_normal((m, r)))[0]
    Xtr = B @ g.standard_normal((r, 40))
    Xq = B @ g.standard_normal((r, 25))
    fit = oracle.rbd_fit(Xtr, 1e-12, 40, rel=True)
    assert fit.d == r
    idx, _, d2, _ = oracle.rbd_classify(fit.Y, fit.T, np.arange(40), Xq)
    full = cdist(Xq.T, Xtr.T, "sqeuclidean")
    assert np.array_equal(idx, np.argmin(full, axis=1))
    assert np.allclose(d2, full.min(axis=1), rtol=1e-10, atol=1e-12)


def test_ties_go_to_the_lowest_index():
    Y = np.eye(3)[:, :2]
    T = np.array([[1.0, 0.0, 1.0, 0.0], [0.0, 1.0, 0.0, 1.0]])     # columns 0 == 2, 1 == 3
    V = np.array([[1.0, 0.0], [0.0, 1.0], [5.0, 5.0]])             # third row is outside span(Y)
    idx, lab, d2, C = oracle.rbd_classify(Y, T, np.array([7, 8, 9, 10]), V)
    assert idx.tolist() == [0, 1] and lab.tolist() == [7, 8]
    assert np.allclose(C, [[1.0, 0.0], [0.0, 1.0]]) and np.all(d2 == 0.0)
    # a query halfway between two distinct training points
    idx, _, _, _ = oracle.rbd_classify(Y, T[:, :2], np.array([0, 1]), np.array([[0.5], [0.5], [0.0]]))
    assert idx.tolist() == [0]


def test_separated_classes_are_recognised():
    vc = synth.view_classes(2, classes=8, rows=30, cols=24, lo=14, hi=20, bumps=8, pose=0.05, noise=0.001)
    Xtr, ytr, Xte, yte = vc.split(train_per_class=6)
    fit = oracle.rbd_fit(Xtr, 1e-4, 30, rel=True)
    _, lab, _, _ = oracle.rbd_classify(fit.Y, fit.T, ytr, Xte)
    assert (lab == yte).mean() == 1.0


# ---------------------------------------------------------------------------
# planted mistakes: each must fail at least one pin
# ---------------------------------------------------------------------------

def _pin_failures(classify):
    vc = synth.view_classes(1, classes=6, rows=24, cols=20, lo=12, hi=16, bumps=6)
    Xtr, ytr, Xte, yte = vc.split(train_per_class=5)
    fit = oracle.rbd_fit(Xtr, 1e-6, 25, rel=True)
    fails = []
    idx, lab, d2, C = classify(fit.Y, fit.T, ytr, Xte)
    D = cdist((fit.Y.T @ Xte).T, fit.T.T, "sqeuclidean")
    if not np.allclose(D[np.arange(len(idx)), idx], D.min(axis=1), rtol=1e-12, atol=1e-14):
        fails.append("not the nearest")
    if not np.allclose(d2, D.min(axis=1), rtol=1e-10, atol=1e-14):
        fails.append("distance")
    if not np.array_equal(lab, ytr[idx]):
        fails.append("labels")
    Y = np.eye(3)[:, :2]
    T = np.array([[1.0, 0.0, 1.0, 0.0], [0.0, 1.0, 0.0, 1.0]])
    idx, _, _, _ = classify(Y, T, np.arange(4), np.array([[1.0, 0.0], [0.0, 1.0], [5.0, 5.0]]))
    if idx.tolist() != [0, 1]:
        fails.append("ties")
    return fails


def _mutant_argmax(Y, T, labels, V):
    C = Y.T @ V
    d2 = cdist(C.T, T.T, "sqeuclidean")
    idx = np.argmax(d2, axis=1)
    return idx, np.asarray(labels)[idx], d2[np.arange(len(idx)), idx], C


def _mutant_last_tie(Y, T, labels, V):
    C = Y.T @ V
    d2 = cdist(C.T, T.T, "sqeuclidean")
    idx = d2.shape[1] - 1 - np.argmin(d2[:, ::-1], axis=1)
    return idx, np.asarray(labels)[idx], d2[np.arange(len(idx)), idx], C


def _mutant_unsquared(Y, T, labels, V):
    C = Y.T @ V
    d = np.stack([np.sum(T - C[:, q:q + 1], axis=0) for q in range(C.shape[1])])
    idx = np.argmin(np.abs(d), axis=1)
    return idx, np.asarray(labels)[idx], np.abs(d[np.arange(len(idx)), idx]), C


def _mutant_label_shift(Y, T, labels, V):
    C = Y.T @ V
    idx, lab, d2, _ = oracle.rbd_classify(Y, T, labels, V)
    return idx, np.asarray(labels)[np.minimum(idx + 1, len(labels) - 1)], d2, C


def test_genuine_oracle_passes_the_pins():
    assert _pin_failures(oracle.rbd_classify) == []


@pytest.mark.parametrize("mutant", [_mutant_argmax, _mutant_last_tie, _mutant_unsquared, _mutant_label_shift])
def test_planted_mistake_is_caught(mutant):
    assert _pin_failures(mutant) != [], mutant.__name__
