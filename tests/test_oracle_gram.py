"""Pins for the Gram-route oracle ``oracle.rbd_fit_gram`` (Algorithm 1 with A = I
through G = X'X and eq. (3)), on the CPU.

  * agreement with the definitional oracle ``rbd_fit`` (itself pinned against
    LAPACK, brute force and the paper's values) on reduced parametric fields,
    bump fields and low-rank inputs, on the prefix whose errors G still resolves;
  * LAPACK's column-pivoted QR (dgeqp3): same pivots and |R_kk| = E_{k-1};
  * with the pivots fixed, T(:, pivots)' is the Cholesky factor of the pivoted
    Gram matrix (numpy's Cholesky);
  * brute force on tiny inputs; ``gram`` over row blocks equals X'X;
  * planted mistakes in the row formula and in eq. (3) are caught.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth


def valid_prefix(ref, floor=1e-5, gap=1e-6):
    """Steps whose error is above floor * E_0 and whose top two errors are separated."""
    E0 = ref.err_hist[0]
    for k in range(ref.d):
        if ref.err_hist[k] < floor * E0 or ref.gap_hist[k] <= gap:
            return k
    return ref.d


def gram_vs_definition(X, d_max, tol=0.0, rel=False):
    X = np.asarray(X, dtype=np.float64)
    o1 = oracle.rbd_fit(X, tol, d_max, rel=rel)
    o2 = oracle.rbd_fit_gram(oracle.gram([X]), tol, d_max, X.shape[0], rel=rel)
    k = min(valid_prefix(o1), o2.d)
    E0 = o1.err_hist[0]
    nx = np.linalg.norm(X, axis=0)
    fails = []
    if not np.array_equal(o1.pivots[:k], o2.pivots[:k]):
        fails.append("pivots")
    elif k:
        if np.max(np.abs(o1.err_hist[:k + 1] - o2.err_hist[:k + 1])) > 1e-8 * E0:
            fails.append("err_hist")
        if np.max(np.linalg.norm(o1.T[:k] - o2.T[:k], axis=0) / nx) > 1e-7:
            fails.append("T")
        if np.max(np.abs(o2.nu[:k] - o1.err_hist[:k])) > 1e-8 * E0:
            fails.append("nu != E_{k-1}")
    return fails, k, o1, o2


@pytest.mark.parametrize("grid,n,dmax", [(24, 160, 80), (48, 300, 120), (64, 1024, 160)])
def test_matches_definition_on_parametric_fields(grid, n, dmax):
    pf = synth.parametric_field(0, grid=grid, n=n)
    for dt in ("f32", "bf16"):
        X = synth.quantize(pf.full(), dt)[1]
        fails, k, o1, o2 = gram_vs_definition(X, dmax)
        assert fails == [], (dt, fails)
        assert k >= 20, (dt, k)


def test_matches_definition_on_bump_field_and_lowrank():
    w = synth.bump_field(0, m=512, n=400)
    fails, k, _, _ = gram_vs_definition(synth.quantize(w.X, "f32")[1], 100, w.tol, rel=True)
    assert fails == [] and k >= 10
    w = synth.lowrank_spectrum(0)
    fails, k, o1, o2 = gram_vs_definition(w.X, w.d_max, w.tol)
    assert fails == [] and k >= 15


def test_qrcp_pivots_and_diagonal():
    X = synth.lowrank_spectrum(1).X
    o2 = oracle.rbd_fit_gram(X.T @ X, 0.0, 20, X.shape[0])
    Q, R, P = sla.qr(X, pivoting=True, mode="economic")
    assert np.array_equal(P[:20], o2.pivots)
    E0 = o2.err_hist[0]
    assert np.max(np.abs(np.abs(np.diag(R))[:20] - o2.err_hist[:20])) < 1e-9 * E0


def test_cholesky_of_pivoted_gram():
    X = synth.rng(89, 0, 0).standard_normal((200, 40))
    G = X.T @ X
    o2 = oracle.rbd_fit_gram(G, 0.0, 40, 200)
    assert o2.d == 40
    P = o2.pivots
    L = np.linalg.cholesky(G[np.ix_(P, P)])
    assert np.max(np.abs(L - o2.T[:, P].T)) < 1e-10 * np.sqrt(G.diagonal().max())


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_tiny(seed):
    X = synth.rng(88, seed, 0).standard_normal((7, 6))
    o2 = oracle.rbd_fit_gram(X.T @ X, 0.0, 5, 7)
    piv, errs = oracle.rbd_brute(X, 5)
    assert np.array_equal(piv, o2.pivots)
    assert np.max(np.abs(errs - o2.err_hist)) < 1e-12 * errs[0]


def test_gram_over_row_blocks():
    X = synth.rng(88, 9, 0).standard_normal((1000, 30))
    G = oracle.gram(X[i:i + 128] for i in range(0, 1000, 128))
    assert np.max(np.abs(G - X.T @ X)) < 1e-12 * np.abs(X.T @ X).max()


def test_stop_rules():
    X = synth.random_rank(3, 80, 40, 3)
    o2 = oracle.rbd_fit_gram(X.T @ X, 1e-6, 20, 80, rel=True)
    assert o2.d == 3 and o2.stop == "tol"
    o2 = oracle.rbd_fit_gram(np.zeros((5, 5)), 0.0, 3, 9)
    assert o2.d == 0 and o2.stop == "break"
    o2 = oracle.rbd_fit_gram(X.T @ X, 0.0, 20, 80, start=11)
    assert o2.pivots[0] == 11


MUTANTS = {
    "row_sign": ("gram_row", lambda G_p, c_p, T_prev, nu: (G_p + c_p @ T_prev) / nu),
    "row_drops_last": ("gram_row", lambda G_p, c_p, T_prev, nu: (G_p - c_p[:-1] @ T_prev[:-1]) / nu
                       if len(c_p) else G_p / nu),
    "err_misses_last_row": ("gram_err2", lambda diag, T: diag - np.einsum("kj,kj->j", T[:-1], T[:-1])),
    "err_not_squared": ("gram_err2", lambda diag, T: diag - np.sum(np.abs(T), axis=0)),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_planted_mistake_is_caught(mutant, monkeypatch):
    pf = synth.parametric_field(0, grid=24, n=160)
    X = synth.quantize(pf.full(), "f32")[1]
    assert gram_vs_definition(X, 60)[0] == []
    attr, fn = MUTANTS[mutant]
    monkeypatch.setattr(oracle, attr, fn)
    try:
        fails = gram_vs_definition(X, 60)[0]
    except Exception:
        fails = ["raised"]
    assert fails, f"planted mistake {mutant} passed"
