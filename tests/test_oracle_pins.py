"""Pins for the FP64 oracle: each check is tied to something other than the oracle
itself (a textbook routine, brute force, a closed form, a theorem, or a value the
paper prints), so that a slip anywhere in the oracle fails at least one of them.

Pins (section / equation of the paper each one follows from):
  P1  Y has orthonormal columns (step 2.2 normalises after Gram-Schmidt)
  P2  A = I with greedy start is QR with column pivoting (LAPACK dgeqp3):
      same pivots, |R_kk| = E_{k-1}, Y = Q diag(sign R_kk)   (steps 2.2-2.3, eq. (3))
  P3  col_err_j = ||x_j - Y T(:, j)||                        (step 2.3 by definition)
  P4  T = Y'X and sum_k T_kj^2 + e_j^2 = ||x_j||^2           (eq. (3) with A = I)
  P5  T(:, pivots) is upper triangular with diagonal E_{k-1} (step 2.2 + 2.3)
  P6  error history non-increasing, pivots distinct          (greedy on nested spaces)
  P7  exact recovery at rank r; Table 3 intrinsic dimensions (section 4.2.1)
  P8  pivots equal those of a brute-force greedy              (step 2.3 by definition)
  P9  Eckart-Young lower bounds                               (SVD optimality)
  P10 section 4.2.2 example: d = 22, pointwise error < 1e-6, ratio > 110
  P11 out-of-sample: v in span(Y) has zero error; v = x_j reproduces T(:, j)
  P12 edge cases of the control flow of Algorithm 1
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth

# ----------------------------------------------------------------------------
# pin checks shared by the plain tests and the planted-mistake tests
# ----------------------------------------------------------------------------


def qrcp_failures(X, fit, gap=1e-9):
    """P2: compare with LAPACK's column-pivoted QR on the well-separated prefix."""
    fails = []
    Q, R, P = sla.qr(X, pivoting=True, mode="economic")
    d = fit.d
    # prefix on which the oracle's top two errors are separated
    k_ok = d
    for k in range(d):
        if fit.gap_hist[k] <= gap:
            k_ok = k
            break
    if not np.array_equal(P[:k_ok], fit.pivots[:k_ok]):
        fails.append("P2 pivots differ from dgeqp3")
        return fails
    rkk = np.abs(np.diag(R))[:k_ok]
    E0 = fit.err_hist[0]
    if k_ok and np.max(np.abs(rkk - fit.err_hist[:k_ok])) > 1e-10 * E0:
        fails.append("P2 |R_kk| != E_{k-1}")
    s = np.sign(np.diag(R)[:k_ok])
    if k_ok and np.max(np.abs(Q[:, :k_ok] * s - fit.Y[:, :k_ok])) > 1e-7:
        fails.append("P2 Y != Q diag(sign R)")
    return fails


def invariant_failures(X, fit):
    fails = []
    d = fit.d
    E0 = fit.err_hist[0]
    nx = np.linalg.norm(X, axis=0)
    if d:
        if np.max(np.abs(fit.Y.T @ fit.Y - np.eye(d))) > 1e-13:
            fails.append("P1 Y not orthonormal")
        if np.max(np.abs(fit.T - fit.Y.T @ X)) > 1e-12 * max(E0, 1e-300):
            fails.append("P4 T != Y'X")
    true_err = np.linalg.norm(X - fit.Y @ fit.T, axis=0)
    true_err[fit.pivots] = 0.0
    if np.max(np.abs(true_err - fit.col_err)) > 1e-12 * max(E0, 1e-300):
        fails.append("P3 col_err != ||x_j - Y T_j||")
    energy = np.sum(fit.T ** 2, axis=0) + fit.col_err ** 2
    mask = np.ones(X.shape[1], bool)
    mask[fit.pivots] = False
    if mask.any() and np.max(np.abs(energy[mask] - nx[mask] ** 2)) > 1e-10 * E0 ** 2:
        fails.append("P4 energy identity violated")
    if d:
        B = fit.T[:, fit.pivots]
        if np.max(np.abs(np.tril(B, -1))) > 1e-12 * E0:
            fails.append("P5 T(:, pivots) not upper triangular")
        if np.max(np.abs(np.diag(B) - fit.err_hist[:d])) > 1e-12 * E0:
            fails.append("P5 diag T(:, pivots) != E_{k-1}")
    if np.any(np.diff(fit.err_hist) > 1e-12 * E0):
        fails.append("P6 error history increases")
    if len(set(fit.pivots.tolist())) != d:
        fails.append("P6 repeated pivot")
    if d and np.any(fit.col_err[fit.pivots] != 0.0):
        fails.append("R3 pivot error not exactly 0")
    return fails


def brute_failures(X, fit):
    piv, errs = oracle.rbd_brute(X, fit.d)
    fails = []
    if not np.array_equal(piv, fit.pivots):
        fails.append("P8 pivots differ from brute force")
    elif np.max(np.abs(errs - fit.err_hist)) > 1e-12 * max(errs[0], 1e-300):
        fails.append("P8 errors differ from brute force")
    return fails


def all_failures(X, fit, brute=False):
    f = invariant_failures(X, fit) + qrcp_failures(X, fit)
    if brute:
        f += brute_failures(X, fit)
    return f


# ----------------------------------------------------------------------------
# inputs
# ----------------------------------------------------------------------------


def small_inputs():
    yield "lowrank_f64", synth.quantize(synth.lowrank_spectrum(0).X, "f64")[1], 1e-8, False, 64
    yield "lowrank_f32", synth.quantize(synth.lowrank_spectrum(1).X, "f32")[1], 1e-8, False, 64
    yield "lowrank_bf16", synth.quantize(synth.lowrank_spectrum(2).X, "bf16")[1], 1e-8, False, 64
    yield "bumps_256", synth.quantize(synth.bump_field(0, m=256, n=192).X, "f32")[1], 1e-4, True, 96
    pf = synth.parametric_field(0, grid=24, n=160)
    yield "param_24", pf.full(), 1e-9, True, 80


@pytest.mark.parametrize("name,X,tol,rel,dmax", list(small_inputs()), ids=lambda v: v if isinstance(v, str) else "")
def test_pins_hold(name, X, tol, rel, dmax):
    fit = oracle.rbd_fit(X, tol, dmax, rel=rel)
    assert fit.d >= 1
    assert all_failures(X, fit) == []


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("shape", [(6, 5), (8, 8), (5, 9), (12, 7)])
def test_brute_force_tiny(seed, shape):
    X = synth.rng(99, seed, 0).standard_normal(shape)
    fit = oracle.rbd_fit(X, 0.0, min(shape))
    assert brute_failures(X, fit) == []
    assert invariant_failures(X, fit) == []


def test_qrcp_on_config_scale_inputs():
    """P2 on the 512 x 256 low-rank workload in all storage precisions."""
    w = synth.lowrank_spectrum(0)
    for dt in ("f64", "f32", "bf16", "f16"):
        X = synth.quantize(w.X, dt)[1]
        fit = oracle.rbd_fit(X, w.tol, w.d_max)
        assert qrcp_failures(X, fit) == [], dt


# ----------------------------------------------------------------------------
# exact recovery, Table 3 and the section 4.2.2 example
# ----------------------------------------------------------------------------


@pytest.mark.parametrize("r", [1, 3, 7, 20])
def test_exact_recovery_random_rank(r):
    X = synth.random_rank(r, 300, 120, r)
    fit = oracle.rbd_fit(X, 1e-10, 60, rel=True)
    assert fit.d == r and fit.stop == "tol"
    assert fit.err_hist[-1] < 1e-13 * fit.err_hist[0]


def test_table3_intrinsic_dimension(golden):
    dims = golden["table3"]["intrinsic_dimension"]
    for which, want in zip((1, 2, 3), dims):
        X = synth.table3(which, 512)
        fit = oracle.rbd_fit(X, 1e-10, 20, rel=True)
        assert fit.d == want and fit.stop == "tol"
        assert np.max(np.abs(X - fit.Y @ fit.T)) < 1e-12


@pytest.mark.slow
def test_approx_field_example(golden):
    g = golden["approx_field"]
    X = synth.approx_field(g["grid"])
    fit = oracle.rbd_fit(X, 0.0, g["d"])
    assert fit.d == g["d"]
    assert np.max(np.abs(X - fit.Y @ fit.T)) < g["max_pointwise_error_below"]
    m, n = X.shape
    assert m * n / (fit.d * (m + n)) > g["compression_ratio_above"]


def test_eckart_young_bounds():
    for X in (synth.quantize(synth.lowrank_spectrum(3).X, "f32")[1],
              synth.bump_field(1, m=200, n=150).X):
        s = np.linalg.svd(X, compute_uv=False)
        fit = oracle.rbd_fit(X, 0.0, 30)
        Rm = X - fit.Y @ fit.T
        d = fit.d
        assert np.sum(Rm ** 2) >= np.sum(s[d:] ** 2) * (1 - 1e-10)
        assert np.linalg.norm(Rm, 2) >= s[d] * (1 - 1e-10)
        # and the greedy indicator bounds the spectral error from above: ||R||_2 <= sqrt(n) E_d
        assert np.linalg.norm(Rm, 2) <= np.sqrt(X.shape[1]) * fit.err_hist[-1] * (1 + 1e-10)


# ----------------------------------------------------------------------------
# out-of-sample compression
# ----------------------------------------------------------------------------


def test_project_closed_forms():
    w = synth.lowrank_spectrum(4)
    X = w.X
    fit = oracle.rbd_fit(X, w.tol, w.d_max)
    coef = synth.rng(98, 0, 0).standard_normal((fit.d, 5))
    V_in = fit.Y @ coef
    C, err = oracle.rbd_project(fit.Y, V_in)
    assert np.max(np.abs(C - coef)) < 1e-12
    assert np.max(err) < 1e-13
    C2, err2 = oracle.rbd_project(fit.Y, X[:, :17])
    assert np.max(np.abs(C2 - fit.T[:, :17])) < 1e-14
    m = np.ones(17, bool)
    m[np.isin(np.arange(17), fit.pivots)] = False
    assert np.max(np.abs(err2[m] - fit.col_err[:17][m])) < 1e-14
    # orthogonal complement: error equals the full norm, coefficients vanish
    z = synth.rng(98, 1, 0).standard_normal(X.shape[0])
    z -= fit.Y @ (fit.Y.T @ z)
    z -= fit.Y @ (fit.Y.T @ z)
    C3, err3 = oracle.rbd_project(fit.Y, z[:, None])
    assert np.max(np.abs(C3)) < 1e-13 and abs(err3[0] - np.linalg.norm(z)) < 1e-13


# ----------------------------------------------------------------------------
# control flow of Algorithm 1 (edge cases)
# ----------------------------------------------------------------------------


def test_zero_matrix_gives_empty_basis():
    fit = oracle.rbd_fit(np.zeros((7, 5)), 0.0, 4)
    assert fit.d == 0 and fit.stop == "break" and fit.err_hist.tolist() == [0.0]


def test_tolerance_above_largest_norm_breaks_at_once():
    X = synth.rng(97, 0, 0).standard_normal((30, 20))
    E0 = np.linalg.norm(X, axis=0).max()
    fit = oracle.rbd_fit(X, E0 * 1.001, 10)
    assert fit.d == 0 and fit.stop == "break"
    # tol == E0: ||v|| < eps_R is false, one vector is taken and the max error then is <= eps_R
    fit = oracle.rbd_fit(X, E0, 10)
    assert fit.d == 1 and fit.stop == "tol"


def test_duplicate_columns_and_ties():
    g = synth.rng(97, 1, 0)
    X = g.standard_normal((20, 8))
    X[:, 5] = X[:, 2] = X[:, 2] * 10.0        # tie for the largest norm at 2 and 5
    fit = oracle.rbd_fit(X, 1e-12, 8)
    assert fit.pivots[0] == 2                 # lowest index wins the tie
    assert 5 not in fit.pivots.tolist()       # its duplicate has zero error afterwards
    assert fit.d == 7


def test_dmax_clamped_and_full_rank():
    X = synth.rng(97, 2, 0).standard_normal((9, 14))
    fit = oracle.rbd_fit(X, 0.0, 50)
    assert fit.d == 9
    assert np.max(np.abs(X - fit.Y @ fit.T)) < 1e-12
    X = synth.rng(97, 3, 0).standard_normal((14, 9))
    fit = oracle.rbd_fit(X, 0.0, 50)
    assert fit.d == 9 and fit.stop in ("dmax", "tol")


def test_single_row_and_column():
    fit = oracle.rbd_fit(np.array([[3.0, -4.0, 1.0]]), 0.0, 3)
    assert fit.d == 1 and fit.pivots.tolist() == [1] and abs(fit.T[0, 1] - 4.0) < 1e-15
    fit = oracle.rbd_fit(np.array([[3.0], [4.0]]), 0.0, 3)
    assert fit.d == 1 and abs(fit.err_hist[0] - 5.0) < 1e-15 and fit.err_hist[1] == 0.0


def test_user_start_column():
    X = synth.rng(97, 4, 0).standard_normal((25, 12))
    fit = oracle.rbd_fit(X, 0.0, 5, start=7)
    assert fit.pivots[0] == 7
    assert np.max(np.abs(fit.Y[:, 0] - X[:, 7] / np.linalg.norm(X[:, 7]))) < 1e-15


def test_nonfinite_rejected():
    X = np.ones((4, 4))
    X[1, 2] = np.nan
    with pytest.raises(FloatingPointError):
        oracle.rbd_fit(X, 0.0, 2)


def test_storage_rounding_changes_stop():
    """The oracle must run on the stored values: FP32 rounding changes the fit."""
    w = synth.lowrank_spectrum(0)
    f64 = oracle.rbd_fit(synth.quantize(w.X, "f64")[1], w.tol, w.d_max)
    bf = oracle.rbd_fit(synth.quantize(w.X, "bf16")[1], w.tol, w.d_max)
    assert bf.d > f64.d     # BF16 rounding noise (~1e-3 relative) is far above tol


# ----------------------------------------------------------------------------
# planted mistakes: every one must be caught by some pin
# ----------------------------------------------------------------------------


def _square_case():
    return synth.quantize(synth.bump_field(3, m=48, n=48, noise=1e-6).X, "f64")[1]


def _tie_case():
    X = synth.rng(96, 0, 0).standard_normal((10, 7))
    X[:, 4] = X[:, 1] = X[:, 1] * 5.0
    return X


MUTANTS = {
    "transposed_T_row": ("project_row", lambda xi, X: X @ xi),
    "residual_sign": ("residual_update", lambda R, xi, t: R.__iadd__(np.outer(xi, t))),
    "dropped_last_gs_term": ("mgs_twice", lambda v, Y, d: _mgs_drop_last(v, Y, d)),
    "squared_norms": ("_colnorms", lambda R: np.einsum("ij,ij->j", R, R)),
    "highest_index_tie": ("_lowest_argmax", lambda e: int(len(e) - 1 - np.argmax(e[::-1]))),
}


def _mgs_drop_last(v, Y, d):
    v = v.copy()
    for _ in range(2):
        for k in range(d - 1):
            v -= (Y[:, k] @ v) * Y[:, k]
    return v


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_planted_mistake_is_caught(mutant, monkeypatch):
    attr, fn = MUTANTS[mutant]
    cases = [_square_case(), _tie_case()]
    # the genuine oracle passes every pin on these cases
    for X in cases:
        fit = oracle.rbd_fit(X, 0.0, min(X.shape) - 1)
        assert all_failures(X, fit, brute=True) == []
    monkeypatch.setattr(oracle, attr, fn)
    caught = False
    for X in cases:
        try:
            fit = oracle.rbd_fit(X, 0.0, min(X.shape) - 1)
        except Exception:
            caught = True
            continue
        if all_failures(X, fit, brute=True):
            caught = True
    assert caught, f"planted mistake {mutant} passed every pin"
