"""FP64 CPU oracle for Reduced Basis Decomposition (test infrastructure only).

This package is the independent reference the device path is checked
against.  It is test infrastructure: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and the
two share no code (the only shared module is ``synth``, which holds input
generators and storage rounding, none of the method's arithmetic).

Contents
--------
``rbd_fit``      Algorithm 1 of the paper (section 3.1), step by step, in FP64:
                 explicit residual, errors evaluated by their definition in
                 step 2.3 (no downdating), Gram-Schmidt done twice.
``rbd_fit_gram`` Algorithm 1 with A = I carried out on the Gram matrix
                 G = X'X alone (for inputs too large to hold in FP64 on the
                 host): the new row of T and every error follow from G by
                 eq. (3); the steps are those of ``rbd_fit``.
``gram``         G = X'X accumulated in FP64 from row blocks of X.
``rbd_brute``    Brute-force greedy for tiny inputs: every step re-derives each
                 column's projection error from a fresh QR of the chosen
                 columns (section 3.1, step 2.3 by definition).
``rbd_project``  Out-of-sample compression v_C = Y' v (section 3.1, the
                 compression of out-of-sample data) with the A = I error
                 of eq. (3) evaluated as the norm of the explicit residual.
``rbd_classify`` Classification of out-of-sample data in the compressed
                 coordinates (the face recognition use of section 4): each
                 query's coordinates c = Y' v, then the training column whose
                 coordinates T(:, j) are nearest in the Euclidean norm.

Readings where the paper is silent or ambiguous (each is listed with its
reason in the design notes):
  * first column: ``start < 0`` takes the lowest index of max_j ||x_j||
    (a deterministic stand-in for the random start of step 1);
  * argmax ties go to the lowest index;
  * a column already chosen as a pivot has error exactly 0;
  * orthonormalisation is modified Gram-Schmidt applied twice;
  * the truncation in step 2.2 keeps the first d-1 *rows* of T;
  * a zero vector (norm exactly 0) also ends the loop, since it cannot be
    normalised even when the tolerance is 0;
  * relative tolerance: tau = tol * max_j ||x_j||.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class OracleFit:
    Y: np.ndarray          # (m, d) orthonormal basis
    T: np.ndarray          # (d, n) transformation, T = Y' X
    pivots: np.ndarray     # (d,) 0-based column chosen at each step
    col_err: np.ndarray    # (n,) ||x_j - Y T(:, j)||, 0 for pivots
    err_hist: np.ndarray   # (d+1,) E_0 = max_j ||x_j||, then E_k after step k
    gap_hist: np.ndarray   # (d+1,) (largest - second largest unmasked error) / E_0 before each pick
    d: int
    tau: float
    stop: str              # "tol" | "dmax" | "break"


def _colnorms(R: np.ndarray) -> np.ndarray:
    """Euclidean norm of every column, summed in FP64."""
    return np.sqrt(np.einsum("ij,ij->j", R, R))


def _lowest_argmax(e: np.ndarray) -> int:
    """Lowest index attaining the maximum (numpy's argmax returns the first one)."""
    return int(np.argmax(e))


def _gap(e: np.ndarray, E0: float) -> float:
    if e.size < 2 or E0 == 0.0:
        return np.inf
    top2 = np.partition(e, e.size - 2)[-2:]
    return float((top2[1] - top2[0]) / E0)


def project_row(xi: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Step 2.2, last line: the new row of T is xi' X."""
    return xi @ X


def residual_update(R: np.ndarray, xi: np.ndarray, t: np.ndarray) -> None:
    """R <- R - xi t', so that R = X - Y(:, 1:d) T(1:d, :) holds after step d."""
    R -= np.outer(xi, t)


def mgs_twice(v: np.ndarray, Y: np.ndarray, d: int) -> np.ndarray:
    """Step 2.2: modified Gram-Schmidt of v against xi_1..xi_{d-1}, applied twice."""
    v = v.copy()
    for _ in range(2):
        for k in range(d):
            v -= (Y[:, k] @ v) * Y[:, k]
    return v


def _anorm_cols(R: np.ndarray, w, A=None) -> np.ndarray:
    """||r_j||_A = sqrt(r_j' A r_j) (section 3.2): A = diag(w), or a general
    symmetric positive definite A (dense or scipy.sparse); both None: A = I."""
    if A is not None:
        q = np.einsum("ij,ij->j", R, np.asarray(A @ R))
        return np.sqrt(np.maximum(q, 0.0))
    if w is None:
        return _colnorms(R)
    return np.sqrt(np.einsum("i,ij,ij->j", w, R, R))


def rbd_fit(X, tol: float, d_max: int, rel: bool = False, start: int = -1, weights=None, A=None) -> OracleFit:
    """Algorithm 1, (Y, T) = RBD(X, eps_R, d_max) (section 3.1).

    ``weights`` = None uses A = I; otherwise A = diag(weights) (the "general
    diagonal" choice of section 3.2); ``A`` (dense or scipy.sparse, symmetric
    positive definite) is the "general SPD" choice.  The basis and T = Y'X are
    unchanged, and every error of step 2.3 (and E_0, and the relative
    tolerance) is the A-norm ||x_j - Y T(:, j)||_A of eq. (3), evaluated here
    by its definition on the explicit residual.

    ``X`` must already hold the stored values (e.g. FP32- or BF16-rounded data
    upcast to FP64).  Returns the first ``d`` basis vectors, rows of T, pivots,
    final per-column errors and the error history.
    """
    X = np.asarray(X, dtype=np.float64)
    if X.ndim != 2:
        raise ValueError("X must be a matrix")
    m, n = X.shape
    if m < 1 or n < 1 or d_max < 1:
        raise ValueError("empty input or d_max < 1")
    if not np.all(np.isfinite(X)):
        raise FloatingPointError("X holds a non-finite value")
    D = min(int(d_max), m, n)

    w = None if weights is None else np.asarray(weights, dtype=np.float64)
    if w is not None and (w.shape != (m,) or not np.all(w > 0) or not np.all(np.isfinite(w))):
        raise ValueError("weights must be m positive finite values")
    if A is not None and (w is not None or A.shape != (m, m)):
        raise ValueError("A must be m x m (and not combined with weights)")
    # pre-computation of diag(X'AX): the error of every column with d = 0
    e = _anorm_cols(X, w, A)
    E0 = float(e.max())
    tau = float(tol) * E0 if rel else float(tol)

    Y = np.zeros((m, D))
    T = np.zeros((D, n))
    R = X.copy()                        # residual X - Y T, kept explicitly
    chosen = np.zeros(n, dtype=bool)
    pivots = []
    err_hist = [E0]
    gap_hist = [_gap(e, E0)]

    # step 1
    i = int(start) if start >= 0 else _lowest_argmax(e)
    if not 0 <= i < n:
        raise ValueError("start column out of range")
    d = 0                               # number of accepted basis vectors (paper's d - 1)
    E_cur = np.inf
    stop = "dmax"

    # step 2: while d <= d_max and E_cur > eps_R  (paper's d is our d + 1)
    while d < D and E_cur > tau:
        v = X[:, i].copy()                              # 2.1
        v = mgs_twice(v, Y, d)                          # 2.2
        nu = float(np.sqrt(v @ v))
        if nu < tau or nu == 0.0:
            stop = "break"                              # keep d columns (paper's d - 1)
            break
        xi = v / nu
        Y[:, d] = xi
        T[d, :] = project_row(xi, X)
        residual_update(R, xi, T[d, :])
        chosen[i] = True
        pivots.append(i)
        d += 1
        # 2.3: errors by their definition, pivots masked
        e = _anorm_cols(R, w, A)
        e[chosen] = 0.0
        E_cur = float(e.max())
        gap_hist.append(_gap(e[~chosen], E0) if (~chosen).sum() >= 2 else np.inf)
        i = _lowest_argmax(e)
        err_hist.append(E_cur)
        # 2.4
        if E_cur <= tau:
            stop = "tol"
    return OracleFit(Y=Y[:, :d].copy(), T=T[:d].copy(), pivots=np.array(pivots, dtype=np.int64),
                     col_err=e, err_hist=np.array(err_hist),
                     gap_hist=np.array(gap_hist), d=d, tau=tau, stop=stop)


@dataclass
class GramFit:
    T: np.ndarray          # (d, n) rows of T = Y' X
    pivots: np.ndarray     # (d,)
    col_err: np.ndarray    # (n,) errors after the last step, 0 for pivots
    err_hist: np.ndarray   # (d+1,)
    gap_hist: np.ndarray   # (d+1,) as in OracleFit
    nu: np.ndarray         # (d,) the norm of each orthogonalised pivot column
    d: int
    tau: float
    stop: str


def gram(blocks):
    """G = X'X in FP64, summed over row blocks of X (an iterable of (rows, n) arrays)."""
    G = None
    for B in blocks:
        B = np.asarray(B, dtype=np.float64)
        P = B.T @ B
        G = P if G is None else G + P
    return G


def gram_row(G_p, c_p, T_prev, nu):
    """The new row of T from the Gram matrix: xi' x_j = (G[p, j] - c_p' T(:, j)) / nu."""
    return (G_p - c_p @ T_prev) / nu


def gram_err2(diag, T_cur):
    """eq. (3) with A = I and orthonormal Y: ||x_j - Y T(:, j)||^2 = G[j, j] - ||T(:, j)||^2."""
    return diag - np.einsum("kj,kj->j", T_cur, T_cur)


def rbd_fit_gram(G, tol: float, d_max: int, m: int, rel: bool = False, start: int = -1) -> GramFit:
    """Algorithm 1 with A = I (section 3.1) when only G = X'X is at hand.

    The basis vector of step 2.2 is xi = (x_p - Y c_p) / nu with c_p = Y' x_p =
    T(:, p), so its inner product with any column is
    xi' x_j = (G[p, j] - c_p' T(:, j)) / nu: the new row of T.  With Y
    orthonormal, eq. (3) for A = I gives every error of step 2.3 as
    e_j^2 = G[j, j] - ||T(:, j)||^2, and the norm of the orthogonalised pivot
    column is nu = e_p.  Pivots are masked, ties go to the lowest index and
    the break / stop tests are those of ``rbd_fit``.  Only the basis itself is
    not formed.  G squares the data's condition number: errors below about
    1e-7 of the largest column norm (for X with a million rows in FP64) carry
    no correct digits.
    """
    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    if G.shape != (n, n) or n < 1 or m < 1 or d_max < 1:
        raise ValueError("G must be n x n, m >= 1, d_max >= 1")
    if not np.all(np.isfinite(G)):
        raise FloatingPointError("G holds a non-finite value")
    D = min(int(d_max), m, n)
    diag = np.diag(G).copy()
    e = np.sqrt(np.maximum(diag, 0.0))
    E0 = float(e.max())
    tau = float(tol) * E0 if rel else float(tol)
    T = np.zeros((D, n))
    chosen = np.zeros(n, dtype=bool)
    pivots, nus = [], []
    err_hist = [E0]
    gap_hist = [_gap(e, E0)]
    i = int(start) if start >= 0 else _lowest_argmax(e)
    if not 0 <= i < n:
        raise ValueError("start column out of range")
    d = 0
    E_cur = np.inf
    stop = "dmax"
    while d < D and E_cur > tau:
        # 2.1-2.2: the orthogonalised pivot column, through its inner products
        c_p = T[:d, i]
        nu2 = float(diag[i] - c_p @ c_p)
        nu = float(np.sqrt(nu2)) if nu2 > 0.0 else 0.0
        if nu < tau or nu == 0.0:
            stop = "break"
            break
        T[d, :] = gram_row(G[i, :], c_p, T[:d, :], nu)
        chosen[i] = True
        pivots.append(i)
        nus.append(nu)
        d += 1
        # 2.3: eq. (3), every column from its Gram diagonal and its coefficients
        e = np.sqrt(np.maximum(gram_err2(diag, T[:d]), 0.0))
        e[chosen] = 0.0
        E_cur = float(e.max())
        gap_hist.append(_gap(e[~chosen], E0) if (~chosen).sum() >= 2 else np.inf)
        i = _lowest_argmax(e)
        err_hist.append(E_cur)
        if E_cur <= tau:
            stop = "tol"
    return GramFit(T=T[:d].copy(), pivots=np.array(pivots, dtype=np.int64), col_err=e,
                   err_hist=np.array(err_hist), gap_hist=np.array(gap_hist), nu=np.array(nus),
                   d=d, tau=tau, stop=stop)


def eq3_error(x, Y, c, weights=None, A=None):
    """eq. (3): ||v - Y c||_A^2 = v'Av - 2 c'Y'Av + c'Y'AYc for A = diag(weights)
    or a given SPD matrix A (dense or scipy.sparse)."""
    x = np.asarray(x, dtype=np.float64)
    if A is not None:
        Av = np.asarray(A @ x).ravel()
        AY = np.asarray(A @ Y)
    else:
        w = np.ones(x.shape[0]) if weights is None else np.asarray(weights, dtype=np.float64)
        Av = w * x
        AY = w[:, None] * Y
    return float(x @ Av - 2.0 * c @ (Y.T @ Av) + c @ (Y.T @ AY) @ c)


def rbd_brute(X, steps: int, start: int = -1):
    """Greedy pivots by brute force: at each step every column's projection error
    onto span(X[:, pivots]) is recomputed from a fresh QR (step 2.3 by definition).

    Returns (pivots, errors) where errors[k] is the largest error after k pivots.
    Meant for tiny X only.
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[1]

    def first_max(vals):
        top = max(vals)
        return min(j for j, val in enumerate(vals) if val == top)

    piv = []
    e = [float(np.linalg.norm(X[:, j])) for j in range(n)]
    errs = [max(e)]
    nxt = int(start) if start >= 0 else first_max(e)
    for _ in range(steps):
        piv.append(nxt)
        Q, _r = np.linalg.qr(X[:, piv])
        e = [0.0 if j in piv else float(np.linalg.norm(X[:, j] - Q @ (Q.T @ X[:, j])))
             for j in range(n)]
        errs.append(max(e))
        nxt = first_max(e)
    return np.array(piv, dtype=np.int64), np.array(errs)


def rbd_project(Y, V):
    """Out-of-sample compression c = Y' v for every column v of V (section 3.1),
    with the A = I error of eq. (3) taken as ||v - Y c|| by its definition."""
    Y = np.asarray(Y, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    C = Y.T @ V
    err = _colnorms(V - Y @ C)
    return C, err


def rbd_classify(Y, T, labels, V):
    """Nearest training sample in the compressed coordinates (section 3.1's
    out-of-sample compression used for recognition as in section 4).

    c_q = Y' v_q; dist2[q, j] = sum_k (c_q[k] - T[k, j])^2 evaluated term by
    term (no expansion into norms and a cross product); the nearest j is the
    lowest index attaining the minimum.  Returns (index, label, dist2_min, C).
    """
    Y = np.asarray(Y, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    labels = np.asarray(labels)
    C = Y.T @ V
    k = C.shape[1]
    index = np.zeros(k, dtype=np.int64)
    best = np.zeros(k)
    for q in range(k):
        diff = T - C[:, q:q + 1]
        d2 = np.sum(diff * diff, axis=0)
        j = int(np.flatnonzero(d2 == d2.min())[0])
        index[q] = j
        best[q] = d2[j]
    return index, labels[index], best, C


def reconstruct(Y, T):
    """Uncompress: X(:, j) ~ Y T(:, j) (section 3.1)."""
    return np.asarray(Y, dtype=np.float64) @ np.asarray(T, dtype=np.float64)


# ---------------------------------------------------------------------------
# differentiating the reconstruction with the pivots held fixed
# ---------------------------------------------------------------------------

def basis_from_pivots(X, pivots):
    """Y, R with X(:, pivots) = Y R, Y orthonormal, R upper triangular with a
    positive diagonal: the basis Algorithm 1 builds from these columns."""
    A = np.asarray(X, dtype=np.float64)[:, np.asarray(pivots)]
    Q, R = np.linalg.qr(A)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def reconstruction_loss(X, pivots, G):
    """L = <G, Y Y' X> with Y the basis spanned by the pivot columns of X."""
    X = np.asarray(X, dtype=np.float64)
    Y, _R = basis_from_pivots(X, pivots)
    return float(np.sum(np.asarray(G, dtype=np.float64) * (Y @ (Y.T @ X))))


def reconstruction_grad(X, pivots, G):
    """dL/dX for L = <G, Y Y' X>, pivots fixed: the direct term Y Y'G plus the
    adjoint of the QR factorisation X(:, P) = Y R with Rbar = 0,
    Abar = (Ybar + Y copyltu(-Ybar'Y)) R^{-T}, Ybar = G T' + X G'Y."""
    import scipy.linalg as sla
    X = np.asarray(X, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    P = np.asarray(pivots)
    Y, R = basis_from_pivots(X, P)
    T = Y.T @ X
    YtG = Y.T @ G
    grad = Y @ YtG
    Ybar = G @ T.T + X @ YtG.T
    M = -(Ybar.T @ Y)
    S = np.tril(M) + np.tril(M, -1).T
    Abar = sla.solve_triangular(R, (Ybar + Y @ S).T, lower=False).T      # Abar R^T = W
    grad[:, P] += Abar
    return grad
