"""Comparison of a device fit with the FP64 oracle (shared by the GPU tests and smoke).

Protocol: pivots must agree on the prefix of steps at which the oracle's two
largest errors are separated by more than ``gap`` * E_0; on that prefix the
basis vectors, rows of T, error history and final errors must agree to
``rtol`` (relative to 1 for unit vectors, to ||x_j|| for T columns, to E_0 for
errors).  d must agree unless the oracle's last error is within 1e-3 tau of
the tolerance or the prefix ended early.  Beyond the prefix, the device
result must still satisfy the invariants (orthonormal Y, T = Y'X, certified
errors) on its own.
"""
from __future__ import annotations

import numpy as np


def separated_prefix(ref, gap: float) -> int:
    for k in range(ref.d):
        if ref.gap_hist[k] <= gap:
            return k
    return ref.d


def compare_fit(dev, ref, X, rtol: float = 1e-5, gap: float = 1e-6, exact_d: bool = True, weights=None,
                norms=None):
    """dev: dict of numpy arrays (Y, T, pivots, col_err, err_hist, d); ref: OracleFit; X: stored values;
    weights: the diagonal of A when the errors are A-norms (eq. (3)), else None;
    norms: a callable giving the column A-norms of a matrix, for a general A."""
    msgs = []
    E0 = ref.err_hist[0]
    k = min(separated_prefix(ref, gap), dev["d"], ref.d)
    piv_ok = np.array_equal(dev["pivots"][:k], ref.pivots[:k])
    if not piv_ok:
        first = int(np.argmax(dev["pivots"][:k] != ref.pivots[:k]))
        msgs.append(f"pivots differ at step {first} (prefix {k}): {dev['pivots'][:k]} vs {ref.pivots[:k]}")
        return msgs
    if k:
        dy = np.max(np.abs(dev["Y"][:, :k] - ref.Y[:, :k]))
        if dy > rtol:
            msgs.append(f"Y differs by {dy:.3e}")
        nx = np.linalg.norm(X, axis=0)
        dt = np.linalg.norm(dev["T"][:k] - ref.T[:k], axis=0)
        bad = dt > rtol * np.maximum(nx, 1e-300)
        if bad.any():
            msgs.append(f"T differs in {bad.sum()} columns (worst {np.max(dt / np.maximum(nx, 1e-300)):.3e})")
        dh = np.max(np.abs(dev["err_hist"][: k + 1] - ref.err_hist[: k + 1]))
        if dh > rtol * E0:
            msgs.append(f"err_hist differs by {dh / E0:.3e} E0")
    full = (k == ref.d == dev["d"])
    if full:
        de = np.max(np.abs(dev["col_err"] - ref.col_err))
        if de > rtol * E0:
            msgs.append(f"col_err differs by {de / E0:.3e} E0")
    near_tol = ref.tau > 0 and abs(ref.err_hist[-1] - ref.tau) <= 1e-3 * ref.tau
    if exact_d and k == ref.d and dev["d"] != ref.d and not near_tol:
        msgs.append(f"d differs after a fully separated run: {dev['d']} vs {ref.d}")
    if dev["d"] == ref.d and abs(dev["err_hist"][dev["d"]] - ref.err_hist[ref.d]) > rtol * E0:
        msgs.append("final error differs: %.6e vs %.6e" % (dev["err_hist"][dev["d"]], ref.err_hist[ref.d]))
    msgs += invariant_msgs(dev, X, rtol, weights=weights, norms=norms)
    return msgs


def _norms(R, weights, norms=None):
    if norms is not None:
        return norms(R)
    if weights is None:
        return np.linalg.norm(R, axis=0)
    return np.sqrt(np.asarray(weights, dtype=np.float64) @ (R * R))


def invariant_msgs(dev, X, rtol=1e-5, weights=None, norms=None):
    """Checks a device fit on its own: orthonormal Y, T = Y'X, certified errors, monotone history
    (with A = I: a Euclidean projection residual can grow in another A-norm)."""
    msgs = []
    d = dev["d"]
    Y, T = dev["Y"][:, :d], dev["T"][:d]
    nx = np.linalg.norm(X, axis=0)
    E0 = _norms(X, weights, norms).max()
    if d:
        o = np.max(np.abs(Y.T @ Y - np.eye(d)))
        if o > 1e-12:
            msgs.append(f"Y not orthonormal ({o:.2e})")
        dt = np.max(np.abs(T - Y.T @ X))
        if dt > 1e-12 * max(nx.max(), 1e-300) * np.sqrt(X.shape[0]):
            msgs.append(f"T != Y'X ({dt:.2e})")
    true_err = _norms(X - Y @ T, weights, norms)
    if d:
        true_err[dev["pivots"][:d]] = 0.0
    de = np.max(np.abs(true_err - dev["col_err"]))
    if de > rtol * max(E0, 1e-300):
        msgs.append(f"col_err not the true residual norm ({de / max(E0, 1e-300):.2e} E0)")
    h = dev["err_hist"][: d + 1]
    if weights is None and norms is None and np.any(np.diff(h) > 1e-9 * max(E0, 1e-300)):
        msgs.append("error history increases")
    if len(set(dev["pivots"][:d].tolist())) != d:
        msgs.append("repeated pivot")
    return msgs
