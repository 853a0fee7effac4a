"""The parity protocol itself (tests/parity.py), on the CPU.

A result taken from the oracle must pass against the oracle; a valid greedy
run that resolves a near-tie the other way must pass as well; planted
mistakes in a stand-in device result (a wrong pivot, a wrong error history,
a too-good residual) must be caught.
"""
import numpy as np

import oracle
import synth
from parity import compare_fit, eckart_young_msgs, invariant_msgs


def as_dev(fit):
    return dict(Y=fit.Y.copy(), T=fit.T.copy(), pivots=fit.pivots.copy(), col_err=fit.col_err.copy(),
                err_hist=fit.err_hist.copy(), d=fit.d)


def test_oracle_passes_against_itself():
    w = synth.lowrank_spectrum(1)
    _, vals = synth.quantize(w.X, "f32")
    ref = oracle.rbd_fit(vals, w.tol, w.d_max)
    rep = compare_fit(as_dev(ref), ref, vals)
    assert rep == [], rep
    assert rep.steps_checked == ref.d and rep.worst_hist < 1e-12 and rep.worst_choice < 1e-12


def test_near_tie_resolved_the_other_way_passes():
    g = synth.rng(90, 0, 0)
    X = g.standard_normal((60, 3)) @ g.standard_normal((3, 25))
    j_max = int(np.argmax(np.linalg.norm(X, axis=0)))
    j_alt = (j_max + 7) % 25
    X[:, j_alt] = X[:, j_alt] * (np.linalg.norm(X[:, j_max]) * (1 - 1e-10) / np.linalg.norm(X[:, j_alt]))
    ref = oracle.rbd_fit(X, 0.0, 3)
    assert ref.pivots[0] == j_max
    alt = oracle.rbd_fit(X, 0.0, 3, start=j_alt)     # a valid greedy run from the other column
    rep = compare_fit(as_dev(alt), ref, X)
    assert rep == [], rep
    assert rep.prefix == 0 and rep.steps_checked == 3


def test_wrong_pivot_caught():
    w = synth.bump_field(3, m=200, n=150)
    ref = oracle.rbd_fit(w.X, 0.0, 20)
    dev = as_dev(ref)
    k = 12
    e_final = ref.col_err
    # relabel step k's pivot as an unchosen column with a small error
    cand = [j for j in np.argsort(e_final) if j not in set(ref.pivots.tolist())]
    dev["pivots"][k] = cand[0]
    rep = compare_fit(dev, ref, w.X, gap=1e-6)
    assert any("pivot" in m for m in rep), rep
    assert invariant_msgs(dev, w.X) != []


def test_wrong_history_caught():
    w = synth.bump_field(3, m=200, n=150)
    ref = oracle.rbd_fit(w.X, 0.0, 20)
    # beyond the separated prefix only the replayed errors see the mistake
    dev = as_dev(ref)
    k = 17
    dev["err_hist"][k] += 3e-5 * ref.err_hist[0]
    rep = compare_fit(dev, ref, w.X, gap=1.0)        # an empty prefix: nothing compared element by element
    assert rep.prefix == 0
    assert any(f"err_hist[{k}]" in m for m in rep), rep


def test_final_error_compared_when_d_differs():
    w = synth.lowrank_spectrum(0)
    ref = oracle.rbd_fit(w.X, w.tol, w.d_max)
    short = oracle.rbd_fit(w.X, 0.0, 10)       # a valid run that stopped early (E_10 ~ 1e-3)
    rep = compare_fit(as_dev(short), ref, w.X, exact_d=False)
    assert any("final error differs" in m for m in rep), rep


def test_eckart_young_rejects_a_too_good_residual():
    g = synth.rng(90, 1, 0)
    X = g.standard_normal((40, 30))
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    d = 5
    R_opt = X - (U[:, :d] * s[:d]) @ Vt[:d]
    assert eckart_young_msgs(X, R_opt, d) == []
    R_better = X - (U[:, :d + 1] * s[:d + 1]) @ Vt[:d + 1]          # rank d + 1 claimed as rank d
    msgs = eckart_young_msgs(X, R_better, d)
    assert len(msgs) == 2, msgs


def test_greedy_result_meets_eckart_young():
    w = synth.bump_field(2, m=300, n=200)
    ref = oracle.rbd_fit(w.X, 0.0, 40)
    R = w.X - ref.Y @ ref.T
    assert eckart_young_msgs(w.X, R, ref.d) == []
