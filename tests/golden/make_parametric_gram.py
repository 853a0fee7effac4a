"""Writes tests/golden/parametric_1048576x4096_gram.json: the Gram-route oracle
(Algorithm 1 with A = I through G = X'X and eq. (3), ``oracle.rbd_fit_gram``)
on the full-size parametric field, 1,048,576 x 4096, as stored in FP32 and in
BF16, tol 0, d_max 512.

The stored values are regenerated on the host in row blocks exactly as the
device holds them (``synth.ParametricField.rows`` then ``synth.quantize``), and
G is accumulated in FP64.  G squares the condition number, so only the steps
whose largest error is at least 1e-6 of E_0 are written, with the first 128
rows of T on 32 sampled columns and the pivot columns (the tests compare
those above 1e-5 of E_0, where the route agrees with the definitional oracle
to about 1e-9 E_0 on reduced grids).

Run from the repository root:  python tests/golden/make_parametric_gram.py
(about ten minutes on eight cores; calls only ``oracle`` and ``synth``).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "parametric_1048576x4096_gram.json")
DTYPES = ("f32", "bf16")
D_MAX = 512
KEEP_FLOOR = 1e-6          # rows of the result written: E_k >= KEEP_FLOOR * E_0
SAMPLE_COLS = 32
T_ROWS = 128             # rows of T written, on the sampled and the pivot columns
BLOCK = 16384


def main():
    pf = synth.parametric_field(seed=0)
    A, B = pf.factors()
    G = {dt: np.zeros((pf.n, pf.n)) for dt in DTYPES}
    t0 = time.time()
    for r0 in range(0, pf.m, BLOCK):
        rows = pf.rows(np.arange(r0, min(pf.m, r0 + BLOCK)), A, B)
        for dt in DTYPES:
            vals = synth.quantize(rows, dt)[1]
            G[dt] += vals.T @ vals
        if r0 // BLOCK % 8 == 0:
            print(f"rows {r0 + BLOCK} / {pf.m}  {time.time() - t0:.0f} s", flush=True)
    out = dict(
        what="Gram-route oracle on the parametric field x_j(s) = sum_k exp(-mu_jk |s - c_k|^2), 1024^2 grid, "
             "n = 4096, seed 0, tol 0, d_max 512, per storage type",
        citation="Algorithm 1 (section 3.1) with A = I; rows of T and errors through eq. (3) from G = X'X",
        command="python tests/golden/make_parametric_gram.py",
        m=pf.m, n=pf.n, d_max=D_MAX, keep_floor=KEEP_FLOOR, results={})
    J = np.linspace(0, pf.n - 1, SAMPLE_COLS).round().astype(int)
    for dt in DTYPES:
        fit = oracle.rbd_fit_gram(G[dt], 0.0, D_MAX, pf.m)
        E0 = float(fit.err_hist[0])
        K = next((k for k in range(fit.d) if fit.err_hist[k] < KEEP_FLOOR * E0), fit.d)
        Kt = min(K, T_ROWS)
        cols = np.unique(np.concatenate([J, fit.pivots[:Kt]]))
        out["results"][dt] = dict(
            E0=E0, steps=int(K), stop_of_full_run=fit.stop, d_of_full_run=int(fit.d),
            pivots=fit.pivots[:K].tolist(),
            err_hist=fit.err_hist[:K + 1].tolist(),
            gap_hist=[float(g) if np.isfinite(g) else None for g in fit.gap_hist[:K + 1]],
            nu=fit.nu[:K].tolist(),
            T_cols=cols.tolist(),
            T_rows=int(Kt),
            T=fit.T[:Kt][:, cols].tolist(),
            col_norm=np.sqrt(np.diag(G[dt])[cols]).tolist())
        print(f"{dt}: E0 = {E0:.6e}, {K} steps above {KEEP_FLOOR:g} E0", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
