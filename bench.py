#!/usr/bin/env python3
"""Throughput of the RBD greedy loop on one MI355X.

Workload: the parametric-field snapshot matrix x_j(s) = sum_{k<8} exp(-mu_jk
|s - c_k|^2) on a 1024 x 1024 grid (m = 1,048,576 rows) with n = 4096
parameter draws, tol = 0, d_max = 512 (every fit runs all 512 greedy steps).
One bench step is one complete rbd_fit.  X is resident in HBM before timing.

Reported: greedy steps/s for FP32 storage (``value``), the same for BF16
storage, the X-scan kernel's achieved bandwidth against the 8 TB/s HBM peak
(kernel time from HIP events recorded on the fit's stream inside the timed
region), the BF16-vs-FP32 time to reach equal error against the FP64 field,
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
EPS_BOTH = (1e-1, 3e-2, 1e-2, 5e-3)
EPS_FP32 = (1e-4, 1e-5, 1e-6)
UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8 + 2.0 ** -24, "f16": 2.0 ** -11, "f64": 2.0 ** -53}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed fits")
    ap.add_argument("--warmup", type=int, default=1, help="untimed fits")
    ap.add_argument("--grid", type=int, default=1024, help="field grid g (m = g*g)")
    ap.add_argument("--n", type=int, default=4096, help="columns (parameter draws)")
    ap.add_argument("--d-max", type=int, default=512)
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-basis32", action="store_true", help="skip the BF16 fit with the basis kept in FP32")
    ap.add_argument("--no-equal-error", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-examples", action="store_true",
                    help="skip the fits of Table 3 and the section 4.2.2 field")
    ap.add_argument("--phases", action="store_true", help="extra profiled fit with a per-phase breakdown")
    ap.add_argument("--sample-cols", type=int, default=64)
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip the batched, backward and recognition sections (all three run by default)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched fit: 4096 matrices, m, n log-uniform in [64, 1024], "
                         "spectrum 10^(-i/8), FP32, relative tol 1e-6")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batched-cache", default=None,
                    help="load the batched matrices (stored values, packed) from this .npy file, or generate them "
                         "and write it; with --write-batched-cache only write it and exit (so that a profiled run "
                         "does no host generation)")
    ap.add_argument("--write-batched-cache", action="store_true")
    ap.add_argument("--next-rows-only", action="store_true",
                    help="run only the batched, backward and recognition sections (for profiling them); the "
                         "line then carries no headline value")
    ap.add_argument("--no-backward", action="store_true",
                    help="skip the reconstruction backward: bump field 65536 x 2048 FP32, d = 128 pivots "
                         "fixed from a tol-0 fit, G ~ N(0,1)")
    ap.add_argument("--no-classify", action="store_true",
                    help="skip recognition of 262144 generated queries in compressed coordinates")
    ap.add_argument("--rows-reps", type=int, default=20,
                    help="timed passes of the backward and recognition rows (at least --steps; a pass takes "
                         "a few ms, so three would time little more than launch overhead)")
    ap.add_argument("--rows-warmup", type=int, default=5,
                    help="untimed passes before them (at least --warmup)")
    ap.add_argument("--spd", action="store_true",
                    help="also time the general SPD A-norm fit (A = I + grid Laplacian) on the FP32 field")
    ap.add_argument("--weighted", action="store_true",
                    help="also time the diagonal A-norm fit (disc of rows weighted 100x) on the FP32 field")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one elementwise kernel over 1 GiB (read 1 GiB, write 1 GiB) before the fits, "
                         "as the reference for hardware traffic counters")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "xscan_parametric_1048576x4096_traffic.json")


# The source text that decides the X-scan's memory traffic: the kernel, the
# storage loaders, the scan's part of the launch plan, and its launcher.
XSCAN_SOURCES = (
    ("rbd_kernels.h", "// X-scan: per row slab", "// update: finish the column sums"),
    ("rbd_device.h", "template <typename Tx> struct Ld;", "// reductions"),
    ("rbd_api.hip", "bool make_fit_plan(", "P->up_ncb"),
    ("rbd_api.hip", "void launch_xscan(", "template <"),
)


def kernel_sources_sha256():
    """Hash of the X-scan's source text; None when a marker is missing."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1503_05947_amd", "csrc")
    h = hashlib.sha256()
    for fname, start, end in XSCAN_SOURCES:
        text = open(os.path.join(csrc, fname)).read()
        i = text.find(start)
        j = text.find(end, i + len(start)) if i >= 0 else -1
        if i < 0 or j < 0:
            return None
        h.update(text[i:j].encode())
    return h.hexdigest()


def measured_traffic(key, m, n):
    """HBM bytes per X-scan launch from the committed counter runs, or None when the
    kernel sources changed since the counters were taken or the shape differs."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    sha = kernel_sources_sha256()
    if sha is None or rec.get("source_sha256") != sha or (m, n) != (1 << 20, 4096):
        return None
    k = rec.get("kernels", {}).get(key)
    return None if k is None else round(k["traffic_bytes"])


def ensure_built():
    from paper_1503_05947_amd import _build, _lib
    if not os.path.exists(_lib.LIB_PATH):
        log("librbd.so missing: building")
        _build.build_library()


def time_fits(rbd, X, d_max, K, W, weights=None, basis="f64"):
    import torch
    from paper_1503_05947_amd import _lib
    bufs = rbd.FitBuffers(X.shape[0], X.shape[1], d_max, X.dtype, X.device, basis=basis)
    for _ in range(W):
        rbd.fit_into(bufs, X, tol=0.0, weights=weights)
    torch.cuda.synchronize()
    with _lib.Profiler(phases=("xscan",), max_steps=d_max) as prof:
        t0 = time.perf_counter()
        for _ in range(K):
            rbd.fit_into(bufs, X, tol=0.0, weights=weights)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    res = bufs.result()
    return dict(seconds=t1 - t0, fits=K, d=res.d, xscan_ms=prof.avg_ms("xscan"),
                xscan_launches=prof.launches["xscan"], step_end_ms=list(prof.step_end_ms), bufs=bufs, res=res)


def phase_breakdown(rbd, X, d_max, weights=None):
    import torch
    from paper_1503_05947_amd import _lib
    bufs = rbd.FitBuffers(X.shape[0], X.shape[1], d_max, X.dtype, X.device)
    torch.cuda.synchronize()
    with _lib.Profiler(max_steps=d_max) as prof:
        rbd.fit_into(bufs, X, tol=0.0, weights=weights)
    torch.cuda.synchronize()
    return {p: dict(ms=round(prof.phase_ms[p], 4), launches=prof.launches[p],
                    avg_us=round(1e3 * prof.avg_ms(p), 3)) for p in _lib.PHASES}


# ---------------------------------------------------------------------------
# equal-error comparison against the FP64 field
# ---------------------------------------------------------------------------
def checkpoints(d):
    pts = list(range(8, min(d, 128) + 1, 8)) + list(range(160, d + 1, 32))
    if d not in pts:
        pts.append(d)
    return sorted(set(p for p in pts if p <= d))


def sampled_true_error(Y, T, X64J, J, ds):
    """max over sampled columns of ||x64_j - Y[:, :d] T[:d, j]|| at each checkpoint d (FP64, host)."""
    import numpy as np
    R = X64J.copy()
    out = []
    k0 = 0
    for d in ds:
        if d > k0:
            R -= Y[:, k0:d] @ T[k0:d][:, J]
            k0 = d
        out.append(float(np.sqrt(np.einsum("ij,ij->j", R, R)).max()))
    return out


def indicator_gap(res, Xs, J):
    """max over the sampled columns of |col_err_j - ||x_j - Y T_j|||, both of the
    stored values, at the final d, in units of E_0 (pivot columns excluded)."""
    import numpy as np
    import torch
    Jt = torch.from_numpy(J).to(Xs.device)
    XJ = Xs.index_select(1, Jt).double()
    R = XJ - res.Y @ res.T.index_select(1, Jt)
    true = torch.linalg.vector_norm(R, dim=0).cpu().numpy()
    ind = res.col_err.cpu().numpy()[J]
    keep = ~np.isin(J, res.pivots.cpu().numpy())
    E0 = float(res.err_hist[0])
    return float(np.max(np.abs(true - ind)[keep]) / E0) if keep.any() else 0.0


def equal_error_report(runs, pf, ncols, stored=None):
    import numpy as np
    import synth
    g = np.random.default_rng(12345)
    J = np.sort(g.choice(pf.n, size=min(ncols, pf.n), replace=False))
    log(f"equal-error: generating {len(J)} FP64 columns on the host")
    A, B = pf.factors(cols=J)
    rows = np.arange(pf.m)
    a, b = rows // pf.grid, rows % pf.grid
    X64J = A[0][a] * B[0][b]
    for k in range(1, A.shape[0]):
        X64J = X64J + A[k][a] * B[k][b]
    nx64 = np.linalg.norm(X64J, axis=0)
    report = {"columns_sampled": int(len(J)), "checkpoints": None, "precisions": {}}
    E0_64_bound = None
    for name, run in runs.items():
        res = run["res"]
        d = res.d
        ds = checkpoints(d)
        report["checkpoints"] = ds
        log(f"equal-error: {name}: copying Y ({res.Y.numel() * 8 / 2**30:.1f} GiB) and evaluating")
        Y = res.Y.cpu().numpy()
        T = res.T.cpu().numpy()
        sampled = sampled_true_error(Y, T, X64J, J, ds)
        del Y
        hist = res.err_hist.cpu().numpy()
        E0 = float(hist[0])                      # max ||x_j^P|| (stored values)
        storage, basis = run.get("storage", name), run.get("basis", "f64")
        u = UNIT_ROUNDOFF[storage]
        # ||x64 - Y t|| <= ||x^P - Y t|| + ||x64 - x^P|| <= E_d + u/(1-u) * max ||x^P||
        q = u / (1.0 - u) * E0
        E0_64_bound = E0 / (1.0 + u)             # lower bound of max ||x64_j||
        # an FP32 basis adds the downdate's indicator error, of order 2^-24 E_0^2 / E_d
        # (taken with a factor 4; the sampled gap below is its measured value)
        ind = (lambda k: 4.0 * 2.0 ** -24 * E0 * E0 / max(float(hist[k]), 1e-300)) if basis == "f32" else (lambda k: 0.0)
        cert = [(float(hist[k]) + ind(k) + q) / E0_64_bound for k in range(d + 1)]
        steps = run["step_end_ms"]
        entry = {"storage": storage, "basis": basis, "E0_stored": E0,
                 "sampled_rel_err": [s / nx64.max() for s in sampled],
                 "certified_rel_err_at_checkpoints": [cert[k] for k in ds], "time_to_eps_ms": {}}
        if stored is not None and storage in stored:
            entry["indicator_gap_final_d"] = indicator_gap(res, stored[storage], J)
        entry["time_to_eps_sampled_ms"] = {}
        # the certified bound cannot go below twice its storage term: at smaller eps
        # the storage type is not certifiable (null), whatever the fit reaches
        floor = 2.0 * q / E0_64_bound
        entry["certifiable_down_to"] = floor
        for eps in EPS_BOTH + (EPS_FP32 if name == "f32" else ()):
            dd = next((k for k in range(1, d + 1) if cert[k] <= eps), None) if eps >= floor else None
            entry["time_to_eps_ms"][f"{eps:g}"] = (
                None if dd is None else {"d": dd, "ms": round(steps[dd - 1], 3) if dd - 1 < len(steps) else None})
            ds_ok = [k for k, e in zip(ds, entry["sampled_rel_err"]) if e <= eps]
            dd = ds_ok[0] if ds_ok else None
            entry["time_to_eps_sampled_ms"][f"{eps:g}"] = (
                None if dd is None else {"d": dd, "ms": round(steps[dd - 1], 3) if dd - 1 < len(steps) else None})
        report["precisions"][name] = entry
    if "f32" in report["precisions"] and "bf16" in report["precisions"]:
        for key, out in (("time_to_eps_ms", "time_fp32_over_bf16_certified"),
                         ("time_to_eps_sampled_ms", "time_fp32_over_bf16_sampled")):
            ratio = {}
            for eps in EPS_BOTH:
                a32 = report["precisions"]["f32"][key][f"{eps:g}"]
                a16 = report["precisions"]["bf16"][key][f"{eps:g}"]
                ratio[f"{eps:g}"] = (round(a32["ms"] / a16["ms"], 3)
                                     if a32 and a16 and a32["ms"] and a16["ms"] else None)
            report[out] = ratio
        report["time_fp32_over_bf16"] = report["time_fp32_over_bf16_sampled"]
    if "f32" in report["precisions"] and "bf16_basis_f32" in report["precisions"]:
        for key, out in (("time_to_eps_ms", "time_fp32_over_bf16_basis_f32_certified"),
                         ("time_to_eps_sampled_ms", "time_fp32_over_bf16_basis_f32_sampled")):
            ratio = {}
            for eps in EPS_BOTH:
                a32 = report["precisions"]["f32"][key][f"{eps:g}"]
                a16 = report["precisions"]["bf16_basis_f32"][key][f"{eps:g}"]
                ratio[f"{eps:g}"] = (round(a32["ms"] / a16["ms"], 3)
                                     if a32 and a16 and a32["ms"] and a16["ms"] else None)
            report[out] = ratio
    report["note"] = ("certified: (E_d of the stored matrix + storage unit roundoff * max ||x||) / max ||x64||, "
                      "an upper bound on max_j ||x64_j - Y T_j|| / max_j ||x64_j|| at every d, null below twice its storage "
                      "term; sampled: the same quantity evaluated exactly on the sampled columns at the checkpoints "
                      "(a lower bound on the max over all columns), the headline time_fp32_over_bf16.  Times are "
                      "the fit's elapsed device time to the end of step d.")
    return report


# ---------------------------------------------------------------------------
# batched fits: many uneven matrices in one persistent launch
# ---------------------------------------------------------------------------
def _gen_batched(args):
    import numpy as np
    import synth
    seed, b, m, n = args
    return synth.quantize(synth.batched_matrix(seed, b, m, n), "f32")[0]


def batched_inputs(count, cache=None):
    """The stored values of the batch, packed (X_b row-major, back to back), from
    `cache` when it exists, else generated in a pool of fresh interpreters (and
    written to `cache` when given)."""
    import numpy as np
    if cache and os.path.exists(cache):
        log(f"batched: loading {cache}")
        return np.load(cache, allow_pickle=False)
    mats = generate_batched(count)
    Xp = np.concatenate([A.reshape(-1) for A in mats])
    if cache:
        np.save(cache, Xp, allow_pickle=False)
    return Xp


def generate_batched(count):
    import multiprocessing as mp

    import synth
    ms, ns = synth.batched_sizes(0, count=count)
    log(f"batched: generating {count} matrices on the host")
    t0 = time.perf_counter()
    # fresh interpreters (spawn), never a fork of this GPU-initialised process;
    # one BLAS thread per worker
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    mats = []
    try:
        with mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1)) as pool:
            work = [(0, b, int(ms[b]), int(ns[b])) for b in range(count)]
            for i, A in enumerate(pool.imap(_gen_batched, work, chunksize=8)):
                mats.append(A)
                if (i + 1) % 512 == 0:
                    log(f"batched: {i + 1} matrices")
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    log(f"batched: generated in {time.perf_counter() - t0:.1f} s")
    return mats


def batched_section(rbd, count, K, W, d_max=128, tol=1e-6, cache=None):
    import numpy as np
    import torch

    import synth
    ms, ns = synth.batched_sizes(0, count=count)
    dev = torch.device("cuda:0")
    plan = rbd.BatchPlan(ms, ns, d_max, torch.float32, dev)
    Xp = torch.from_numpy(batched_inputs(count, cache)).to(dev)
    cfg = plan.autotune(Xp, tol=tol, rel=True)
    for _ in range(W):
        plan.run(Xp, tol=tol, rel=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        plan.run(Xp, tol=tol, rel=True)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / K
    ds = plan.ints[0].cpu().numpy().astype(np.int64)
    status = plan.ints[1].cpu().numpy()
    # algorithmic bytes: every greedy step streams X_b once (T row) and reads the
    # basis twice (Gram-Schmidt passes); the exact refreshes are not counted
    xbytes = float(np.sum(ds * ms * ns * 4))
    ybytes = float(np.sum(ms * ds * (ds - 1) * 8))           # sum over steps of 2 * m * k * 8
    gbs = (xbytes + ybytes) / sec / 1e9
    return {"workload": f"{count} matrices, m, n log-uniform in [64, 1024], X_b = U diag(10^(-i/8)) V', FP32, "
                        f"relative tol {tol:g}, d_max {d_max}, one persistent launch",
            "value": round(count / sec, 1), "unit": "matrices/s", "ms_per_batch": round(sec * 1e3, 3),
            "greedy_steps_per_s": round(float(ds.sum()) / sec, 1), "mean_d": round(float(ds.mean()), 2),
            "status_ok": int((status == 0).sum()),
            "config": {"threads": cfg.threads, "wg_per_cu": cfg.wg_per_cu},
            "autotune_ms": {f"{t}x{w}": round(v, 3) for (t, w), v in plan.trials.items()},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(gbs / PEAK_HBM_GBS, 4), "algorithmic_GB": round((xbytes + ybytes) / 1e9, 3),
                         "note": "algorithmic bytes: X_b once per greedy step plus two reads of the basis per step "
                                 "(exact refreshes not counted); the matrices in flight fit in the 256 MB "
                                 "Infinity Cache, so this can exceed HBM's rate"}}


def backward_section(rbd, K, W, m=65536, n=2048, d=128, cpu=True, cpu_rows=8192):
    """Gradient of L = <G, Y Y' X> with the pivots of a tol-0, d-step fit held fixed
    (bump field 65536 x 2048, FP32 storage, G ~ N(0,1) in FP64): FP64 matrix-core GEMMs."""
    import numpy as np
    import torch

    import synth
    log(f"backward: bump field {m} x {n}, d = {d}")
    dev = torch.device("cuda:0")
    X = torch.empty((m, n), dtype=torch.float32, device=dev)
    synth.bump_fill(0, X)
    G64 = synth.cotangent(0, m, n)
    G = torch.from_numpy(G64).to(dev)
    res = rbd.fit(X, tol=0.0, d_max=d)
    for _ in range(W):
        rbd.reconstruct_backward(X, G, res.Y, res.T, res.pivots)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        rbd.reconstruct_backward(X, G, res.Y, res.T, res.pivots)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / K
    t0 = time.perf_counter()
    for _ in range(K):
        Z = rbd.reconstruct(res.Y, res.T)
    torch.cuda.synchronize()
    fsec = (time.perf_counter() - t0) / K
    del Z
    flops = 8.0 * m * n * d + 6.0 * m * d * d
    out = {"workload": f"bump field {m} x {n} (FP32 storage), d = {d} pivots fixed from a tol-0 fit, "
                       f"G ~ N(0,1) (FP64), L = <G, Y Y'X>",
           "value": round(1.0 / sec, 2), "unit": "backward passes/s", "ms": round(sec * 1e3, 3),
           "roofline": {"bound": "mfma", "achieved": round(flops / sec / 1e12, 2), "peak": 78.6,
                        "unit": "TFLOP/s", "frac": round(flops / sec / 78.6e12, 4),
                        "algorithmic_GFLOP": round(flops / 1e9, 2),
                        "note": "8mnd + 6md^2 algorithmic flops, FP64 matrix cores (78.6 TFLOP/s dense FP64)"},
           "reconstruct_ms": round(fsec * 1e3, 3), "reconstruct_TFLOPs": round(2.0 * m * n * d / fsec / 1e12, 2),
           "timed_passes": K, "warmup_passes": W}
    if cpu:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
        except Exception:
            cores = os.cpu_count() or 1
        Xs = X[:cpu_rows].double().cpu().numpy()
        Gs = G64[:cpu_rows]
        piv = res.pivots.cpu().numpy()
        t0 = time.perf_counter()
        oracle.reconstruction_grad(Xs, piv, Gs)
        t = time.perf_counter() - t0
        scale = m / cpu_rows                          # the gradient's cost is linear in m
        out["cpu_baseline"] = {"value": round(1.0 / (t * scale), 4), "unit": "backward passes/s",
                               "cores": int(cores), "kind": "oracle",
                               "sample": f"the oracle gradient on rows 0..{cpu_rows - 1} of the field with the same "
                                         f"pivots ({t:.2f} s), scaled by m / {cpu_rows} = {scale:g}"}
    del X, G
    torch.cuda.empty_cache()
    return out


def classify_section(rbd, K, W, k=262144, d_max=40, cpu=True):
    """Recognition at scale: RBD of 200 training views (20 classes x 10, 112 x 92
    grid, FP32), then k generated query views classified in compressed coordinates."""
    import numpy as np
    import torch

    import synth
    dev = torch.device("cuda:0")
    vc = synth.view_classes(0)
    Xtr, ytr, Xte, yte = vc.split()
    m, n = Xtr.shape
    log(f"classify: training fit {m} x {n}, d_max {d_max}; {k} queries")
    Xd = torch.from_numpy(synth.quantize(Xtr, "f32")[0]).to(dev)
    fit = rbd.fit(Xd, tol=0.0, d_max=d_max)
    d = fit.d
    Y = fit.Y.contiguous()
    T = fit.T.contiguous()
    labels = torch.from_numpy(ytr.astype(np.int32)).to(dev)
    lab_q = torch.arange(k, dtype=torch.int32, device=dev) % len(vc.counts)
    V = torch.empty((m, k), dtype=torch.float32, device=dev)
    vc.fill_queries(V, lab_q, coeff_seed=1)
    from paper_1503_05947_amd import _lib
    ws = torch.empty(_lib.classify_workspace_size(m, d, k), dtype=torch.uint8, device=dev)
    for _ in range(W):
        res = rbd.classify(Y, T, V, labels=labels, sync=False, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        res = rbd.classify(Y, T, V, labels=labels, sync=False, workspace=ws)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / K
    acc = (res.label == lab_q).double().mean().item()
    flops = 2.0 * m * d * k
    out = {"workload": f"view classes: 20 classes, {m} pixels (112 x 92), {n} training views, "
                       f"{k} generated query views (FP32)", "d": d, "queries": k,
           "value": round(k / sec, 1), "unit": "queries/s", "ms": round(sec * 1e3, 3),
           "accuracy": round(acc, 4), "timed_passes": K, "warmup_passes": W,
           "roofline": {"bound": "mfma", "achieved": round(flops / sec / 1e12, 2), "peak": 78.6, "unit": "TFLOP/s",
                        "frac": round(flops / sec / 78.6e12, 4), "algorithmic_GFLOP": round(flops / 1e9, 1),
                        "note": "2 m d k flops of the projection Y'V (FP64 matrix cores); the query stream is "
                                f"{m * k * 4 / 1e9:.2f} GB"}}
    if cpu:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
        except Exception:
            cores = os.cpu_count() or 1
        sample = 4096
        Vs = V[:, :sample].cpu().numpy().astype(np.float64)
        Yh, Th = Y.cpu().numpy(), T.cpu().numpy()
        t0 = time.perf_counter()
        oracle.rbd_classify(Yh, Th, ytr, Vs)
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(sample / t, 1), "unit": "queries/s", "cores": int(cores),
                               "kind": "oracle", "sample": f"the first {sample} queries ({t:.2f} s)"}
    del V
    torch.cuda.empty_cache()
    return out


def _time_fit(rbd, X, tol, rel, d_max, reps, warm):
    import torch
    bufs = rbd.FitBuffers(X.shape[0], X.shape[1], d_max, X.dtype, X.device)
    for _ in range(max(warm, 1)):
        rbd.fit_into(bufs, X, tol=tol, rel=rel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        rbd.fit_into(bufs, X, tol=tol, rel=rel)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    d = bufs.result().d
    return bufs, {"greedy_steps": d, "ms_per_fit": round(sec * 1e3, 4), "greedy_steps_per_s": round(d / sec, 1),
                  "us_per_step": round(sec / max(d, 1) * 1e6, 2)}


def _with_driver(loop, fn):
    """Run fn() with RBD_LOOP set (None: the library's own choice)."""
    old = os.environ.get("RBD_LOOP")
    if loop is None:
        os.environ.pop("RBD_LOOP", None)
    else:
        os.environ["RBD_LOOP"] = loop
    try:
        return fn()
    finally:
        if old is None:
            os.environ.pop("RBD_LOOP", None)
        else:
            os.environ["RBD_LOOP"] = old


def bump_field_section(rbd, K, W, cpu=True):
    """The 2048 x 2048 bump field (FP32), relative tol 1e-4 with d_max 256, and the
    same field in fixed-step mode (tol 0, all 256 steps): cache-resident, so the
    step time is latency, not HBM bandwidth.  The library runs such fits as one
    persistent launch; the one-launch-per-kernel driver is timed beside it."""
    import torch

    import synth
    wl = synth.bump_field(0)
    X = torch.from_numpy(synth.quantize(wl.X, "f32")[0]).to("cuda:0")
    out = {"workload": "bump_field 2048x2048 (50 Gaussian bumps + 1e-4 noise), FP32, d_max 256"}
    reps = max(K, 1) * 5
    for name, tol, rel in (("rel_tol_1e-4", wl.tol, True), ("fixed_256_steps", 0.0, False)):
        bufs, r = _with_driver(None, lambda: _time_fit(rbd, X, tol, rel, wl.d_max, reps, W))
        # the same fit captured once as a graph and replayed
        def graph():
            g = rbd.FitGraph(bufs, X, tol=tol, rel=rel)
            g.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                g.replay()
            torch.cuda.synchronize()
            gsec = (time.perf_counter() - t0) / reps
            g.close()
            return gsec
        gsec = _with_driver(None, graph)
        r["graph_ms_per_fit"] = round(gsec * 1e3, 4)
        _, r1 = _with_driver("0", lambda: _time_fit(rbd, X, tol, rel, wl.d_max, reps, W))
        r["one_launch_per_kernel"] = r1
        if cpu:
            X64 = synth.quantize(wl.X, "f32")[1]
            r["cpu_baseline"] = oracle_fit_time(X64, tol, rel, wl.d_max)
        out[name] = r
    return out


def lowrank_section(rbd, K, W, cpu=True):
    """The 512 x 256 low-rank workload (FP32 storage, abs tol 1e-8, d_max 64)."""
    import torch

    import synth
    wl = synth.lowrank_spectrum(0)
    X = torch.from_numpy(synth.quantize(wl.X, "f32")[0]).to("cuda:0")
    reps = max(K, 1) * 10
    _, r = _with_driver(None, lambda: _time_fit(rbd, X, wl.tol, False, wl.d_max, reps, W))
    _, r1 = _with_driver("0", lambda: _time_fit(rbd, X, wl.tol, False, wl.d_max, reps, W))
    r["one_launch_per_kernel"] = r1
    r["workload"] = "low-rank spectrum 512x256 (sigma_i = 10^(-i/4), i < 32, + 1e-10 noise), FP32, tol 1e-8, d_max 64"
    if cpu:
        r["cpu_baseline"] = oracle_fit_time(synth.quantize(wl.X, "f32")[1], wl.tol, False, wl.d_max)
    return r


def _host_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def oracle_fit_time(X64, tol, rel, d_max, sample_steps=None):
    """The oracle (FP64 numpy, as it stands) on the stored values of a small
    configuration, with the host's BLAS threads and with one thread.  With
    sample_steps, a fit of that many steps is timed and scaled to the full
    fit's step count (the oracle's step cost is about constant at these d)."""
    import oracle
    from threadpoolctl import threadpool_limits
    out = {"kind": "oracle", "threads": int(_host_threads())}

    def run():
        dm = sample_steps or d_max
        t0 = time.perf_counter()
        r = oracle.rbd_fit(X64, tol, dm, rel=rel)
        return time.perf_counter() - t0, r.d

    sec, d = run()
    if sample_steps:
        out["sample"] = f"{d} greedy steps timed, scaled to {d_max}"
        sec *= d_max / max(d, 1)
        d = d_max
    out["greedy_steps"] = d
    out["ms_per_fit"] = round(sec * 1e3, 2)
    out["us_per_step"] = round(sec / max(d, 1) * 1e6, 1)
    with threadpool_limits(limits=1):
        sec1, d1 = run()
    if sample_steps:
        sec1 *= d_max / max(d1, 1)
    out["single_thread_ms_per_fit"] = round(sec1 * 1e3, 2)
    return out


def paper_examples_section(rbd, K, W, cpu=True):
    """The paper's worked examples on the device, beside the oracle: the three
    separable functions of Table 3 (512^2 grid, FP64, relative tol 1e-10) and
    the section 4.2.2 field (5001^2 grid, FP64, 22 steps)."""
    import torch

    import synth
    out = {}
    for which in (1, 2, 3):
        X = synth.table3(which, 512)
        Xd = torch.from_numpy(X).to("cuda:0")
        _, r = _time_fit(rbd, Xd, 1e-10, True, 20, max(K, 1) * 10, W)
        if cpu:
            r["cpu_baseline"] = oracle_fit_time(X, 1e-10, True, 20)
        out[f"table3_f{which}_512"] = r
    X = synth.approx_field(5001)
    Xd = torch.from_numpy(X).to("cuda:0")
    _, r = _time_fit(rbd, Xd, 0.0, False, 22, max(K, 1), W)
    if cpu:
        r["cpu_baseline"] = oracle_fit_time(X, 0.0, False, 22)
    out["approx_field_5001"] = r
    del Xd
    torch.cuda.empty_cache()
    return out


def stream_ceiling(rbd, t, reps=5):
    """GB/s of one read of every byte of tensor t (non-temporal 16-byte loads, as the
    X-scan reads X): the ceiling for a scan of that buffer."""
    import torch
    rbd.read_stream(t)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        rbd.read_stream(t)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    nbytes = t.numel() * t.element_size()
    return {"bytes": nbytes, "ms": round(ms, 4), "GBs": round(nbytes / (ms * 1e-3) / 1e9, 1),
            "frac": round(nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}


def batched_cpu_baseline(count=4096, sample=24, d_max=128, tol=1e-6):
    import numpy as np
    import oracle
    import synth
    ms, ns = synth.batched_sizes(0, count=count)
    idx = np.linspace(0, count - 1, sample).astype(int)
    t = 0.0
    for b in idx:
        X = synth.quantize(synth.batched_matrix(0, int(b), int(ms[b]), int(ns[b])), "f32")[1]
        t0 = time.perf_counter()
        oracle.rbd_fit(X, tol, d_max, rel=True)
        t += time.perf_counter() - t0
    scale = float((ms * ns).sum()) / float((ms[idx] * ns[idx]).sum())
    return {"value": round(count / (t * scale), 3), "unit": "matrices/s", "kind": "oracle",
            "sample": f"{sample} evenly spaced matrices of the batch fitted one by one ({t:.1f} s), scaled by the "
                      f"ratio of total to sampled m*n ({scale:.1f})"}


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample of the same workload
# ---------------------------------------------------------------------------
def cpu_baseline(full_m, grid_sample=256, n=4096, steps=24):
    import numpy as np
    import oracle
    import synth
    cores = _host_threads()
    pf = synth.parametric_field(0, grid=grid_sample, n=n)
    X = synth.quantize(pf.full(), "f32")[1]
    m = X.shape[0]
    t0 = time.perf_counter()
    oracle.rbd_fit(X, 0.0, 1)                    # set-up plus one step
    t1 = time.perf_counter()
    oracle.rbd_fit(X, 0.0, 1 + steps)
    t2 = time.perf_counter()
    per_step = ((t2 - t1) - (t1 - t0)) / steps
    per_step = max(per_step, 1e-9)
    scale = full_m / m                           # the oracle's step cost is linear in m
    return {"value": round(1.0 / (per_step * scale), 6), "unit": "greedy steps/s", "cores": int(cores),
            "kind": "oracle",
            "sample": (f"oracle rbd_fit (FP64 numpy) on the same generator at a {grid_sample}x{grid_sample} grid "
                       f"({m} x {n}, FP32-rounded), {steps} greedy steps timed (difference of a {1 + steps}-step "
                       f"and a 1-step fit: {per_step:.3f} s/step), scaled by m_full/m_sample = {scale:g}")}


def next_rows(rbd, args):
    import torch
    out = {}
    if not args.no_batched:
        out["batched"] = batched_section(rbd, args.batch_count, args.steps, args.warmup, cache=args.batched_cache)
        if not args.no_cpu_baseline:
            out["batched"]["cpu_baseline"] = batched_cpu_baseline(args.batch_count)
    reps, warm = max(args.steps, args.rows_reps), max(args.warmup, args.rows_warmup)
    if not args.no_backward:
        torch.cuda.empty_cache()
        out["backward"] = backward_section(rbd, reps, warm, cpu=not args.no_cpu_baseline)
    if not args.no_classify:
        torch.cuda.empty_cache()
        out["recognition"] = classify_section(rbd, reps, warm, cpu=not args.no_cpu_baseline)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path. "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.write_batched_cache:
        if not args.batched_cache:
            sys.exit("--write-batched-cache needs --batched-cache PATH")
        batched_inputs(args.batch_count, args.batched_cache)
        log(f"wrote {args.batched_cache}")
        return
    ensure_built()
    import numpy as np
    import torch

    import paper_1503_05947_amd as rbd
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.next_rows_only:
        print(json.dumps({"next_rows_only": True, **next_rows(rbd, args)}), flush=True)
        return
    pf = synth.parametric_field(seed=0, grid=args.grid, n=args.n)
    m, n = pf.m, pf.n
    log(f"generating the parametric field {m} x {n} (FP32) on {torch.cuda.get_device_name(0)}")
    X32 = torch.empty((m, n), dtype=torch.float32, device=dev)
    pf.fill_device(X32)
    torch.cuda.synchronize()

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: one neg kernel, 1 GiB read + 1 GiB written")

    runs = {}
    log(f"FP32 storage: {args.warmup} warm-up + {args.steps} timed fits, d_max {args.d_max}")
    runs["f32"] = time_fits(rbd, X32, args.d_max, args.steps, args.warmup)
    if not args.no_bf16:
        X16 = X32.to(torch.bfloat16)
        log("BF16 storage")
        runs["bf16"] = time_fits(rbd, X16, args.d_max, args.steps, args.warmup)
        if not args.no_basis32:
            log("BF16 storage, basis kept in FP32")
            runs["bf16_basis_f32"] = time_fits(rbd, X16, args.d_max, args.steps, args.warmup, basis="f32")
            runs["bf16_basis_f32"].update(storage="bf16", basis="f32")

    log("read-stream ceiling on X's own buffers")
    ceiling = {"f32": stream_ceiling(rbd, X32)}
    if "bf16" in runs:
        ceiling["bf16"] = stream_ceiling(rbd, X16)

    phases = None
    if args.phases:
        phases = {k: phase_breakdown(rbd, X32 if k == "f32" else X16, args.d_max) for k in runs if k != "bf16_basis_f32"}

    def summary(r, sx):
        sec = r["seconds"] / r["fits"]
        gbs = m * n * sx / (r["xscan_ms"] * 1e-3) / 1e9
        return sec, gbs

    sec32, gbs32 = summary(runs["f32"], 4)
    steps_s = runs["f32"]["d"] / sec32
    out = {
        "metric": "greedy steps/s + X-scan HBM GB/s (% peak); BF16 vs FP32 at equal error",
        "value": round(steps_s, 3),
        "unit": "greedy steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec32 * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"parametric_field {m}x{n} (x_j(s) = sum_k exp(-mu_jk |s-c_k|^2), "
                               f"{args.grid}^2 grid), FP32 storage, tol 0, d_max {args.d_max}",
                   "m": m, "n": n, "d_max": args.d_max, "tol": 0.0, "storage": "f32",
                   "greedy_steps_per_fit": runs["f32"]["d"], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(gbs32, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs32 / PEAK_HBM_GBS, 4), "traffic": measured_traffic("f32", m, n),
                     "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE, calibrated)",
                     "algorithmic_bytes": m * n * 4,
                     "kernel": "xscan (T(d,:) = xi' X)", "kernel_avg_ms": round(runs["f32"]["xscan_ms"], 4),
                     "launches_timed": runs["f32"]["xscan_launches"],
                     "read_stream_ceiling": ceiling["f32"]},
    }
    if "bf16" in runs:
        sec16, gbs16 = summary(runs["bf16"], 2)
        out["bf16_storage"] = {"value": round(runs["bf16"]["d"] / sec16, 3), "unit": "greedy steps/s",
                               "ms_per_fit": round(sec16 * 1e3, 3),
                               "xscan_GBs": round(gbs16, 1), "xscan_frac": round(gbs16 / PEAK_HBM_GBS, 4),
                               "traffic": measured_traffic("bf16", m, n), "algorithmic_bytes": m * n * 2,
                               "kernel_avg_ms": round(runs["bf16"]["xscan_ms"], 4),
                               "read_stream_ceiling": ceiling["bf16"]}
    if "bf16_basis_f32" in runs:
        r = runs["bf16_basis_f32"]
        secb, gbsb = summary(r, 2)
        out["bf16_storage_basis_f32"] = {
            "value": round(r["d"] / secb, 3), "unit": "greedy steps/s", "ms_per_fit": round(secb * 1e3, 3),
            "xscan_GBs": round(gbsb, 1), "xscan_frac": round(gbsb / PEAK_HBM_GBS, 4),
            "kernel_avg_ms": round(r["xscan_ms"], 4), "speedup_vs_fp64_basis": round(sec16 / secb, 3),
            "note": "rbd_fit_basis(RBD_BASIS_F32): the basis is stored in FP32 while the loop runs, all "
                    "arithmetic FP64; accuracy in equal_error.precisions.bf16_basis_f32"}
    if args.weighted:
        w64 = torch.from_numpy(synth.disc_weights(args.grid)).to(dev)
        log("diagonal A-norm (disc weights), FP32 storage")
        rw = time_fits(rbd, X32, args.d_max, args.steps, args.warmup, weights=w64)
        secw, gbsw = summary(rw, 4)
        out["weighted"] = {"A": f"diag: rows in a disc of radius 0.25 about (0.5, 0.5) weighted 100, others 1",
                           "value": round(rw["d"] / secw, 3), "unit": "greedy steps/s",
                           "ms_per_fit": round(secw * 1e3, 3), "greedy_steps_per_fit": rw["d"],
                           "xscan_GBs": round(gbsw, 1), "xscan_frac": round(gbsw / PEAK_HBM_GBS, 4),
                           "algorithmic_bytes": m * n * 4, "kernel_avg_ms": round(rw["xscan_ms"], 4),
                           "cost_vs_identity": round(secw / sec32, 3)}
        if args.phases:
            out["weighted"]["phases"] = phase_breakdown(rbd, X32, args.d_max, weights=w64)
        del rw["bufs"], rw["res"]
    if args.spd:
        import numpy as np
        ip, ix, av = synth.grid_laplacian_spd(args.grid, args.grid, 1.0)
        A = rbd.CsrMatrix(torch.from_numpy(ip).to(dev), torch.from_numpy(ix).to(dev), torch.from_numpy(av).to(dev))
        log("general SPD A = I + L (5-point grid Laplacian), FP32 storage")
        bufs = rbd.FitBuffers(m, n, args.d_max, X32.dtype, dev, spd=True)
        for _ in range(args.warmup):
            rbd.fit_into(bufs, X32, tol=0.0, A=A)
        torch.cuda.synchronize()
        from paper_1503_05947_amd import _lib
        with _lib.Profiler(max_steps=args.d_max) as prof:
            t0 = time.perf_counter()
            for _ in range(args.steps):
                rbd.fit_into(bufs, X32, tol=0.0, A=A)
            torch.cuda.synchronize()
            secs = (time.perf_counter() - t0) / args.steps
        rs = bufs.result()
        gbs = m * n * 4 / (prof.avg_ms("xscan") * 1e-3) / 1e9
        out["spd"] = {"A": f"I + L, 5-point Laplacian of the {args.grid} x {args.grid} grid (CSR, nnz {len(av)})",
                      "value": round(rs.d / secs, 3), "unit": "greedy steps/s", "ms_per_fit": round(secs * 1e3, 3),
                      "greedy_steps_per_fit": rs.d, "xscan_GBs": round(gbs, 1),
                      "xscan_frac": round(gbs / PEAK_HBM_GBS, 4), "cost_vs_identity": round(secs / sec32, 3),
                      "phases_ms_per_fit": {p: round(prof.phase_ms[p] / args.steps, 2) for p in _lib.PHASES}}
        del bufs, A
        torch.cuda.empty_cache()
    cpu = not args.no_cpu_baseline
    log("bump field 2048 x 2048 (FP32)")
    out["bump_field_2048"] = bump_field_section(rbd, args.steps, args.warmup, cpu=cpu)
    log("low-rank 512 x 256 (FP32)")
    out["lowrank_512x256"] = lowrank_section(rbd, args.steps, args.warmup, cpu=cpu)
    if not args.no_paper_examples:
        log("the paper's worked examples (Table 3, section 4.2.2)")
        out["paper_examples"] = paper_examples_section(rbd, args.steps, args.warmup, cpu=cpu)
    if phases:
        out["phases"] = phases
    if not args.no_equal_error:
        stored = {"f32": X32}
        if "bf16" in runs:
            stored["bf16"] = X16
        out["equal_error"] = equal_error_report(runs, pf, args.sample_cols, stored)
    for r in runs.values():
        del r["bufs"], r["res"]
    nxt = not args.no_next_rows
    del X32
    if "bf16" in runs:
        del X16
    torch.cuda.empty_cache()
    if nxt:
        out.update(next_rows(rbd, args))
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle on a bounded sample)")
        out["cpu_baseline"] = cpu_baseline(m, n=n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
