// Host side of the batched fit: batch planning (offsets, longest-first order),
// the persistent launch, and the empirical autotuner over workgroup shapes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

#include "../../include/rbd.h"
#include "rbd_batched.h"

namespace {

using namespace rbd;

int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

int elem_size(rbd_dtype t) {
    switch (t) {
        case RBD_F32: return 4;
        case RBD_BF16: return 2;
        case RBD_F16: return 2;
        case RBD_F64: return 8;
    }
    return 0;
}

int cu_count() {
    static int cached = 0;
    if (cached == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 256;
    }
    return cached;
}

constexpr size_t kHeader = 256;   // queue counter lives at the start of the workspace

template <typename Tx, int TPB>
hipError_t launch_batched(const Tx* X, const int64_t* desc, const int* order, int nitems, int stride, double tol,
                          int rel, int d_max, double* Y, double* T, int64_t* pivots, double* col_err,
                          double* err_hist, int32_t* d_out, int32_t* status, int64_t max_m, char* ws, int grid,
                          hipStream_t s) {
    unsigned* queue = reinterpret_cast<unsigned*>(ws);
    double* wsd = reinterpret_cast<double*>(ws + kHeader);
    // LDS: v (max_m doubles), then as many basis vectors as fit in this
    // workgroup's share of the CU's LDS (grid / CUs workgroups per CU)
    int dev = 0, per_cu = 0, per_block = 0;
    hipFuncAttributes attr{};
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&batched_fit_kernel<Tx, TPB>)) != hipSuccess)
        return hipErrorInvalidValue;
    const int wg_per_cu = std::max(1, grid / std::max(1, cu_count()));
    const int64_t share = std::min<int64_t>(per_block, per_cu / wg_per_cu) - (int64_t)attr.sharedSizeBytes - 256;
    const int64_t vbytes = 8 * max_m;
    const int ycap = (int)std::max<int64_t>(0, (share - vbytes) / 8);
    const size_t dyn = (size_t)vbytes + 8 * (size_t)ycap;
    if ((int64_t)dyn > std::max<int64_t>(vbytes, share)) return hipErrorInvalidValue;
    // allow dynamic LDS beyond the default per-launch limit (the request is checked at launch)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&batched_fit_kernel<Tx, TPB>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    batch_queue_reset_kernel<<<1, 64, 0, s>>>(queue);
    batched_fit_kernel<Tx, TPB><<<grid, TPB, dyn, s>>>(X, desc, order, nitems, stride, queue, tol, rel, d_max, Y, T,
                                                        pivots, col_err, err_hist, d_out, status, wsd, (int)max_m,
                                                        ycap);
    return hipGetLastError();
}

template <typename Tx>
hipError_t dispatch(int threads, const Tx* X, const int64_t* desc, const int* order, int nitems, int stride,
                    double tol, int rel, int d_max, double* Y, double* T, int64_t* pivots, double* col_err,
                    double* err_hist, int32_t* d_out, int32_t* status, int64_t max_m, char* ws, int grid,
                    hipStream_t s) {
    switch (threads) {
        case 64:
            return launch_batched<Tx, 64>(X, desc, order, nitems, stride, tol, rel, d_max, Y, T, pivots, col_err,
                                          err_hist, d_out, status, max_m, ws, grid, s);
        case 128:
            return launch_batched<Tx, 128>(X, desc, order, nitems, stride, tol, rel, d_max, Y, T, pivots, col_err,
                                           err_hist, d_out, status, max_m, ws, grid, s);
        case 256:
            return launch_batched<Tx, 256>(X, desc, order, nitems, stride, tol, rel, d_max, Y, T, pivots, col_err,
                                           err_hist, d_out, status, max_m, ws, grid, s);
        case 512:
            return launch_batched<Tx, 512>(X, desc, order, nitems, stride, tol, rel, d_max, Y, T, pivots, col_err,
                                           err_hist, d_out, status, max_m, ws, grid, s);
        case 1024:
            return launch_batched<Tx, 1024>(X, desc, order, nitems, stride, tol, rel, d_max, Y, T, pivots, col_err,
                                            err_hist, d_out, status, max_m, ws, grid, s);
    }
    return hipErrorInvalidValue;
}

int run(const void* X, rbd_dtype xt, const int64_t* desc, const int32_t* order, int nitems, int stride, double tol,
        int rel, int d_max, rbd_batch_config cfg, double* Y, double* T, int64_t* pivots, double* col_err,
        double* err_hist, int32_t* d_out, int32_t* status, int64_t max_m, void* workspace, hipStream_t s) {
    const int grid = std::max(1, cfg.wg_per_cu) * cu_count();
    char* ws = reinterpret_cast<char*>(workspace);
    hipError_t e = hipErrorInvalidValue;
    switch (xt) {
        case RBD_F32:
            e = dispatch<float>(cfg.threads, static_cast<const float*>(X), desc, order, nitems, stride, tol, rel, d_max,
                                Y, T, pivots, col_err, err_hist, d_out, status, max_m, ws, grid, s);
            break;
        case RBD_F64:
            e = dispatch<double>(cfg.threads, static_cast<const double*>(X), desc, order, nitems, stride, tol, rel,
                                 d_max, Y, T, pivots, col_err, err_hist, d_out, status, max_m, ws, grid, s);
            break;
        case RBD_BF16:
            e = dispatch<bf16_t>(cfg.threads, static_cast<const bf16_t*>(X), desc, order, nitems, stride, tol, rel,
                                 d_max, Y, T, pivots, col_err, err_hist, d_out, status, max_m, ws, grid, s);
            break;
        case RBD_F16:
            e = dispatch<f16_t>(cfg.threads, static_cast<const f16_t*>(X), desc, order, nitems, stride, tol, rel,
                                d_max, Y, T, pivots, col_err, err_hist, d_out, status, max_m, ws, grid, s);
            break;
    }
    return e == hipSuccess ? RBD_OK : RBD_EDEVICE;
}

bool valid_config(rbd_batch_config c) {
    return (c.threads == 64 || c.threads == 128 || c.threads == 256 || c.threads == 512 || c.threads == 1024) &&
           c.wg_per_cu >= 1 &&
           c.wg_per_cu <= 16;
}

}  // namespace

extern "C" {

int rbd_batch_plan(const int64_t* m, const int64_t* n, int32_t batch, int32_t d_max, int64_t* desc, int32_t* order,
                   rbd_batch_sizes* sizes) {
    if (!m || !n || !desc || !order || !sizes || batch < 1 || d_max < 1 || d_max > kBatchMaxD) return RBD_EINVAL;
    int64_t xo = 0, yo = 0, to = 0, co = 0, wo = 0, mm = 0, mn = 0;
    std::vector<double> cost(batch);
    for (int b = 0; b < batch; ++b) {
        if (m[b] < 1 || n[b] < 1 || m[b] > kBatchMaxM || n[b] >= (int64_t)INT32_MAX) return RBD_EINVAL;
        const int64_t D = std::min<int64_t>(d_max, std::min(m[b], n[b]));
        int64_t* dsc = desc + (int64_t)b * kDescWords;
        dsc[kDescM] = m[b];
        dsc[kDescN] = n[b];
        dsc[kDescX] = xo;
        dsc[kDescY] = yo;
        dsc[kDescT] = to;
        dsc[kDescC] = co;
        dsc[kDescW] = wo;
        dsc[kDescD] = D;
        xo += m[b] * n[b];
        yo += m[b] * d_max;
        to += (int64_t)d_max * n[b];
        co += n[b];
        wo += D * m[b] + 2 * n[b];
        mm = std::max(mm, m[b]);
        mn = std::max(mn, n[b]);
        cost[b] = (double)m[b] * (double)n[b] * (double)D;
    }
    std::vector<int32_t> idx(batch);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t c) { return cost[a] > cost[c]; });
    std::copy(idx.begin(), idx.end(), order);
    sizes->x_elems = xo;
    sizes->y_elems = yo;
    sizes->t_elems = to;
    sizes->c_elems = co;
    sizes->max_m = mm;
    sizes->max_n = mn;
    sizes->workspace_bytes = kHeader + sizeof(double) * (size_t)wo;
    return RBD_OK;
}

int rbd_fit_batched(const void* X, rbd_dtype xt, const int64_t* desc, const int32_t* order, int32_t batch,
                    double tol, rbd_tol_mode mode, int32_t d_max, rbd_batch_config cfg, double* Y, double* T,
                    int64_t* pivots, double* col_err, double* err_hist, int32_t* d_out, int32_t* status,
                    int64_t max_m, void* workspace, size_t workspace_bytes, void* stream) {
    if (!X || !desc || !order || !Y || !T || !pivots || !col_err || !err_hist || !d_out || !status || !workspace)
        return RBD_EINVAL;
    if (batch < 1 || d_max < 1 || d_max > kBatchMaxD || max_m < 1 || max_m > kBatchMaxM) return RBD_EINVAL;
    if (elem_size(xt) == 0 || !valid_config(cfg)) return RBD_EINVAL;
    if (!(tol >= 0.0) || tol == HUGE_VAL || (mode != RBD_TOL_ABS && mode != RBD_TOL_REL)) return RBD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return RBD_EINVAL;
    if (workspace_bytes < kHeader) return RBD_EWORKSPACE;
    return run(X, xt, desc, order, batch, 1, tol, mode == RBD_TOL_REL, d_max, cfg, Y, T, pivots, col_err, err_hist,
               d_out, status, max_m, workspace, reinterpret_cast<hipStream_t>(stream));
}

int rbd_batched_autotune(const void* X, rbd_dtype xt, const int64_t* desc, const int32_t* order, int32_t batch,
                         double tol, rbd_tol_mode mode, int32_t d_max, int32_t sample_stride, double* Y, double* T,
                         int64_t* pivots, double* col_err, double* err_hist, int32_t* d_out, int32_t* status,
                         int64_t max_m, void* workspace, size_t workspace_bytes, void* stream,
                         rbd_batch_config* best, double* trial_ms) {
    if (!best || sample_stride < 1) return RBD_EINVAL;
    if (!X || !desc || !order || !Y || !T || !pivots || !col_err || !err_hist || !d_out || !status || !workspace)
        return RBD_EINVAL;
    if (batch < 1 || d_max < 1 || d_max > kBatchMaxD || max_m < 1 || max_m > kBatchMaxM || elem_size(xt) == 0)
        return RBD_EINVAL;
    if (!(tol >= 0.0) || tol == HUGE_VAL || (mode != RBD_TOL_ABS && mode != RBD_TOL_REL)) return RBD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return RBD_EINVAL;
    if (workspace_bytes < kHeader) return RBD_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int nitems = (int)cdiv64(batch, sample_stride);
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return RBD_EDEVICE;
    const int threads[4] = {128, 256, 512, 1024};
    const int wgs[4] = {1, 2, 4, 8};
    float best_ms = 0.f;
    int t = 0, rc = RBD_OK;
    bool found = false;
    for (int ti = 0; ti < 4 && rc == RBD_OK; ++ti)
        for (int wi = 0; wi < 4 && rc == RBD_OK; ++wi, ++t) {
            rbd_batch_config c{threads[ti], wgs[wi]};
            float ms = 0.f;
            bool ok = true;
            for (int rep = 0; rep < 2 && ok && rc == RBD_OK; ++rep) {   // first run warms caches and code
                if (hipEventRecord(a, s) != hipSuccess) rc = RBD_EDEVICE;
                if (rc == RBD_OK && run(X, xt, desc, order, nitems, sample_stride, tol, mode == RBD_TOL_REL, d_max, c,
                                        Y, T, pivots, col_err, err_hist, d_out, status, max_m, workspace,
                                        s) != RBD_OK) {
                    ok = false;                 // shape not launchable here (e.g. LDS): skip it
                    (void)hipGetLastError();
                    if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess) rc = RBD_EDEVICE;
                    break;
                }
                if (rc == RBD_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                                     hipEventElapsedTime(&ms, a, b) != hipSuccess))
                    rc = RBD_EDEVICE;
            }
            if (trial_ms) trial_ms[t] = ok ? ms : -1.0;
            if (rc == RBD_OK && ok && (!found || ms < best_ms)) {
                best_ms = ms;
                *best = c;
                found = true;
            }
        }
    if (rc == RBD_OK && !found) rc = RBD_EDEVICE;
    if (hipEventDestroy(a) != hipSuccess || hipEventDestroy(b) != hipSuccess) rc = RBD_EDEVICE;
    return rc;
}

}  // extern "C"
