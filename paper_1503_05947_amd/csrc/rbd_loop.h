// Persistent greedy loop (Algorithm 1 with A = I, section 3.1) for inputs that
// stay in the caches: one launch runs the column norms, every step and the
// epilogue, so a fit that stops early (step 2.4) costs only the steps it
// takes, and a step costs two grid-wide barriers instead of a dozen launches.
//
// G workgroups, all resident at once (G <= the number of CUs, one workgroup
// per CU by its LDS use).  Roles within a step d:
//   A  (the first Gc workgroups, RB rows each) write the previous step's basis
//      column Y(:, d-1) = (v1' - Y h2') / nu' (lagged, as in the multi-launch
//      path) and form v1 = x_p - Y(:, 0:d) T(0:d, p) for their rows, with
//      partial sums of h2 = Y' v1 and ||v1||^2.              -- barrier --
//   B  (every workgroup) sums the partials in a fixed order, nu^2 =
//      ||v1||^2 - ||h2||^2 and the break test of step 2.2; for its own CW
//      columns it forms T(d, j) = (v1' x_j - h2' T(0:d, j)) / nu, downdates
//      e_j^2 (eq. (3)), flags columns for an exact refresh and takes its
//      lowest-index argmax.                                  -- barrier --
//   C  (every workgroup) merges the G partial maxima.  When any column was
//      flagged, each workgroup re-evaluates ||x_j - Y T(:, j)||^2 exactly for
//      its own columns below kRefreshEager of their last exact value, with
//      the pending column xi_d formed on the fly, and the maxima are merged
//      again (one more barrier).  Then pivot, E_d and the stop test of 2.4.
// Every workgroup takes the same decisions from the same data, so the loop
// ends in all of them at the same step.
//
// Workgroups exchange data only through device-scope loads and stores
// (coherent across the XCDs' L2 caches without cache write-backs or
// invalidations); a barrier waits for the workgroup's stores, then counts on a
// device-scope atomic.  X is read with ordinary loads: it is never written, so
// each XCD keeps its workgroups' columns of X in its L2 from step to step
// (workgroups of one XCD own adjacent column slices).  Every barrier wait is
// bounded in time: past the limit the workgroup raises the abort flag, every
// workgroup leaves the loop, and the fit reports RBD_EDEVICE in *status.
#pragma once

#include "rbd_device.h"

namespace rbd {

constexpr int kLoopThreads = 256;
constexpr int kLoopMaxCW = 64;            // columns per workgroup
constexpr int kLoopMaxRB = 1024;          // rows per Gram-Schmidt workgroup
constexpr int kLoopChunk = 2048;          // rows of v1 staged in LDS per pass of the scan
constexpr int kLoopRefCols = 8;           // queued columns per pass of an exact refresh
constexpr unsigned long long kLoopWaitTicks = 400000000ull;   // 4 s of the 100 MHz real-time counter

template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct LoopWs {
    unsigned* bar;        // barrier counter, zero at launch
    int* abort_flag;      // zero at launch
    double* part;         // Gc x (D + 1): Y'v1 partials and ||v1||^2 per Gram-Schmidt workgroup
    double* v1;           // m
    double* bval;         // 2 x G partial maxima (two sets, used alternately)
    int64_t* bidx;        // 2 x G
    double* bcnt;         // 2 x G flagged-column counts
};

struct LoopOut {
    double* Y;            // m x d_max
    double* T;            // d_max x n
    int64_t* pivots;
    double* col_err;
    double* err_hist;
    int32_t* d_out;
    int32_t* status;
    int32_t* stop_reason;
};

// Grid-wide barrier.  Stores issued before it are complete (device scope)
// before the workgroup is counted.  Returns false in every thread when the
// wait ran out of time or another workgroup gave up.
__device__ __forceinline__ bool loop_sync(const LoopWs& ws, unsigned& target, int* s_flag) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        target += gridDim.x;
        __hip_atomic_fetch_add(ws.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        while (ld_dev(ws.bar) < target) {
            if (ld_dev(ws.abort_flag)) { ok = 0; break; }
            __builtin_amdgcn_s_sleep(1);
            if (__builtin_amdgcn_s_memrealtime() - t0 > kLoopWaitTicks) {
                st_dev(ws.abort_flag, 1);
                ok = 0;
                break;
            }
        }
        *s_flag = ok;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Merge the G partial maxima of set `set`; every thread gets the result.
__device__ __forceinline__ void loop_merge(const LoopWs& ws, int set, double& v, int64_t& i, double& cnt,
                                           double* sv, int64_t* si) {
    const int G = gridDim.x;
    v = -1.0;
    i = INT64_MAX;
    double c = 0.0;
    for (int q = threadIdx.x; q < G; q += kLoopThreads) {
        argmax_merge(v, i, ld_dev(ws.bval + set * G + q), ld_dev(ws.bidx + set * G + q));
        c += ld_dev(ws.bcnt + set * G + q);
    }
    cnt = block_sum(c, sv);
    block_argmax(v, i, sv, si);
}

template <typename Tx>
__global__ __launch_bounds__(kLoopThreads) void loop_kernel(const Tx* __restrict__ X, int64_t ldx, int m, int n,
                                                            int D, int d_max, double tol, int rel, int64_t start,
                                                            LoopOut out, LoopWs ws, int Gc, int RB, int CW) {
    using L = Ld<Tx>;
    const int G = gridDim.x, w = blockIdx.x, tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int D1 = D + 1;

    __shared__ double s_h1[RBD_MAX_D + 1];          // T(0:d, p) of this step
    __shared__ double s_h2[RBD_MAX_D + 1];          // h2 and ||v1||^2 of the last step
    __shared__ double s_v1own[kLoopMaxRB];          // v1 on this workgroup's Gram-Schmidt rows
    __shared__ double s_vc[kLoopChunk];             // v1 staged for the scan
    __shared__ double s_e2[kLoopMaxCW], s_b2[kLoopMaxCW], s_tcol[kLoopMaxCW];
    __shared__ double s_red[4 * (RBD_MAX_D + 1)];   // per-wave partial rows; scan partials
    __shared__ double s_tq[kLoopRefCols * (RBD_MAX_D + 1)];   // refresh: T(0:d+1, queued columns)
    __shared__ int s_list[kLoopMaxCW];
    __shared__ int s_flag, s_nq;
    __shared__ double sv[4];
    __shared__ int64_t si[4];

    // XCD-aware column slice: consecutive workgroup indices go to different
    // XCDs, so the G / 8 workgroups of one XCD own adjacent slices.
    const int slice = (G % 8 == 0) ? (w % 8) * (G / 8) + w / 8 : w;
    const int c0 = slice * CW;
    const int nc = max(0, min(n - c0, CW));
    const int col = tid % CW, rsub = tid / CW, rpi = kLoopThreads / CW;
    const bool gs = w < Gc;
    const int r0 = w * RB, r1 = gs ? min(m, r0 + RB) : r0;
    unsigned target = 0;

    // ---- pre-computation of diag(X'X) (section 3.3): e_j^2 = ||x_j||^2 ----
    {
        double acc = 0.0;
        if (col < nc) {
            const Tx* xc = X + c0 + col;
#pragma unroll 8
            for (int i = rsub; i < m; i += rpi) {
                const double x = L::one(xc + (int64_t)i * ldx);
                acc = fma(x, x, acc);
            }
        }
        s_red[tid] = acc;
        __syncthreads();
        double best = -1.0, nonfin = 0.0;
        int64_t bi = INT64_MAX;
        if (tid < nc) {
            double s = 0.0;
            for (int q = 0; q < rpi; ++q) s += s_red[q * CW + tid];
            if (!isfinite(s)) nonfin = 1.0;
            s_e2[tid] = s;
            s_b2[tid] = s;
            best = s;
            bi = c0 + tid;
        }
        __syncthreads();
        nonfin = block_sum(nonfin, sv);
        block_argmax(best, bi, sv, si);
        if (tid == 0) {
            st_dev(ws.bval + w, best);
            st_dev(ws.bidx + w, bi);
            st_dev(ws.bcnt + w, nonfin);
        }
    }
    bool alive = loop_sync(ws, target, &s_flag);
    double E0 = 0.0, tau = 0.0, nu_prev = 0.0;
    int p = 0, d = 0, stop = 0, status = RBD_OK;
    bool pending = false;             // Y(:, d-1) not yet written
    if (alive) {
        double v, nonfin;
        int64_t i;
        loop_merge(ws, 0, v, i, nonfin, sv, si);
        if (nonfin > 0.0) {
            status = RBD_ENONFINITE;
            stop = kStopError;
        } else {
            E0 = sqrt(v);
            tau = rel ? tol * E0 : tol;
            p = start >= 0 ? (int)start : (int)i;
        }
        if (w == 0 && tid == 0) out.err_hist[0] = stop ? NAN : E0;
    }

    int set = 1;
    while (alive && !stop && d < D) {
        // ---- A: lagged basis column, v1 = x_p - Y(:, 0:d) T(0:d, p), partials ----
        if (gs) {
            for (int k = tid; k < d; k += kLoopThreads) s_h1[k] = ld_dev(out.T + (int64_t)k * n + p);
            __syncthreads();
            const int dl = pending ? d - 1 : d;          // columns of Y already written
            const double inv_prev = pending ? 1.0 / nu_prev : 0.0;
            double h2acc[RBD_MAX_D / kWave];
#pragma unroll
            for (int c = 0; c < RBD_MAX_D / kWave; ++c) h2acc[c] = 0.0;
            double q = 0.0;
            for (int i = r0 + wave; i < r1; i += kLoopThreads / kWave) {
                double* yrow = out.Y + (int64_t)i * d_max;
                double y[RBD_MAX_D / kWave];
                double g = 0.0;
#pragma unroll
                for (int c = 0; c < RBD_MAX_D / kWave; ++c) {
                    const int k = lane + c * kWave;
                    y[c] = (c * kWave < dl && k < dl) ? ld_dev(yrow + k) : 0.0;
                    if (pending && k < dl) g = fma(y[c], s_h2[k], g);
                }
                if (pending) {
                    g = wave_sum(g);
                    const double xi = (s_v1own[i - r0] - g) * inv_prev;
                    const int k = d - 1;
                    if (lane == (k & (kWave - 1))) {
                        st_dev(yrow + k, xi);
                        y[k / kWave] = xi;
                    }
                    // lanes other than k's hold 0 in that slot already
                }
                double dot = 0.0;
#pragma unroll
                for (int c = 0; c < RBD_MAX_D / kWave; ++c) {
                    const int k = lane + c * kWave;
                    if (k < d) dot = fma(y[c], s_h1[k], dot);
                }
                dot = wave_sum(dot);
                const double v = L::one(X + (int64_t)i * ldx + p) - dot;
#pragma unroll
                for (int c = 0; c < RBD_MAX_D / kWave; ++c) h2acc[c] = fma(y[c], v, h2acc[c]);
                if (lane == 0) {
                    s_v1own[i - r0] = v;
                    st_dev(ws.v1 + i, v);
                    q = fma(v, v, q);
                }
            }
            pending = false;
#pragma unroll
            for (int c = 0; c < RBD_MAX_D / kWave; ++c) {
                const int k = lane + c * kWave;
                if (k < d) s_red[wave * (RBD_MAX_D + 1) + k] = h2acc[c];
            }
            if (lane == 0) s_red[wave * (RBD_MAX_D + 1) + d] = q;
            __syncthreads();
            for (int k = tid; k <= d; k += kLoopThreads) {
                double s = s_red[k];
                for (int u = 1; u < kLoopThreads / kWave; ++u) s += s_red[u * (RBD_MAX_D + 1) + k];
                st_dev(ws.part + (int64_t)w * D1 + k, s);
            }
        }
        alive = loop_sync(ws, target, &s_flag);
        if (!alive) break;

        // ---- B: h2, nu, break test; T(d, own columns), downdate, local argmax ----
        for (int k = tid; k <= d; k += kLoopThreads) {
            double s = 0.0;
            for (int c = 0; c < Gc; ++c) s += ld_dev(ws.part + (int64_t)c * D1 + k);
            s_h2[k] = s;
        }
        __syncthreads();
        double hh = 0.0;
        for (int k = tid; k < d; k += kLoopThreads) hh = fma(s_h2[k], s_h2[k], hh);
        hh = block_sum(hh, sv);
        const double nu2 = s_h2[d] - hh;
        const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
        if (nu < tau || nu == 0.0) {
            stop = RBD_STOP_BREAK;
            break;
        }
        nu_prev = nu;
        pending = true;
        {
            double acc = 0.0;
            const Tx* xc = X + c0 + col;
            for (int base = 0; base < m; base += kLoopChunk) {
                const int len = min(kLoopChunk, m - base);
                __syncthreads();
                for (int i = tid; i < len; i += kLoopThreads) s_vc[i] = ld_dev(ws.v1 + base + i);
                __syncthreads();
                if (col < nc) {
#pragma unroll 8
                    for (int i = rsub; i < len; i += rpi) acc = fma(s_vc[i], L::one(xc + (int64_t)(base + i) * ldx), acc);
                }
            }
            double corr = 0.0;
            if (col < nc) {
                for (int k = rsub; k < d; k += rpi) corr = fma(s_h2[k], ld_dev(out.T + (int64_t)k * n + c0 + col), corr);
            }
            __syncthreads();
            s_red[tid] = acc;
            s_red[kLoopThreads + tid] = corr;
            __syncthreads();
        }
        double best = -1.0, flagged = 0.0;
        int64_t bi = INT64_MAX;
        if (tid < nc) {
            double a = 0.0, c = 0.0;
            for (int q = 0; q < rpi; ++q) {
                a += s_red[q * CW + tid];
                c += s_red[kLoopThreads + q * CW + tid];
            }
            const int j = c0 + tid;
            const double t = (a - c) / nu;
            st_dev(out.T + (int64_t)d * n + j, t);
            s_tcol[tid] = t;
            double e = s_e2[tid] - t * t;
            if (!(e > 0.0)) e = 0.0;
            double b = s_b2[tid];
            if (j == p) {
                e = 0.0;
                b = 0.0;
                s_b2[tid] = 0.0;
            }
            s_e2[tid] = e;
            if (e < kRefresh * b) flagged = 1.0;
            best = e;
            bi = j;
        }
        flagged = block_sum(flagged, sv);
        block_argmax(best, bi, sv, si);
        if (tid == 0) {
            st_dev(ws.bval + set * G + w, best);
            st_dev(ws.bidx + set * G + w, bi);
            st_dev(ws.bcnt + set * G + w, flagged);
        }
        alive = loop_sync(ws, target, &s_flag);
        if (!alive) break;

        // ---- C: merge; exact refresh when flagged; pivot, E_d, stop test ----
        double vmax, cnt;
        int64_t imax;
        loop_merge(ws, set, vmax, imax, cnt, sv, si);
        set ^= 1;
        if (cnt > 0.0) {
            if (tid == 0) {
                int nq = 0;
                for (int c = 0; c < nc; ++c)
                    if (s_e2[c] < kRefreshEager * s_b2[c]) s_list[nq++] = c;
                s_nq = nq;
            }
            __syncthreads();
            const int nq = s_nq;
            const double inv_nu = 1.0 / nu;
            for (int q0 = 0; q0 < nq; q0 += kLoopRefCols) {
                const int nch = min(kLoopRefCols, nq - q0);
                __syncthreads();
                for (int e = tid; e < nch * (d + 1); e += kLoopThreads) {
                    const int c = e / (d + 1), k = e % (d + 1);
                    s_tq[c * (RBD_MAX_D + 1) + k] = ld_dev(out.T + (int64_t)k * n + c0 + s_list[q0 + c]);
                }
                __syncthreads();
                double acc[kLoopRefCols];
#pragma unroll
                for (int c = 0; c < kLoopRefCols; ++c) acc[c] = 0.0;
                for (int i = tid; i < m; i += kLoopThreads) {
                    const double* yrow = out.Y + (int64_t)i * d_max;
                    double a[kLoopRefCols];
#pragma unroll
                    for (int c = 0; c < kLoopRefCols; ++c) a[c] = 0.0;
                    double g = 0.0;
                    for (int k = 0; k < d; ++k) {
                        const double y = ld_dev(yrow + k);
                        g = fma(y, s_h2[k], g);
#pragma unroll
                        for (int c = 0; c < kLoopRefCols; ++c) a[c] = fma(y, s_tq[c * (RBD_MAX_D + 1) + k], a[c]);
                    }
                    const double xi = (ld_dev(ws.v1 + i) - g) * inv_nu;     // the pending column Y(i, d)
#pragma unroll
                    for (int c = 0; c < kLoopRefCols; ++c) {
                        if (c < nch) {
                            const double r = L::one(X + (int64_t)i * ldx + c0 + s_list[q0 + c]) - a[c] -
                                             xi * s_tq[c * (RBD_MAX_D + 1) + d];
                            acc[c] = fma(r, r, acc[c]);
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int c = 0; c < kLoopRefCols; ++c) s_red[c * kLoopThreads + tid] = acc[c];
                __syncthreads();
                if (tid < nch) {
                    double s = 0.0;
                    for (int u = 0; u < kLoopThreads; ++u) s += s_red[tid * kLoopThreads + u];
                    const int c = s_list[q0 + tid];
                    s_e2[c] = s;
                    s_b2[c] = s;
                }
            }
            __syncthreads();
            double best2 = -1.0;
            int64_t bi2 = INT64_MAX;
            if (tid < nc) {
                best2 = s_e2[tid];
                bi2 = c0 + tid;
            }
            block_argmax(best2, bi2, sv, si);
            if (tid == 0) {
                st_dev(ws.bval + set * G + w, best2);
                st_dev(ws.bidx + set * G + w, bi2);
                st_dev(ws.bcnt + set * G + w, 0.0);
            }
            alive = loop_sync(ws, target, &s_flag);
            if (!alive) break;
            loop_merge(ws, set, vmax, imax, cnt, sv, si);
            set ^= 1;
        }
        const double E = sqrt(vmax);
        if (w == 0 && tid == 0) {
            out.pivots[d] = p;
            out.err_hist[d + 1] = E;
        }
        d += 1;
        p = (int)imax;
        if (E <= tau) stop = RBD_STOP_TOL;
        else if (d >= D) stop = RBD_STOP_DMAX;
    }
    if (!alive) {
        status = RBD_EDEVICE;
        stop = kStopError;
    }

    // ---- epilogue: the pending basis column, final errors, zero fill, d ----
    if (alive && pending && gs) {
        const double inv_prev = 1.0 / nu_prev;
        const int dl = d - 1;
        for (int i = r0 + wave; i < r1; i += kLoopThreads / kWave) {
            double* yrow = out.Y + (int64_t)i * d_max;
            double g = 0.0;
            for (int k = lane; k < dl; k += kWave) g = fma(ld_dev(yrow + k), s_h2[k], g);
            g = wave_sum(g);
            if (lane == 0) st_dev(yrow + dl, (s_v1own[i - r0] - g) * inv_prev);
        }
    }
    const int dfin = (status == RBD_OK) ? d : 0;
    if (tid < nc) out.col_err[c0 + tid] = status == RBD_OK ? sqrt(s_e2[tid]) : NAN;
    for (int e = tid; e < (d_max - dfin) * nc; e += kLoopThreads) {
        const int k = dfin + e / nc, c = e % nc;
        out.T[(int64_t)k * n + c0 + c] = 0.0;
    }
    if (gs) {
        for (int e = tid; e < (r1 - r0) * (d_max - dfin); e += kLoopThreads) {
            const int i = r0 + e / (d_max - dfin), k = dfin + e % (d_max - dfin);
            out.Y[(int64_t)i * d_max + k] = 0.0;
        }
    }
    if (w == 0) {
        for (int k = dfin + tid; k < d_max; k += kLoopThreads) out.pivots[k] = -1;
        for (int k = dfin + 1 + tid; k <= d_max; k += kLoopThreads) out.err_hist[k] = 0.0;
        if (tid == 0) {
            *out.d_out = dfin;
            *out.status = status;
            if (out.stop_reason) *out.stop_reason = (stop == kStopError) ? 0 : stop;
        }
    }
}

}  // namespace rbd
