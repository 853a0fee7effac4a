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
//      flagged, every column below kRefreshEager of its last exact value (each
//      workgroup publishes its own in step B) is re-evaluated exactly:
//      every workgroup sums ||x_j - Y T(:, j)||^2 over a block of rows for all
//      queued columns (the pending column xi_d formed on the fly), and after
//      a barrier the owners add the blocks' partial sums in a fixed order;
//      the maxima are merged again (a third barrier).  Then pivot, E_d and
//      the stop test of 2.4.
// Every workgroup takes the same decisions from the same data, so the loop
// ends in all of them at the same step.
//
// Memory: data one workgroup writes and another reads (Gram-Schmidt partials,
// v1, the partial maxima, T(:, p), rows of Y in a refresh) move through
// device-scope loads and stores, which are coherent across the XCDs' L2
// caches without cache write-backs or invalidations; a barrier waits for the
// workgroup's stores, then counts on a device-scope atomic.  A workgroup
// reads what it wrote itself (its rows of Y, its columns of T) with ordinary
// loads, and X, which is never written, too: each XCD keeps its workgroups'
// columns of X in its L2 from step to step (workgroups of one XCD own
// adjacent column slices).  Every phase issues its loads in batches before
// using them: the steps are latency-bound.  Every barrier wait is bounded in
// time: past the limit the workgroup raises the abort flag, every workgroup
// leaves the loop, and the fit reports RBD_EDEVICE in *status.
#pragma once

#include "rbd_device.h"

namespace rbd {

constexpr int kLoopThreads = 256;
constexpr int kLoopWaves = kLoopThreads / kWave;
constexpr int kLoopMaxCW = 64;            // columns per workgroup
constexpr int kLoopMaxRB = 1024;          // rows per Gram-Schmidt workgroup
constexpr int kLoopChunk = 2048;          // rows of v1 staged in LDS per pass of the scan
constexpr int kLoopRefCols = 8;           // s_tq holds kLoopRefCols * (RBD_MAX_D + 1) values of T
constexpr int kLoopRefRows = 512;         // rows of Y staged per pass of an exact refresh (at most)
constexpr int kLoopMaxG = 256;            // workgroups
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
    int* qcnt;            // G: columns each workgroup queues for an exact refresh this step
    int* qlist;           // G x CW: their indices
    double* rpart;        // G x n: per row block, the refresh sums of the queued columns
};

// Fixed-order sum over s of red[s * W + c] (S a power of two) into red[c]:
// pairwise halving, the same pairing for every column.
__device__ __forceinline__ void tree_rows(double* red, int S, int W) {
    for (int h = S / 2; h >= 1; h >>= 1) {
        __syncthreads();
        for (int e = threadIdx.x; e < h * W; e += kLoopThreads) red[e] += red[e + h * W];
    }
    __syncthreads();
}

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
    const int q = threadIdx.x;
    if (q < G) {
        v = ld_dev(ws.bval + set * G + q);
        i = ld_dev(ws.bidx + set * G + q);
        c = ld_dev(ws.bcnt + set * G + q);
    }
    cnt = block_sum(c, sv);
    block_argmax(v, i, sv, si);
}

// Column sums for the workgroup's columns c0 .. c0 + nc - 1 over all m rows:
// SQR: acc_c = sum_i x_ic^2; DOT: acc_c = sum_i vs[i - base] x_ic with v1
// staged in LDS chunk by chunk.  16-byte loads (V elements) with eight rows
// in flight per thread; LPR threads cover a row's CW columns.  Each thread's
// V sums go to red[sub * CW + column] for a fixed-order sum over sub.
template <typename Tx, bool DOT>
__device__ __forceinline__ void loop_scan(const Tx* __restrict__ X, int64_t ldx, int m, int c0, int nc, int CW,
                                          bool vec_ok, const double* __restrict__ v1g, double* vs, double* red,
                                          int& rpp_out, bool staged0 = false) {
    using L = Ld<Tx>;
    using R = typename L::raw;
    constexpr int V = L::N;
    const int tid = threadIdx.x;
    if (vec_ok && CW >= V) {
        const int lpr = CW / V, rpp = kLoopThreads / lpr;
        const int cg = tid % lpr, sub = tid / lpr;
        const int cc = c0 + cg * V;
        const bool full = cg * V + V <= nc;
        const bool any = cg * V < nc;
        double acc[V];
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] = 0.0;
        for (int base = 0; base < m; base += DOT ? kLoopChunk : m) {
            const int len = DOT ? min(kLoopChunk, m - base) : m;
            if (DOT && !(staged0 && base == 0)) {
                __syncthreads();
                constexpr int kB = kLoopChunk / kLoopThreads;
                double t[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const int i = tid + u * kLoopThreads;
                    t[u] = i < len ? ld_dev(v1g + base + i) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kB; ++u) vs[tid + u * kLoopThreads] = t[u];
                __syncthreads();
            }
            if (full) {
                constexpr int U = 16;
                for (int i0 = sub; i0 < len; i0 += U * rpp) {
                    R r[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int i = min(i0 + u * rpp, len - 1);      // clamped rows are loaded, not used
                        r[u] = *reinterpret_cast<const R*>(X + (int64_t)(base + i) * ldx + cc);
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int i = i0 + u * rpp;
                        double x[V];
                        L::cvt(r[u], x);
                        const double a = i < len ? (DOT ? vs[i] : 1.0) : 0.0;
#pragma unroll
                        for (int e = 0; e < V; ++e) acc[e] = fma(a * (DOT ? 1.0 : x[e]), x[e], acc[e]);
                    }
                }
            } else if (any) {
                for (int i = sub; i < len; i += rpp) {
                    const double a = DOT ? vs[i] : 1.0;
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        if (cg * V + e < nc) {
                            const double x = L::one(X + (int64_t)(base + i) * ldx + cc + e);
                            acc[e] = fma(a * (DOT ? 1.0 : x), x, acc[e]);
                        }
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < V; ++e) red[sub * CW + cg * V + e] = acc[e];
        rpp_out = rpp;
    } else {
        const int col = tid % CW, sub = tid / CW, rpp = kLoopThreads / CW;
        double acc = 0.0;
        for (int base = 0; base < m; base += DOT ? kLoopChunk : m) {
            const int len = DOT ? min(kLoopChunk, m - base) : m;
            if (DOT && !(staged0 && base == 0)) {
                __syncthreads();
                constexpr int kB = kLoopChunk / kLoopThreads;
                double t[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const int i = tid + u * kLoopThreads;
                    t[u] = i < len ? ld_dev(v1g + base + i) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kB; ++u) vs[tid + u * kLoopThreads] = t[u];
                __syncthreads();
            }
            if (col < nc) {
                const Tx* xc = X + c0 + col;
                constexpr int U = 8;
                for (int i0 = sub; i0 < len; i0 += U * rpp) {
                    double x[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) x[u] = L::one(xc + (int64_t)(base + min(i0 + u * rpp, len - 1)) * ldx);
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int i = i0 + u * rpp;
                        const double a = i < len ? (DOT ? vs[i] : x[u]) : 0.0;
                        acc = fma(a, x[u], acc);
                    }
                }
            }
        }
        __syncthreads();
        red[sub * CW + col] = acc;
        rpp_out = rpp;
    }
    __syncthreads();
}

// Step A on rows [r0, r1) of this Gram-Schmidt workgroup: write the pending
// basis column Y(:, d-1) (when `pending`), then v1 = x_p - Y(:, 0:d) h1 with
// h1 = T(0:d, p) (loaded by every wave for its own lanes, with the first
// rows of Y), and per-wave partials of h2 = Y' v1 (into red, one row of
// RBD_MAX_D + 1 per wave) and ||v1||^2 (at index d).  One wave per row, lanes
// along the columns of Y, RU rows in flight (RU * KC <= 32).
template <typename Tx, int KC>
__device__ __forceinline__ void loop_gs(const Tx* __restrict__ X, int64_t ldx, int p, double* __restrict__ Y,
                                        const double* __restrict__ T, int n, int d_max, int d, bool pending,
                                        double inv_prev, int r0, int r1, const double* s_h2, double* s_v1own,
                                        double* __restrict__ v1g, double* red) {
    constexpr int RU = (32 / KC) > 16 ? 16 : (32 / KC < 1 ? 1 : 32 / KC);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int dl = pending ? d - 1 : d;              // columns of Y already written
    const int cl = pending ? (d - 1) / kWave : -1, ll = pending ? (d - 1) % kWave : 0;
    double h1[KC], h2p[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
        const int k = lane + kWave * c;
        h1[c] = k < d ? ld_dev(T + (int64_t)k * n + p) : 0.0;
        h2p[c] = k < dl ? s_h2[k] : 0.0;
    }
    double acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = 0.0;
    double nacc = 0.0;
    for (int rb = r0 + wave * RU; rb < r1; rb += kLoopWaves * RU) {
        const int rl = rb + lane;
        const bool okl = lane < RU && rl < r1;
        const double xl = okl ? Ld<Tx>::one(X + (int64_t)rl * ldx + p) : 0.0;
        const double vl = (okl && pending) ? s_v1own[rl - r0] : 0.0;
        double y[RU][KC];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int r = min(rb + u, r1 - 1);                 // clamped rows: loaded, not used
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const int k = lane + kWave * c;
                y[u][c] = k < dl ? Y[(int64_t)r * d_max + k] : 0.0;
            }
        }
        // h1 of the pending column, from the lane that holds it
        double hsel = 0.0;
#pragma unroll
        for (int c = 0; c < KC; ++c)
            if (c == cl) hsel = h1[c];
        const double hl = pending ? lane_bcast(hsel, ll) : 0.0;
        double da[RU], db[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                a = fma(y[u][c], h2p[c], a);
                b = fma(y[u][c], h1[c], b);
            }
            da[u] = a;
            db[u] = b;
        }
        if (pending) wave_sum_n<RU>(da);
        wave_sum_n<RU>(db);
        double vo = 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const bool ok = rb + u < r1;
            const double yl = pending ? (lane_bcast(vl, u) - da[u]) * inv_prev : 0.0;
            const double v = lane_bcast(xl, u) - db[u] - yl * hl;
#pragma unroll
            for (int c = 0; c < KC; ++c)
                if (c == cl && lane == ll) {
                    y[u][c] = ok ? yl : 0.0;
                    if (ok) st_dev(Y + (int64_t)(rb + u) * d_max + d - 1, yl);
                }
            if (ok) {
#pragma unroll
                for (int c = 0; c < KC; ++c) acc[c] = fma(y[u][c], v, acc[c]);
            }
            if (lane == u) vo = v;
        }
        if (okl) {
            s_v1own[rl - r0] = vo;
            st_dev(v1g + rl, vo);
            nacc = fma(vo, vo, nacc);
        }
    }
    nacc = wave_sum(nacc);
#pragma unroll
    for (int c = 0; c < KC; ++c) {
        const int k = lane + kWave * c;
        if (k < d) red[wave * (RBD_MAX_D + 1) + k] = acc[c];
    }
    if (lane == 0) red[wave * (RBD_MAX_D + 1) + d] = nacc;
}

template <typename Tx>
__global__ __launch_bounds__(kLoopThreads) void loop_kernel(const Tx* __restrict__ X, int64_t ldx, int m, int n,
                                                            int D, int d_max, double tol, int rel, int64_t start,
                                                            LoopOut out, LoopWs ws, int Gc, int RB, int CW,
                                                            int vec_ok) {
    using L = Ld<Tx>;
    const int G = gridDim.x, w = blockIdx.x, tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int D1 = D + 1;

    __shared__ double s_h2[RBD_MAX_D + 1];          // h2 and ||v1||^2 of the last step
    __shared__ double s_v1own[kLoopMaxRB];          // v1 on this workgroup's Gram-Schmidt rows
    __shared__ double s_vc[kLoopChunk];             // v1 staged for the scan
    __shared__ double s_e2[kLoopMaxCW], s_b2[kLoopMaxCW];
    __shared__ double s_red[4 * (RBD_MAX_D + 1)];   // per-wave partial rows; scan partials
    __shared__ double s_tq[kLoopRefCols * (RBD_MAX_D + 1)];   // refresh: T(0:d+1, queued columns)
    __shared__ double s_xi[kLoopRefRows];           // refresh: the pending column on the row chunk
    __shared__ int s_qoff[kLoopMaxG + 1];           // refresh: queue offsets of the workgroups
    __shared__ int s_jq[4 * kLoopThreads];          // refresh: the columns of a pass
    __shared__ int s_list[kLoopMaxCW];
    __shared__ int s_flag, s_nq;
    __shared__ double sv[4];
    __shared__ int64_t si[4];

    // XCD-aware column slice: consecutive workgroup indices go to different
    // XCDs, so the G / 8 workgroups of one XCD own adjacent slices.
    const int slice = (G % 8 == 0) ? (w % 8) * (G / 8) + w / 8 : w;
    const int c0 = slice * CW;
    const int nc = max(0, min(n - c0, CW));
    const bool gs = w < Gc;
    const int r0 = w * RB, r1 = gs ? min(m, r0 + RB) : r0;
    unsigned target = 0;

    // ---- pre-computation of diag(X'X) (section 3.3): e_j^2 = ||x_j||^2 ----
    {
        int rpp = 1;
        loop_scan<Tx, false>(X, ldx, m, c0, nc, CW, vec_ok != 0, nullptr, s_vc, s_red, rpp);
        tree_rows(s_red, rpp, CW);
        double best = -1.0, nonfin = 0.0;
        int64_t bi = INT64_MAX;
        if (tid < nc) {
            const double s = s_red[tid];
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
    const int RBr = (m + G - 1) / G;                 // rows per workgroup in an exact refresh
    const int rr0 = min(m, w * RBr), rr1 = min(m, rr0 + RBr);
    while (alive && !stop && d < D) {
        // ---- A: lagged basis column, v1 = x_p - Y(:, 0:d) T(0:d, p), partials ----
        if (gs) {
            const double inv_prev = pending ? 1.0 / nu_prev : 0.0;
            const int kc = d <= 64 ? 1 : d <= 128 ? 2 : d <= 256 ? 4 : d <= 512 ? 8 : 16;
#define RBD_LOOP_GS(K)                                                                                          \
    loop_gs<Tx, K>(X, ldx, p, out.Y, out.T, n, d_max, d, pending, inv_prev, r0, r1, s_h2, s_v1own, ws.v1, s_red)
            switch (kc) {
                case 1: RBD_LOOP_GS(1); break;
                case 2: RBD_LOOP_GS(2); break;
                case 4: RBD_LOOP_GS(4); break;
                case 8: RBD_LOOP_GS(8); break;
                default: RBD_LOOP_GS(16); break;
            }
#undef RBD_LOOP_GS
            pending = false;
            __syncthreads();
            for (int k = tid; k <= d; k += kLoopThreads) {
                double sum = s_red[k];
                for (int u = 1; u < kLoopWaves; ++u) sum += s_red[u * (RBD_MAX_D + 1) + k];
                st_dev(ws.part + (int64_t)w * D1 + k, sum);
            }
        }
        alive = loop_sync(ws, target, &s_flag);
        if (!alive) break;

        // ---- B: h2, nu, break test; T(d, own columns), downdate, queue, local argmax ----
        {
            // v1's first chunk and the partials of h2 are loaded together
            constexpr int kB = kLoopChunk / kLoopThreads;
            const int len0 = min(kLoopChunk, m);
            double tv[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int i = tid + u * kLoopThreads;
                tv[u] = i < len0 ? ld_dev(ws.v1 + i) : 0.0;
            }
            for (int k = tid; k <= d; k += kLoopThreads) {
                constexpr int kP = 16;
                double sum = 0.0;
                for (int cg = 0; cg < Gc; cg += kP) {
                    double t[kP];
#pragma unroll
                    for (int u = 0; u < kP; ++u) t[u] = cg + u < Gc ? ld_dev(ws.part + (int64_t)(cg + u) * D1 + k) : 0.0;
#pragma unroll
                    for (int u = 0; u < kP; ++u) sum += t[u];
                }
                s_h2[k] = sum;
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) s_vc[tid + u * kLoopThreads] = tv[u];
            __syncthreads();
        }
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
        // correction h2' T(0:d, j) for the own columns (own rows of T: ordinary loads)
        double corr = 0.0;
        {
            const int col = tid % CW, rsub = tid / CW, rpi = kLoopThreads / CW;
            if (col < nc) {
                constexpr int U = 8;
                for (int k0 = rsub; k0 < d; k0 += U * rpi) {
                    double t[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int k = min(k0 + u * rpi, d - 1);
                        t[u] = out.T[(int64_t)k * n + c0 + col];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (k0 + u * rpi < d) corr = fma(s_h2[k0 + u * rpi], t[u], corr);
                }
            }
        }
        int rpp = 1;
        loop_scan<Tx, true>(X, ldx, m, c0, nc, CW, vec_ok != 0, ws.v1, s_vc, s_red, rpp, true);
        s_red[8 * kLoopThreads + tid] = corr;         // past the scan's partials (at most 8 x 256)
        tree_rows(s_red, rpp, CW);
        tree_rows(s_red + 8 * kLoopThreads, kLoopThreads / CW, CW);
        double best = -1.0, flagged = 0.0;
        int64_t bi = INT64_MAX;
        bool queued = false;
        if (tid < nc) {
            const int j = c0 + tid;
            const double t = (s_red[tid] - s_red[8 * kLoopThreads + tid]) / nu;
            st_dev(out.T + (int64_t)d * n + j, t);
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
            queued = e < kRefreshEager * b;
            best = e;
            bi = j;
        }
        // this workgroup's refresh queue (its columns are threads of wave 0)
        if (wave == 0) {
            const unsigned long long mask = __ballot(queued);
            if (queued) {
                const int pos = __popcll(mask & ((1ull << lane) - 1ull));
                s_list[pos] = tid;
                st_dev(ws.qlist + w * CW + pos, c0 + tid);
            }
            if (lane == 0) {
                s_nq = __popcll(mask);
                st_dev(ws.qcnt + w, (int)__popcll(mask));
            }
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
            // queue offsets of the workgroups (exclusive prefix in workgroup order)
            if (tid < G) s_qoff[tid + 1] = ld_dev(ws.qcnt + tid);
            __syncthreads();
            if (tid == 0) {
                s_qoff[0] = 0;
                for (int q = 1; q <= G; ++q) s_qoff[q] += s_qoff[q - 1];
            }
            __syncthreads();
            const int nq = s_qoff[G];
            // R1: this workgroup's rows [rr0, rr1) against every queued column
            const double inv_nu = 1.0 / nu;
            const int d1 = d + 1;
            const int cq = min(kLoopRefCols * (RBD_MAX_D + 1) / d1, 4 * kLoopThreads);   // columns per pass
            const int rc = min(kLoopRefRows, 4 * (RBD_MAX_D + 1) / d1);                  // rows per pass
            for (int q0 = 0; q0 < nq; q0 += cq) {
                const int nqc = min(cq, nq - q0);
                // the pass's column indices (owner by binary search over the offsets), then T(0:d+1, j)
                __syncthreads();
                for (int qq = tid; qq < nqc; qq += kLoopThreads) {
                    const int gq = q0 + qq;
                    int lo = 0, hi = G - 1;                       // largest wq with s_qoff[wq] <= gq
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) / 2;
                        if (s_qoff[mid] <= gq) lo = mid;
                        else hi = mid - 1;
                    }
                    s_jq[qq] = ld_dev(ws.qlist + lo * CW + (gq - s_qoff[lo]));
                }
                __syncthreads();
                for (int e0 = tid; e0 < nqc * d1; e0 += 8 * kLoopThreads) {       // eight loads in flight
                    double t[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = min(e0 + u * kLoopThreads, nqc * d1 - 1);
                        t[u] = ld_dev(out.T + (int64_t)(e % d1) * n + s_jq[e / d1]);
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + u * kLoopThreads;
                        if (e < nqc * d1) s_tq[(e / d1) * d1 + e % d1] = t[u];
                    }
                }
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                int jcol[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int qq = tid + u * kLoopThreads;
                    jcol[u] = qq < nqc ? s_jq[qq] : -1;
                }
                for (int ra = rr0; ra < rr1; ra += rc) {
                    const int nr = min(rc, rr1 - ra);
                    // rows of Y (other workgroups wrote them) into s_red, then the pending column
                    __syncthreads();
                    for (int e0 = tid; e0 < nr * d; e0 += 8 * kLoopThreads) {
                        double t[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int e = min(e0 + u * kLoopThreads, nr * d - 1);
                            t[u] = ld_dev(out.Y + (int64_t)(ra + e / d) * d_max + e % d);
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int e = e0 + u * kLoopThreads;
                            if (e < nr * d) s_red[(e / d) * d1 + e % d] = t[u];
                        }
                    }
                    __syncthreads();
                    for (int i = tid; i < nr; i += kLoopThreads) {
                        double g = 0.0;
                        for (int k = 0; k < d; ++k) g = fma(s_red[i * d1 + k], s_h2[k], g);
                        s_xi[i] = (ld_dev(ws.v1 + ra + i) - g) * inv_nu;
                    }
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int qq = tid + u * kLoopThreads;
                        if (jcol[u] >= 0) {
                            const double* tq = s_tq + qq * d1;
                            for (int i0 = 0; i0 < nr; i0 += 8) {
                                double x[8];
#pragma unroll
                                for (int v = 0; v < 8; ++v)
                                    x[v] = L::one(X + (int64_t)(ra + min(i0 + v, nr - 1)) * ldx + jcol[u]);
#pragma unroll
                                for (int v = 0; v < 8; ++v) {
                                    const int i = i0 + v;
                                    if (i < nr) {
                                        double a = 0.0;
                                        for (int k = 0; k < d; ++k) a = fma(s_red[i * d1 + k], tq[k], a);
                                        const double r = x[v] - a - s_xi[i] * tq[d];
                                        acc[u] = fma(r, r, acc[u]);
                                    }
                                }
                            }
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int qq = tid + u * kLoopThreads;
                    if (qq < nqc) st_dev(ws.rpart + (int64_t)w * n + q0 + qq, acc[u]);
                }
            }
            alive = loop_sync(ws, target, &s_flag);
            if (!alive) break;
            // R2: the owners add the row blocks' sums in workgroup order
            {
                const int own = s_nq, off = s_qoff[w];
                constexpr int kS = 4;                         // threads per queued column
                const int qi = tid / kS, part4 = tid % kS;
                double sum = 0.0;
                if (qi < own) {
                    constexpr int kP = 16;
                    for (int g0 = part4 * kP; g0 < G; g0 += kS * kP) {
                        double t[kP];
#pragma unroll
                        for (int u = 0; u < kP; ++u)
                            t[u] = g0 + u < G ? ld_dev(ws.rpart + (int64_t)(g0 + u) * n + off + qi) : 0.0;
#pragma unroll
                        for (int u = 0; u < kP; ++u) sum += t[u];
                    }
                }
                __syncthreads();
                s_red[tid] = sum;
                __syncthreads();
                if (tid < own) {
                    double e = 0.0;
                    for (int u = 0; u < kS; ++u) e += s_red[tid * kS + u];
                    const int c = s_list[tid];
                    s_e2[c] = e;
                    s_b2[c] = e;
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
        for (int i = r0 + wave; i < r1; i += kLoopWaves) {
            double* yrow = out.Y + (int64_t)i * d_max;
            double g = 0.0;
            for (int k = lane; k < dl; k += kWave) g = fma(yrow[k], s_h2[k], g);
            g = wave_sum(g);
            if (lane == 0) yrow[dl] = (s_v1own[i - r0] - g) * inv_prev;
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
