// Kernels of the greedy loop of Reduced Basis Decomposition (Algorithm 1,
// section 3.1) and of its A-norm variants (section 3.2, eq. (3)).  One greedy
// step is a fixed sequence of stream-ordered kernels; every kernel reads the
// device-side stop flag first, so steps past the end of the loop cost one
// empty launch each and the host never waits.
//
// A = I (lagged reorthogonalisation: one pass over Y per step):
//   gather_col    x_p into a contiguous FP64 vector
//   cgs1_lag      writes the previous step's basis column, then
//                 v1 = x_p - Y h1 with h1 = T(0:d, p) (h1 = Y' x_p is already a
//                 column of T), with per-block partials of h2 = Y' v1, ||v1||^2
//   reduce        h2 and ||v1||^2 = fixed-order sums (one or two small launches)
//   nu_tcorr      nu^2 = ||v1||^2 - ||h2||^2, step 2.2's break test, and the
//                 correction rows -h2' T(0:d, :) / nu
//   xscan         partial (v1 / nu)' X per row slab
//   reduce        slab partials (and correction rows) into group partials
//   update        T(d, :); e_j^2 -= T(d, j)^2; queue columns for an exact
//                 refresh; lowest-index argmax
//   ycol          the deferred basis column, when a refresh needs it
//   resid_mfma    exact ||x_j - Y T(:, j)||^2 of queued columns (FP64 MFMA)
//   resid_finish  store the exact values, argmax, stop test of step 2.4
// Diagonal A (two passes over Y per step, M = Y'WY kept up to date):
//   gather_col, cgs1w (v1, h2, a = Y'(w . v1), sum w v1^2), reduce x2,
//   mv (M h2), nuw (nu, break test, hw = Y'(W xi), ||xi||_A^2, new row of M),
//   gvec2 (Y(:, d) = xi, v2, g = w . xi - Y hw), xscan of xi and g,
//   reduce, update<kStepW> (e_j^2 -= 2 t_j g'x_j - t_j^2 ||xi||_A^2),
//   resid_mfma, resid_finish.
// General SPD A in CSR form (two passes over Y per step, M = Y'AY):
//   gather_col, cgs1 (v1, h2, ||v1||^2), reduce, nu_lag, spmv (u = A v1),
//   cgs2u (Y(:, d) = xi, v2, Y'u, v1'u), reduce, mv, nuw, spmv (A xi),
//   tcorr2 (rows -hw' T(0:d, :)), xscan of xi and A xi, reduce,
//   update<kStepW>; exact refreshes store residual chunks (resid_mfma in
//   store mode) and reduce r'Ar with csr_quad.
//
// Wide kernels (thousands of workgroups) never synchronise across the grid:
// a device-scope release fence per workgroup writes back the XCD's L2 and
// costs far more than a kernel boundary.  Grid-wide combination therefore
// happens in separate launches, and ticket counters (last workgroup to arrive
// finishes the job) are used only by kernels with a few dozen workgroups.
#pragma once

#include "rbd_device.h"

namespace rbd {


// kScanDot:  acc_j = sum_i xi_i x_ij            (xi = v2 / nu)
// kScanSqr:  acc_j = sum_i x_ij^2
// kScanSqrW: acc_j = sum_i w_i x_ij^2            (diagonal A; w passed as v2)
// kScanDot2: acc_j = sum_i xi_i x_ij and acc2_j = sum_i g_i x_ij (diagonal A)
enum { kScanDot = 0, kScanSqr = 1, kScanSqrW = 2, kScanDot2 = 3 };

// ---------------------------------------------------------------------------
__device__ __forceinline__ void finish_step(State* st, int d, double vmax, int64_t imax,
                                            int64_t* pivots, double* err_hist) {
    const double E = sqrt(vmax);
    pivots[d] = st->p;
    err_hist[d + 1] = E;
    st->d = d + 1;
    st->p = (int)imax;
    if (E <= st->tau) st->stop = RBD_STOP_TOL;
    else if (d + 1 >= st->D) st->stop = RBD_STOP_DMAX;
}

// ---------------------------------------------------------------------------
__global__ void init_state_kernel(State* st, unsigned* tickets, int ntickets, int D) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gid; i < ntickets; i += stride) tickets[i] = 0u;
    if (gid == 0) {
        st->d = 0; st->p = 0; st->stop = 0; st->status = RBD_OK; st->nflag = 0; st->D = D;
        st->nonfinite = 0; st->bad_index = 0;
        st->tau = 0.0; st->E0 = 0.0; st->nu = 0.0; st->inv_nu = 0.0; st->wxx = 0.0; st->pad1 = 0.0;
    }
}

// ---------------------------------------------------------------------------
// X-scan: per row slab, acc_j = sum_i w_i x_ij (DOT, w = xi) or sum_i x_ij^2
// (SQR).  Grid (column tiles, row slabs).  Each thread owns CH chunks of
// Ld<Tx>::N adjacent columns, blockDim * N columns apart, and streams the
// slab's rows with 16-byte loads, U rows in flight.  The slab's xi values are
// staged in LDS (every lane reads the same address: a broadcast).
// ---------------------------------------------------------------------------
template <typename Tx, int MODE, int U, bool NT, int CH>
__global__ __launch_bounds__(256) void xscan_kernel(const Tx* __restrict__ X, int64_t ldx, int64_t m,
                                                     int64_t n, const double* __restrict__ v2,
                                                     State* __restrict__ st, double* __restrict__ Y,
                                                     int64_t ldy, int dcol, int rows_per_slab,
                                                     double* __restrict__ part, int vec_ok,
                                                     const double* __restrict__ g2) {
    constexpr bool DOT = (MODE == kScanDot || MODE == kScanDot2);
    constexpr bool TWO = (MODE == kScanDot2);
    constexpr bool WTS = (MODE != kScanSqr);       // a per-row weight is staged in LDS
    if (DOT && st->stop) return;
    using L = Ld<Tx>;
    using R = typename L::raw;
    constexpr int N = L::N;
    extern __shared__ double xi_s[];               // rows_per_slab (x2 for kScanDot2)
    const int tile = blockIdx.x, slab = blockIdx.y;
    const int64_t r0 = (int64_t)slab * rows_per_slab;
    const int64_t r1 = min(m, r0 + (int64_t)rows_per_slab);
    const int nr = (int)(r1 - r0);
    if (WTS) {
        // eight rows per thread per round, every load issued before any value is
        // used (clamped rows past the slab's end are loaded and not stored)
        const double inv = DOT ? st->inv_nu : 1.0;
        constexpr int kSt = 8;
        for (int rb = threadIdx.x; rb < nr; rb += kSt * (int)blockDim.x) {
            double xv[kSt], gv[kSt];
#pragma unroll
            for (int u = 0; u < kSt; ++u) {
                const int64_t rr = r0 + min(rb + u * (int)blockDim.x, nr - 1);
                xv[u] = v2[rr];
                gv[u] = TWO ? g2[rr] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kSt; ++u) {
                const int r = rb + u * (int)blockDim.x;
                const double xi = xv[u] * inv;
                if (r < nr) {
                    xi_s[r] = xi;
                    if (TWO) xi_s[rows_per_slab + r] = gv[u];
                    if (DOT && dcol >= 0 && tile == 0) Y[(r0 + r) * ldy + dcol] = xi;
                }
            }
        }
        __syncthreads();
    }
    const int64_t cstep = (int64_t)blockDim.x * N;
    const int64_t cbase = (int64_t)tile * cstep * CH + (int64_t)threadIdx.x * N;
    // chunk q covers columns cbase + q*cstep .. +N-1: full (vector), partial (scalar) or empty
    bool full[CH];
    int ncols[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        const int64_t c = cbase + q * cstep;
        ncols[q] = (int)max((int64_t)0, min((int64_t)N, n - c));
        full[q] = vec_ok && ncols[q] == N;
    }
    double acc[CH][N];
    double acc2[TWO ? CH : 1][N];
#pragma unroll
    for (int q = 0; q < CH; ++q)
#pragma unroll
        for (int e = 0; e < N; ++e) acc[q][e] = 0.0;
#pragma unroll
    for (int q = 0; q < (TWO ? CH : 1); ++q)
#pragma unroll
        for (int e = 0; e < N; ++e) acc2[q][e] = 0.0;
    auto fold = [&](int q, const double* x, double w, double g) {
#pragma unroll
        for (int e = 0; e < N; ++e) {
            if (MODE == kScanSqr) acc[q][e] = fma(x[e], x[e], acc[q][e]);
            else if (MODE == kScanSqrW) acc[q][e] = fma(w * x[e], x[e], acc[q][e]);
            else acc[q][e] = fma(w, x[e], acc[q][e]);
            if (TWO) acc2[TWO ? q : 0][e] = fma(g, x[e], acc2[TWO ? q : 0][e]);
        }
    };
    const Tx* p = X + r0 * ldx + cbase;
    int r = 0;
    for (; r + U <= nr; r += U) {
        R raw[U][CH];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < CH; ++q)
                if (full[q]) {
                    const R* a = reinterpret_cast<const R*>(p + (int64_t)(r + u) * ldx + q * cstep);
                    raw[u][q] = NT ? __builtin_nontemporal_load(a) : *a;
                }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double w = WTS ? xi_s[r + u] : 0.0;
            const double g = TWO ? xi_s[rows_per_slab + r + u] : 0.0;
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                double x[N];
                if (full[q]) {
                    L::cvt(raw[u][q], x);
                } else {
#pragma unroll
                    for (int e = 0; e < N; ++e)
                        x[e] = e < ncols[q] ? L::one(p + (int64_t)(r + u) * ldx + q * cstep + e) : 0.0;
                }
                fold(q, x, w, g);
            }
        }
    }
    for (; r < nr; ++r) {
        const double w = WTS ? xi_s[r] : 0.0;
        const double g = TWO ? xi_s[rows_per_slab + r] : 0.0;
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            double x[N];
            if (full[q]) {
                L::cvt(*reinterpret_cast<const R*>(p + (int64_t)r * ldx + q * cstep), x);
            } else {
#pragma unroll
                for (int e = 0; e < N; ++e) x[e] = e < ncols[q] ? L::one(p + (int64_t)r * ldx + q * cstep + e) : 0.0;
            }
            fold(q, x, w, g);
        }
    }
    // partial rows: n values (acc), then n more (acc2) for kScanDot2
    const int64_t ldp = TWO ? 2 * n : n;
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        double* out = part + (int64_t)slab * ldp + cbase + q * cstep;
        for (int e = 0; e < ncols[q]; ++e) {
            out[e] = acc[q][e];
            if (TWO) out[n + e] = acc2[TWO ? q : 0][e];
        }
    }
}

// ---------------------------------------------------------------------------
// update: finish the column sums (slab groups, fixed order), then either
// initialise the errors (INIT) or downdate them (STEP), and take the
// lowest-index argmax.  One block per 256 columns; the last block to arrive
// combines the block maxima and closes the step.
// ---------------------------------------------------------------------------
// kStepW: diagonal A; l2 rows hold t_j (first n) and s_j = g' x_j (next n), and
// e_j^2 -= 2 t_j s_j - t_j^2 ||xi||_A^2.
enum { kInit = 0, kStep = 1, kStepW = 2 };

template <int MODE>
__global__ __launch_bounds__(256) void update_kernel(int64_t n, State* __restrict__ st, int d,
                                                      const double* __restrict__ l2, int SG,
                                                      unsigned* __restrict__ tickets,
                                                      double* __restrict__ e2, double* __restrict__ base2,
                                                      double* __restrict__ T, int64_t ldt,
                                                      int* __restrict__ flist,
                                                      double* __restrict__ bres_v, int64_t* __restrict__ bres_i,
                                                      int64_t* __restrict__ pivots, double* __restrict__ err_hist,
                                                      int64_t start, double tol, int rel) {
    constexpr bool STEP = (MODE != kInit);
    if (STEP && st->stop) return;
    __shared__ double sv[4];
    __shared__ int64_t si[4];
    const int cb = blockIdx.x, ncb = gridDim.x;
    const int64_t ldl = (MODE == kStepW) ? 2 * n : n;
    const int64_t j = (int64_t)cb * blockDim.x + threadIdx.x;

    double best = -1.0;
    int64_t bi = INT64_MAX;
    if (j < n) {
        double t = 0.0;
        // unrolled so that eight loads are in flight; the sum stays in ascending q
#pragma unroll 8
        for (int q = 0; q < SG; ++q) t += l2[(int64_t)q * ldl + j];
        double e;
        if (MODE == kInit) {
            e = t;
            e2[j] = e;
            base2[j] = e;
            if (!isfinite(e)) atomicOr(&st->nonfinite, 1);
        } else {
            T[(int64_t)d * ldt + j] = t;
            if (MODE == kStepW) {
                double sj = 0.0;
#pragma unroll 8
                for (int q = 0; q < SG; ++q) sj += l2[(int64_t)q * ldl + n + j];
                e = e2[j] - (2.0 * t * sj - t * t * st->wxx);
            } else {
                e = e2[j] - t * t;
            }
            if (!(e > 0.0)) e = 0.0;
            double b = base2[j];
            if (j == (int64_t)st->p) {
                e = 0.0;
                b = 0.0;
                base2[j] = 0.0;
            }
            e2[j] = e;
            if (e < kRefresh * b) atomicAdd(&st->nflag, 1);
        }
        if (e == e) { best = e; bi = j; }
    }
    block_argmax(best, bi, sv, si);
    if (threadIdx.x == 0) { bres_v[cb] = best; bres_i[cb] = bi; }
    if (!last_to_arrive(&tickets[ncb], (unsigned)ncb)) return;
    if (STEP && __hip_atomic_load(&st->nflag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0) {
        // Some column needs an exact refresh: queue every column whose
        // downdated e^2 is below kRefreshEager of its last exact value, so
        // the refreshes of columns that decay alike happen together (denser
        // gathers of X, fewer refresh steps).  Ascending order, so
        // neighbouring columns share the cache lines of X.
        __shared__ int scan[256];
        const int64_t per = (n + blockDim.x - 1) / blockDim.x;
        const int64_t a = (int64_t)threadIdx.x * per, b = min(n, a + per);
        int cnt = 0;
        for (int64_t c = a; c < b; ++c) cnt += (e2[c] < kRefreshEager * base2[c]);
        scan[threadIdx.x] = cnt;
        __syncthreads();
        for (int off = 1; off < (int)blockDim.x; off <<= 1) {
            const int add = (int)threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
            __syncthreads();
            scan[threadIdx.x] += add;
            __syncthreads();
        }
        int pos = scan[threadIdx.x] - cnt;
        for (int64_t c = a; c < b; ++c)
            if (e2[c] < kRefreshEager * base2[c]) flist[pos++] = (int)c;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) st->nflag = scan[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double v = -1.0;
        int64_t i = INT64_MAX;
        for (int c = 0; c < ncb; ++c) argmax_merge(v, i, bres_v[c], bres_i[c]);
        if (MODE == kInit) {
            if (st->bad_index) {
                st->status = RBD_EMATRIX;
                st->stop = kStopError;
                st->E0 = NAN;
                err_hist[0] = NAN;
            } else if (st->nonfinite) {
                st->status = RBD_ENONFINITE;
                st->stop = kStopError;
                st->E0 = NAN;
                err_hist[0] = NAN;
            } else {
                const double E0 = sqrt(v);
                st->E0 = E0;
                st->tau = rel ? tol * E0 : tol;
                st->p = start >= 0 ? (int)start : (int)i;
                err_hist[0] = E0;
            }
        } else if (st->nflag == 0) {
            finish_step(st, d, v, i, pivots, err_hist);
        }
    }
}

// ---------------------------------------------------------------------------
// gather_col: xp = X(:, p) widened to FP64 into a contiguous vector.  One row
// per thread, so the whole strided column is in flight at once.
// ---------------------------------------------------------------------------
template <typename Tx>
__global__ __launch_bounds__(256) void gather_col_kernel(const Tx* __restrict__ X, int64_t ldx, int64_t m,
                                                          const State* __restrict__ st, double* __restrict__ xp) {
    if (st->stop) return;
    const int64_t p = st->p;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += stride)
        xp[r] = Ld<Tx>::one(X + r * ldx + p);
}

// value of lane u (wave-uniform u) in every lane
__device__ __forceinline__ double lane_bcast(double v, int u) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), u);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), u);
    return __hiloint2double(hi, lo);
}

// Staged basis columns.  Writing one column of row-major Y costs a partial
// cache-line write per row (measured: a quarter of a Gram-Schmidt pass's time
// at m = 2^20), so a new column c goes to slot c % 8 of ys (m x 8,
// column-major, contiguous per slot) and reaches Y when its block of 8 is
// complete, as one 64-byte segment per row.  With c columns formed, columns
// below 8 floor(c / 8) are in Y and columns [8 floor(c / 8), c) only in ys;
// ys_flush / ycol copy the staged ones into Y wherever Y must be complete
// (before an exact refresh, after the loop).
template <typename Tb>
__device__ __forceinline__ const Tb* y_src(const Tb* Y, int64_t ldy, const Tb* ys, int64_t m, int64_t r, int k,
                                           int yb) {
    return k < yb ? Y + r * ldy + k : ys + (int64_t)min(k - yb, 7) * m + r;
}

// Entries (rb + u, lane + 64 c) of the basis for u < RU, c < KC, zero for rows
// >= r1 or columns >= cols.  FP64: loads under the bounds test (the compiler
// issues them all before the first use).  FP32: every load is issued from a
// clamped address (row min(r, r1 - 1); a column past the end reads staged
// slot 7 of that row) and the bounds test selects after the widening, since
// a widening inside the test would make each load wait for its data.
template <bool NT, int RU, int KC, typename Tb>
__device__ __forceinline__ void load_y_rows(double (&y)[RU][KC], const Tb* Y, int64_t ldy, const Tb* ys, int64_t m,
                                            int64_t rb, int64_t r1, int lane, int cols, int yb) {
    if constexpr (sizeof(Tb) == 8) {
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t r = rb + u;
            const bool ok = r < r1;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const int k = lane + kWave * c;
                y[u][c] = (ok && k < cols) ? (double)ld_y<NT>(y_src<Tb>(Y, ldy, ys, m, r, k, yb)) : 0.0;
            }
        }
    } else {
        Tb raw[RU][KC];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t r = min(rb + u, r1 - 1);
#pragma unroll
            for (int c = 0; c < KC; ++c) raw[u][c] = ld_y<NT>(y_src<Tb>(Y, ldy, ys, m, r, lane + kWave * c, yb));
        }
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const double v = (double)raw[u][c];
                y[u][c] = (rb + u < r1 && lane + kWave * c < cols) ? v : 0.0;
            }
    }
}

// ys_flush: copies the staged columns [8 floor(c / 8), c) into Y, with c the
// final d (FINAL) or c = cols before an exact refresh (skipped when none is
// queued).  Eight consecutive threads write the eight entries of one row.
template <bool FINAL>
__global__ __launch_bounds__(256) void ys_flush_kernel(double* __restrict__ Y, int64_t ldy, int64_t m,
                                                        const State* __restrict__ st, int cols,
                                                        const double* __restrict__ ys) {
    int c;
    if (FINAL) {
        if (st->stop == kStopError) return;
        c = st->d;
    } else {
        if (st->stop || st->nflag == 0) return;
        c = cols;
    }
    const int yb = c & ~7, nc = c - yb;
    if (nc <= 0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m * 8; t += stride) {
        const int64_t r = t >> 3;
        const int j = (int)(t & 7);
        if (j < nc) Y[r * ldy + yb + j] = ys[(int64_t)j * m + r];
    }
}

// ---------------------------------------------------------------------------
// cgs1: v1 = x_p - Y(:, 0:d) h1, h1 = T(0:d, p); per block the partials of
// h2 = Y' v1 (part[blk * ldp + k], k < d) and of ||v1||^2 (part[blk * ldp + d]).
// One wave per row of Y (lanes run along k), RU rows in flight per wave; the
// wave keeps its share of h2 in registers, so Y is read once.
// ---------------------------------------------------------------------------
template <int KC, int RU, bool NT>
__global__ __launch_bounds__(256) void cgs1_kernel(const double* __restrict__ xp, int64_t m,
                                                    const double* __restrict__ Y, int64_t ldy,
                                                    const double* __restrict__ T, int64_t ldt,
                                                    State* __restrict__ st, int d, int rows_per_blk,
                                                    const double* __restrict__ ys, double* __restrict__ v1,
                                                    double* __restrict__ part, int64_t ldp) {
    if (st->stop) return;
    constexpr int KW = kWave * KC;
    __shared__ double hs[KW];
    __shared__ double accs[KW];
    __shared__ double sred[4];
    const int p = st->p;
    for (int k = threadIdx.x; k < KW; k += blockDim.x) {
        hs[k] = (k < d) ? T[(int64_t)k * ldt + p] : 0.0;
        accs[k] = 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int yb = d & ~7;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min(m, r0 + (int64_t)rows_per_blk);
    double acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = 0.0;
    double nacc = 0.0;
    for (int64_t rb = r0 + (int64_t)w * RU; rb < r1; rb += (int64_t)nw * RU) {
        double y[RU][KC];
        double xv[RU];
        double dot[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t r = rb + u;
            const bool ok = r < r1;
            xv[u] = ok ? xp[r] : 0.0;
            dot[u] = 0.0;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const int k = lane + kWave * c;
                y[u][c] = (ok && k < d) ? ld_y<NT>(y_src(Y, ldy, ys, m, r, k, yb)) : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
            for (int c = 0; c < KC; ++c) dot[u] = fma(y[u][c], hs[lane + kWave * c], dot[u]);
        wave_sum_n<RU>(dot);
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const double v = xv[u] - dot[u];   // rows past the end have y = 0
#pragma unroll
            for (int c = 0; c < KC; ++c) acc[c] = fma(y[u][c], v, acc[c]);
            if (lane == u && rb + u < r1) {
                v1[rb + u] = v;
                nacc = fma(v, v, nacc);
            }
        }
    }
    const double nn = block_sum(nacc, sred);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * ldp + d] = nn;
    if (d == 0) return;
    for (int q = 0; q < nw; ++q) {
        if (w == q) {
#pragma unroll
            for (int c = 0; c < KC; ++c) accs[lane + kWave * c] += acc[c];
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < d; k += blockDim.x) part[(int64_t)blockIdx.x * ldp + k] = accs[k];
}

// ---------------------------------------------------------------------------
// Diagonal A = diag(w) with two passes over Y per step.  With M = Y'WY kept
// up to date (one new row and column per step), the second Gram-Schmidt pass
// and g = (I - YY')(W xi) need no pass of their own:
//   a  = Y'(w . v1),  hw = Y'(W xi) = (a - M h2) / nu,
//   ||xi||_A^2 = (sum w v1^2 - 2 h2'a + h2'M h2) / nu^2,  nu^2 = ||v1||^2 - ||h2||^2,
// and one pass forms v2 = v1 - Y h2, xi = v2 / nu (written to Y(:, d)) and
// g = w . xi - Y hw.  h2 is at rounding level after the first pass, so the
// corrections through M are tiny and M's own rounding does not matter.
// ---------------------------------------------------------------------------

// cgs1w: v1 = x_p - Y h1 as in cgs1, with per-block partials of h2 = Y'v1
// and ||v1||^2 (part[blk * ldp + k], k <= d) and of a = Y'(w . v1) and
// sum w v1^2 (the same layout, gridDim.x * ldp further on).
template <int KC, int RU, bool NT>
__global__ __launch_bounds__(256) void cgs1w_kernel(const double* __restrict__ xp, int64_t m,
                                                     const double* __restrict__ Y, int64_t ldy,
                                                     const double* __restrict__ T, int64_t ldt,
                                                     State* __restrict__ st, int d, int rows_per_blk,
                                                     const double* __restrict__ w, const double* __restrict__ ys,
                                                     double* __restrict__ v1, double* __restrict__ part,
                                                     int64_t ldp) {
    if (st->stop) return;
    constexpr int KW = kWave * KC;
    __shared__ double hs[KW];
    __shared__ double accs[KW];
    __shared__ double accw[KW];
    __shared__ double sred[4];
    const int p = st->p;
    for (int k = threadIdx.x; k < KW; k += blockDim.x) {
        hs[k] = (k < d) ? T[(int64_t)k * ldt + p] : 0.0;
        accs[k] = 0.0;
        accw[k] = 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int yb = d & ~7;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min(m, r0 + (int64_t)rows_per_blk);
    double acc[KC], acw[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = acw[c] = 0.0;
    double nacc = 0.0, wacc = 0.0;
    for (int64_t rb = r0 + (int64_t)wv * RU; rb < r1; rb += (int64_t)nw * RU) {
        double y[RU][KC];
        double xv[RU], wr[RU], dot[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t r = rb + u;
            const bool ok = r < r1;
            xv[u] = ok ? xp[r] : 0.0;
            wr[u] = ok ? w[r] : 0.0;
            dot[u] = 0.0;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const int k = lane + kWave * c;
                y[u][c] = (ok && k < d) ? ld_y<NT>(y_src(Y, ldy, ys, m, r, k, yb)) : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
            for (int c = 0; c < KC; ++c) dot[u] = fma(y[u][c], hs[lane + kWave * c], dot[u]);
        wave_sum_n<RU>(dot);
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const double v = xv[u] - dot[u];   // rows past the end have y = 0, x = 0, w = 0
            const double wvv = wr[u] * v;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                acc[c] = fma(y[u][c], v, acc[c]);
                acw[c] = fma(y[u][c], wvv, acw[c]);
            }
            if (lane == u && rb + u < r1) {
                v1[rb + u] = v;
                nacc = fma(v, v, nacc);
                wacc = fma(wvv, v, wacc);
            }
        }
    }
    const double nn = block_sum(nacc, sred);
    const double ww = block_sum(wacc, sred);
    double* p0 = part + (int64_t)blockIdx.x * ldp;
    double* p1 = part + (int64_t)gridDim.x * ldp + (int64_t)blockIdx.x * ldp;
    if (threadIdx.x == 0) {
        p0[d] = nn;
        p1[d] = ww;
    }
    if (d == 0) return;
    for (int q = 0; q < nw; ++q) {
        if (wv == q) {
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                accs[lane + kWave * c] += acc[c];
                accw[lane + kWave * c] += acw[c];
            }
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        p0[k] = accs[k];
        p1[k] = accw[k];
    }
}

// mv: Mh = M(0:d, 0:d) h2.  M is symmetric, so output k is the dot of row k
// (contiguous) with h2: one wave per output, lanes along the row.
__global__ __launch_bounds__(256) void mv_kernel(const State* __restrict__ st, const double* __restrict__ M,
                                                  int64_t ldm, int d, const double* __restrict__ h2,
                                                  double* __restrict__ Mh) {
    if (st->stop) return;
    const int lane = threadIdx.x % kWave;
    const int k = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (k >= d) return;                            // whole waves leave together
    const double* row = M + (int64_t)k * ldm;
    double s = 0.0;
    for (int j = lane; j < d; j += kWave) s = fma(row[j], h2[j], s);
    s = wave_sum(s);
    if (lane == 0) Mh[k] = s;
}

// nuw: nu, the break test, hw, ||xi||_A^2, and the new row / column of M.
// h2[0:d] and h2[d] = ||v1||^2; a[0:d] and a[d] = sum w v1^2; Mh = M h2.
__global__ __launch_bounds__(256) void nuw_kernel(State* __restrict__ st, const double* __restrict__ h2,
                                                   const double* __restrict__ a, const double* __restrict__ Mh,
                                                   int d, double* __restrict__ hw, double* __restrict__ M,
                                                   int64_t ldm) {
    if (st->stop) return;
    __shared__ double sred[4];
    __shared__ int s_ok;
    __shared__ double s_inv;
    double q = 0.0, ha = 0.0, hm = 0.0;
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        q = fma(h2[k], h2[k], q);
        ha = fma(h2[k], a[k], ha);
        hm = fma(h2[k], Mh[k], hm);
    }
    q = block_sum(q, sred);
    ha = block_sum(ha, sred);
    hm = block_sum(hm, sred);
    if (threadIdx.x == 0) {
        const double s = h2[d] - q;
        const double nu = s > 0.0 ? sqrt(s) : 0.0;
        st->nu = nu;
        s_ok = 0;
        if (nu < st->tau || nu == 0.0) {
            st->stop = RBD_STOP_BREAK;
        } else {
            const double inv = 1.0 / nu;
            const double wxx = (a[d] - 2.0 * ha + hm) * inv * inv;
            st->inv_nu = inv;
            st->wxx = wxx;
            M[(int64_t)d * ldm + d] = wxx;
            s_inv = inv;
            s_ok = 1;
        }
    }
    __syncthreads();
    if (!s_ok) return;
    const double inv = s_inv;
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        const double h = (a[k] - Mh[k]) * inv;
        hw[k] = h;
        M[(int64_t)k * ldm + d] = h;
        M[(int64_t)d * ldm + k] = h;
    }
}

// gvec2: v2 = v1 - Y h2, xi = v2 / nu written to Y(:, d), g = w . xi - Y hw.
template <int KC, int RU, bool NT>
__global__ __launch_bounds__(256) void gvec2_kernel(double* __restrict__ Y, int64_t ldy, int64_t m,
                                                     const State* __restrict__ st, int d, int rows_per_blk,
                                                     const double* __restrict__ v1, const double* __restrict__ h2,
                                                     const double* __restrict__ hw, const double* __restrict__ w,
                                                     double* __restrict__ ys, double* __restrict__ v2,
                                                     double* __restrict__ g) {
    if (st->stop) return;
    constexpr int KW = kWave * KC;
    __shared__ double hs[KW];
    __shared__ double gs[KW];
    for (int k = threadIdx.x; k < KW; k += blockDim.x) {
        hs[k] = (k < d) ? h2[k] : 0.0;
        gs[k] = (k < d) ? hw[k] : 0.0;
    }
    __syncthreads();
    const double inv = st->inv_nu;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    static_assert(RU <= kWave / 8, "eight lanes per row in flight for the block write");
    const int yb = d & ~7;
    const bool blk = (d & 7) == 7;                 // this column completes its block
    const int ju = lane >> 3, jj = lane & 7;       // lane 8u + j writes Y(rb + u, yb + j)
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min(m, r0 + (int64_t)rows_per_blk);
    for (int64_t rb = r0 + (int64_t)wv * RU; rb < r1; rb += (int64_t)nw * RU) {
        const bool okb = blk && ju < RU && rb + ju < r1;
        const double sv = (okb && jj < 7) ? ys[(int64_t)jj * m + rb + ju] : 0.0;
        const double vb = (okb && jj == 7) ? v1[rb + ju] : 0.0;
        double y[RU][KC];
        double dots[2 * RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t r = rb + u;
            const bool ok = r < r1;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const int k = lane + kWave * c;
                y[u][c] = (ok && k < d) ? ld_y<NT>(y_src(Y, ldy, ys, m, r, k, yb)) : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                a = fma(y[u][c], hs[lane + kWave * c], a);
                b = fma(y[u][c], gs[lane + kWave * c], b);
            }
            dots[u] = a;
            dots[RU + u] = b;
        }
        wave_sum_n<2 * RU>(dots);
        double xb = 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t r = rb + u;
            if (lane == u && r < r1) {
                const double v = v1[r] - dots[u];
                const double xi = v * inv;
                v2[r] = v;
                ys[(int64_t)(d - yb) * m + r] = xi;
                g[r] = w[r] * xi - dots[RU + u];
            }
            if (ju == u) xb = (vb - dots[u]) * inv;     // the same value, in the lanes of row u's block write
        }
        if (okb) Y[(rb + ju) * ldy + yb + jj] = jj < 7 ? sv : xb;
    }
}

// ---------------------------------------------------------------------------
// General SPD A, two passes over Y per step.  After the first pass (cgs1:
// v1, h2 = Y'v1, ||v1||^2) and u = A v1, the second pass forms
// v2 = v1 - Y h2 and xi = v2 / nu (written to Y(:, d)) and, in the same read
// of Y, the partials of Y'u and v1'u.  With M = Y'AY kept up to date,
//   hw = Y'(A xi) = (Y'u - M h2) / nu,
//   ||xi||_A^2 = (v1'u - 2 h2'(Y'u) + h2'M h2) / nu^2
// (the algebra of the diagonal case, with A v1 in place of w . v1).
// A xi = (A v2) / nu comes from a second sparse product, and
// g' x_j = (A xi)' x_j - hw' T(0:d, j) from the scan of A xi plus correction
// rows through T, so g itself is never formed.
// ---------------------------------------------------------------------------

// cgs2u: v2 = v1 - Y h2 (stored), Y(:, d) = v2 / nu; per block the partials
// of Y'u (part[blk * ldp + k], k < d) and of v1'u (part[blk * ldp + d]).
template <int KC, int RU, bool NT>
__global__ __launch_bounds__(256) void cgs2u_kernel(double* __restrict__ Y, int64_t ldy, int64_t m,
                                                     const State* __restrict__ st, int d, int rows_per_blk,
                                                     const double* __restrict__ v1, const double* __restrict__ h2,
                                                     const double* __restrict__ u, double* __restrict__ ys,
                                                     double* __restrict__ v2, double* __restrict__ part,
                                                     int64_t ldp) {
    if (st->stop) return;
    constexpr int KW = kWave * KC;
    __shared__ double hs[KW];
    __shared__ double accs[KW];
    __shared__ double sred[4];
    for (int k = threadIdx.x; k < KW; k += blockDim.x) {
        hs[k] = (k < d) ? h2[k] : 0.0;
        accs[k] = 0.0;
    }
    __syncthreads();
    const double inv = st->inv_nu;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    static_assert(RU <= kWave / 8, "eight lanes per row in flight for the block write");
    const int yb = d & ~7;
    const bool blk = (d & 7) == 7;                 // this column completes its block
    const int ju = lane >> 3, jj = lane & 7;       // lane 8u + j writes Y(rb + u, yb + j)
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min(m, r0 + (int64_t)rows_per_blk);
    double acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = 0.0;
    double nacc = 0.0;
    for (int64_t rb = r0 + (int64_t)wv * RU; rb < r1; rb += (int64_t)nw * RU) {
        const bool okb = blk && ju < RU && rb + ju < r1;
        const double sv = (okb && jj < 7) ? ys[(int64_t)jj * m + rb + ju] : 0.0;
        double y[RU][KC];
        double vv[RU], ur[RU], dot[RU];
#pragma unroll
        for (int q = 0; q < RU; ++q) {
            const int64_t r = rb + q;
            const bool ok = r < r1;
            vv[q] = ok ? v1[r] : 0.0;
            ur[q] = ok ? u[r] : 0.0;
            dot[q] = 0.0;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const int k = lane + kWave * c;
                y[q][c] = (ok && k < d) ? ld_y<NT>(y_src(Y, ldy, ys, m, r, k, yb)) : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < RU; ++q)
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                dot[q] = fma(y[q][c], hs[lane + kWave * c], dot[q]);
                acc[c] = fma(y[q][c], ur[q], acc[c]);
            }
        wave_sum_n<RU>(dot);
        double xb = 0.0;
#pragma unroll
        for (int q = 0; q < RU; ++q) {
            const int64_t r = rb + q;
            const double v = vv[q] - dot[q];
            if (lane == q && r < r1) {
                v2[r] = v;
                ys[(int64_t)(d - yb) * m + r] = v * inv;
                nacc = fma(vv[q], ur[q], nacc);
            }
            if (ju == q) xb = v * inv;
        }
        if (okb) Y[(rb + ju) * ldy + yb + jj] = jj < 7 ? sv : xb;
    }
    const double s = block_sum(nacc, sred);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * ldp + d] = s;
    if (d == 0) return;
    for (int q = 0; q < nw; ++q) {
        if (wv == q) {
#pragma unroll
            for (int c = 0; c < KC; ++c) accs[lane + kWave * c] += acc[c];
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < d; k += blockDim.x) part[(int64_t)blockIdx.x * ldp + k] = accs[k];
}

// ---------------------------------------------------------------------------
// Lagged reorthogonalisation (A = I).  The second Gram-Schmidt pass of step d
// is not formed as a vector: with v1 the first-pass vector and
// h2 = Y(:, 0:d)' v1, the new basis vector is xi = (v1 - Y h2) / nu, where
// nu^2 = ||v1||^2 - ||h2||^2 (v1 - Y h2 is orthogonal to Y), and its row of T is
//   T(d, :) = xi' X = (v1' X - h2' T(0:d, :)) / nu        (T(0:d, :) = Y' X).
// The column xi itself is written by the next step's first pass, which reads
// Y anyway; so each step reads Y once instead of twice.
// ---------------------------------------------------------------------------

// cgs1_lag: first forms this row's entry of the deferred column d-1,
//   Y(i, d-1) = (v1p_i - Y(i, 0:d-1) h2p) / nu_prev,
// stages it, then v1 = x_p - Y(:, 0:d) h1 (h1 = T(0:d, p)); per block the
// share of h2 = Y(:, 0:d)' v1 (part[blk*ldp + k], k < d) and of ||v1||^2
// (part[blk*ldp + d]).
template <int KC, int RU, bool NT, typename Tb, typename Tx>
__global__ __launch_bounds__(256) void cgs1_lag_kernel(const Tx* __restrict__ X, int64_t ldx, int64_t m,
                                                        Tb* __restrict__ Y, int64_t ldy,
                                                        const double* __restrict__ T, int64_t ldt,
                                                        State* __restrict__ st, int d, int rows_per_blk,
                                                        const double* __restrict__ v1p,
                                                        const double* __restrict__ h2p, double* __restrict__ v1,
                                                        Tb* __restrict__ ys, double* __restrict__ part,
                                                        int64_t ldp) {
    static_assert(RU <= kWave / 8, "eight lanes per row in flight for the block write");
    if (st->stop) return;
    constexpr int KW = kWave * KC;
    __shared__ double hs[KW];
    __shared__ double gs[KW];
    __shared__ double accs[KW];
    __shared__ double sred[4];
    const int p = st->p;
    const double invp = st->inv_nu;               // 1/nu of the previous step
    const int dl = d - 1;                          // the deferred column (none at d = 0)
    for (int k = threadIdx.x; k < KW; k += blockDim.x) {
        hs[k] = (k < d) ? T[(int64_t)k * ldt + p] : 0.0;
        gs[k] = (k < dl) ? h2p[k] : 0.0;
        accs[k] = 0.0;
    }
    __syncthreads();
    const double hl = dl >= 0 ? hs[dl] : 0.0;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int cl = dl >= 0 ? dl / kWave : -1, ll = dl >= 0 ? dl % kWave : -1;
    const int yb = dl >= 0 ? (dl & ~7) : 0;       // columns below yb are in Y, [yb, dl) in ys
    const bool blk = dl >= 0 && (dl & 7) == 7;    // this column completes its block
    const int ju = lane >> 3, jj = lane & 7;       // lane 8u + j writes Y(rb + u, yb + j)
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min(m, r0 + (int64_t)rows_per_blk);
    double acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = 0.0;
    // the deferred column's products, kept apart (its loaded entries are zero;
    // chunk cl is uniform) and added into acc[cl] at the end: the same sums
    // as forming them in place, without a select per entry
    double accl = 0.0;
    double nacc = 0.0;
    for (int64_t rb = r0 + (int64_t)w * RU; rb < r1; rb += (int64_t)nw * RU) {
        // lane u < RU carries row rb + u's scalars (one load / store instruction per group)
        const int64_t rl = rb + lane;
        const bool okl = lane < RU && rl < r1;
        // x_p's entries straight from X, widened after the group's other loads
        // have issued (a widening under the test would wait for the load)
        const Tx xr = okl ? X[rl * ldx + p] : Tx{};
        const double vl = (okl && dl >= 0) ? v1p[rl] : 0.0;
        const bool okb = blk && ju < RU && rb + ju < r1;
        const Tb sv = (okb && jj < 7) ? ys[(int64_t)jj * m + rb + ju] : Tb(0);
        double y[RU][KC];
        double dots[2 * RU];
        load_y_rows<NT, RU, KC>(y, Y, ldy, ys, m, rb, r1, lane, dl, yb);
        const double xl = Ld<Tx>::from(xr);
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                a = fma(y[u][c], gs[lane + kWave * c], a);
                b = fma(y[u][c], hs[lane + kWave * c], b);
            }
            dots[u] = a;
            dots[RU + u] = b;
        }
        wave_sum_n<2 * RU>(dots);
        double vo = 0.0, yo = 0.0, yb7 = 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            // rows past the end: 0; the stored (Tb) value is what every pass uses
            const double yl = dl >= 0 ? (double)(Tb)((lane_bcast(vl, u) - dots[u]) * invp) : 0.0;
            const double v = lane_bcast(xl, u) - dots[RU + u] - yl * hl;
#pragma unroll
            for (int c = 0; c < KC; ++c) acc[c] = fma(y[u][c], v, acc[c]);
            accl = fma(lane == ll ? yl : 0.0, v, accl);
            if (lane == u) { vo = v; yo = yl; }
            if (ju == u) yb7 = yl;
        }
        if (okl) {
            v1[rl] = vo;
            nacc = fma(vo, vo, nacc);
            if (dl >= 0) ys[(int64_t)(dl - yb) * m + rl] = (Tb)yo;
        }
        if (okb) Y[(rb + ju) * ldy + yb + jj] = jj < 7 ? sv : (Tb)yb7;
    }
#pragma unroll
    for (int c = 0; c < KC; ++c)
        if (c == cl) acc[c] += accl;
    const double nn = block_sum(nacc, sred);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * ldp + d] = nn;
    if (d == 0) return;
    for (int q = 0; q < nw; ++q) {
        if (w == q) {
#pragma unroll
            for (int c = 0; c < KC; ++c) accs[lane + kWave * c] += acc[c];
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < d; k += blockDim.x) part[(int64_t)blockIdx.x * ldp + k] = accs[k];
}

// nu_lag: h2[0:d] and h2[d] = ||v1||^2 summed; nu^2 = ||v1||^2 - ||h2||^2 and
// step 2.2's break test.
__global__ __launch_bounds__(256) void nu_lag_kernel(State* __restrict__ st, const double* __restrict__ h2, int d) {
    if (st->stop) return;
    __shared__ double sred[4];
    double q = 0.0;
    for (int k = threadIdx.x; k < d; k += blockDim.x) q = fma(h2[k], h2[k], q);
    q = block_sum(q, sred);
    if (threadIdx.x == 0) {
        const double s = h2[d] - q;
        const double nu = s > 0.0 ? sqrt(s) : 0.0;
        st->nu = nu;
        if (nu < st->tau || nu == 0.0) st->stop = RBD_STOP_BREAK;
        else st->inv_nu = 1.0 / nu;
    }
}

// Correction rows -h2' T(0:d, :) / nu of the lagged step, one partial row per
// chunk of kTcorr rows of T (grid: column blocks x chunks); summed after the
// scan's slab partials in a fixed order.
constexpr int kTcorr = 32;

// nu_tcorr: nu and the break test with the correction rows, in one launch.
// Every block forms nu from h2 in the same fixed order (so all agree with each
// other and with nu_lag_kernel), block (0, 0) records nu / the break test, and
// the blocks write the correction rows of their column block and chunk.
__global__ __launch_bounds__(256) void nu_tcorr_kernel(State* __restrict__ st, const double* __restrict__ h2, int d,
                                                        const double* __restrict__ T, int64_t ldt, int64_t n,
                                                        double* __restrict__ out) {
    if (st->stop) return;
    __shared__ double sred[4];
    double q = 0.0;
    for (int k = threadIdx.x; k < d; k += blockDim.x) q = fma(h2[k], h2[k], q);
    q = block_sum(q, sred);
    const double s2 = h2[d] - q;
    const double nu = s2 > 0.0 ? sqrt(s2) : 0.0;
    const bool brk = nu < st->tau || nu == 0.0;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        st->nu = nu;
        if (brk) st->stop = RBD_STOP_BREAK;
        else st->inv_nu = 1.0 / nu;
    }
    if (brk || d == 0) return;
    const double inv = 1.0 / nu;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int k0 = blockIdx.y * kTcorr, k1 = min(d, k0 + kTcorr);
    double c = 0.0;
#pragma unroll 8
    for (int k = k0; k < k1; ++k) c = fma(h2[k], T[(int64_t)k * ldt + j], c);
    out[(int64_t)blockIdx.y * n + j] = -c * inv;
}


// tcorr2: rows of 2n for the two-vector scan: zeros in the first n, then
// -hw' T(k0:k1, :) for a chunk of kTcorr rows of T (hw already divided by nu).
__global__ __launch_bounds__(256) void tcorr2_kernel(const State* __restrict__ st, const double* __restrict__ hw,
                                                      int d, const double* __restrict__ T, int64_t ldt, int64_t n,
                                                      double* __restrict__ out) {
    if (st->stop) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int k0 = blockIdx.y * kTcorr, k1 = min(d, k0 + kTcorr);
    double c = 0.0;
#pragma unroll 8
    for (int k = k0; k < k1; ++k) c = fma(hw[k], T[(int64_t)k * ldt + j], c);
    double* row = out + (int64_t)blockIdx.y * 2 * n;
    row[j] = 0.0;
    row[n + j] = -c;
}

// ycol: writes the deferred column, Y(:, col) = (v1 - Y(:, 0:col) h2) / nu,
// and copies the staged columns [8 floor(col / 8), col) from ys into Y, so
// that Y(:, 0:col+1) is complete.
// FINAL = false: col = d, before an exact refresh of this step (skipped when
// none is queued).  FINAL = true: col = (final d) - 1, after the loop, written
// only when col < d (rbd_fit_basis keeps later columns in FP32); the buffers
// of that step are chosen by the parity of col.
template <int KC, int RU, bool FINAL, bool NT, typename Tb = double>
__global__ __launch_bounds__(256) void ycol_kernel(Tb* __restrict__ Y, int64_t ldy, int64_t m,
                                                    const State* __restrict__ st, int d, int rows_per_blk,
                                                    const double* __restrict__ v1a, const double* __restrict__ v1b,
                                                    const double* __restrict__ h2a, const double* __restrict__ h2b,
                                                    const Tb* __restrict__ ys) {
    int col;
    if (FINAL) {                 // d: only a final column below d is written here
        if (st->stop == kStopError) return;
        col = st->d - 1;
        if (col < 0 || col >= d) return;
    } else {
        if (st->stop || st->nflag == 0) return;
        col = d;
    }
    const double* v1 = (col & 1) ? v1b : v1a;
    const double* h2 = (col & 1) ? h2b : h2a;
    constexpr int KW = kWave * KC;
    __shared__ double hs[KW];
    for (int k = threadIdx.x; k < KW; k += blockDim.x) hs[k] = (k < col) ? h2[k] : 0.0;
    __syncthreads();
    const double inv = st->inv_nu;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int yb = col & ~7;                       // columns below yb are in Y, [yb, col) in ys
    const int ju = lane >> 3, jj = lane & 7;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min(m, r0 + (int64_t)rows_per_blk);
    for (int64_t rb = r0 + (int64_t)wv * RU; rb < r1; rb += (int64_t)nw * RU) {
        double y[RU][KC];
        load_y_rows<NT, RU, KC>(y, Y, ldy, ys, m, rb, r1, lane, col, yb);
        double dot[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            dot[u] = 0.0;
#pragma unroll
            for (int c = 0; c < KC; ++c) dot[u] = fma(y[u][c], hs[lane + kWave * c], dot[u]);
        }
        wave_sum_n<RU>(dot);
#pragma unroll
        for (int u = 0; u < RU; ++u)
            if (lane == u && rb + u < r1) Y[(rb + u) * ldy + col] = (Tb)((v1[rb + u] - dot[u]) * inv);
        // the staged columns [yb, col) of these rows into Y
        if (ju < RU && rb + ju < r1 && yb + jj < col) Y[(rb + ju) * ldy + yb + jj] = ys[(int64_t)jj * m + rb + ju];
    }
}


// ---------------------------------------------------------------------------
// The same two passes with the basis kept in FP32 (rbd_fit_basis).  A lane
// holds two adjacent columns (k = 2 lane + 128 c, c < KC2), read from Y with
// one 8-byte load: FP32 values read one per lane halved the bytes each wave
// keeps in flight and ran at 4.7 TB/s against 6.2.  The staged columns keep
// the FP64 column-major slots of the FP64 pass (slot j of row r at
// ys[j m + r], holding the FP32-rounded values): a step's store is then 64
// contiguous bytes per row group (FP32 slots, stored 32 or 4 bytes at a time,
// made every step 25-50 us slower), and the chunk that holds the staged block
// reads a staged pair with two loads.  ldy is even.
// ---------------------------------------------------------------------------
// Entries (rb + u, k) and (rb + u, k + 1), k = 2 lane + 128 c, widened to
// FP64; zero for rows >= r1 or columns >= cols.  Loads from clamped
// addresses, all issued before the first widening.
// FREE: the caller's KC2 is the one the host sizes from the step (kc2_of(kc_for(d))
// with cols = d - 1, yb = cols rounded down to 8), so the chunks below KC2 / 2 lie
// wholly below yb and take no select; rows past r1 are zeroed by one uniform test.
template <bool NT, int RU, int KC2, bool FREE = false>
__device__ __forceinline__ void load_y32_rows(double (&y)[RU][KC2][2], const float* Y, int64_t ldy,
                                              const double* ys, int64_t m, int64_t rb, int64_t r1, int lane,
                                              int cols, int yb) {
    const int cyb = yb / 128;                       // the chunk that holds the staged block (uniform)
    f32x2 raw[RU][KC2];
    double s0[RU], s1[RU];
    const int ks = 2 * lane + 128 * cyb - yb;       // this lane's pair within the staged block
    const bool in_st = ks >= 0 && ks < 8 && ks < cols - yb;     // at most four lanes read staged slots
#pragma unroll
    for (int u = 0; u < RU; ++u) {
        const int64_t r = min(rb + u, r1 - 1);
#pragma unroll
        for (int c = 0; c < KC2; ++c) {
            const int k = min(2 * lane + 128 * c, max(yb - 2, 0));
            const f32x2* p = reinterpret_cast<const f32x2*>(Y + r * ldy + k);
            raw[u][c] = NT ? __builtin_nontemporal_load(p) : *p;
        }
        s0[u] = in_st ? ys[ks * m + r] : 0.0;               // FP64: no widening under the test
        s1[u] = in_st ? ys[(ks + 1) * m + r] : 0.0;
    }
    __builtin_amdgcn_sched_barrier(0);              // every load above issues before the first use below
    constexpr int kFree = FREE ? KC2 / 2 : 0;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
#pragma unroll
        for (int c = 0; c < kFree; ++c) {
            y[u][c][0] = (double)raw[u][c].x;
            y[u][c][1] = (double)raw[u][c].y;
        }
#pragma unroll
        for (int c = kFree; c < KC2; ++c) {
            const int k = 2 * lane + 128 * c;
            const bool ok = rb + u < r1;
            const bool st = k >= yb;                    // a staged pair (it lies in chunk cyb)
            const double a = st ? s0[u] : (double)raw[u][c].x, b = st ? s1[u] : (double)raw[u][c].y;
            y[u][c][0] = (ok && k < cols) ? a : 0.0;
            y[u][c][1] = (ok && k + 1 < cols) ? b : 0.0;
        }
    }
    if (kFree > 0 && rb + RU > r1) {
#pragma unroll
        for (int u = 0; u < RU; ++u)
            if (rb + u >= r1) {
#pragma unroll
                for (int c = 0; c < kFree; ++c) y[u][c][0] = y[u][c][1] = 0.0;
            }
    }
}

// cgs1_lag for an FP32 basis: the arithmetic of cgs1_lag_kernel, the deferred
// column rounded to FP32 as it is stored (every pass uses the stored value).
template <int KC2, int RU, bool NT>
__global__ __launch_bounds__(256) void cgs1_lag32_kernel(const double* __restrict__ xp, int64_t m,
                                                          float* __restrict__ Y, int64_t ldy,
                                                          const double* __restrict__ T, int64_t ldt,
                                                          State* __restrict__ st, int d, int rows_per_blk,
                                                          const double* __restrict__ v1p,
                                                          const double* __restrict__ h2p, double* __restrict__ v1,
                                                          double* __restrict__ ys, double* __restrict__ part,
                                                          int64_t ldp) {
    static_assert(RU <= kWave / 8, "eight lanes per row in flight for the block write");
    if (st->stop) return;
    constexpr int KW = 128 * KC2;
    __shared__ double hs[KW];
    __shared__ double gs[KW];
    __shared__ double accs[KW];
    __shared__ double sred[4];
    const int p = st->p;
    const double invp = st->inv_nu;
    const int dl = d - 1;                          // the deferred column (none at d = 0)
    for (int k = threadIdx.x; k < KW; k += blockDim.x) {
        hs[k] = (k < d) ? T[(int64_t)k * ldt + p] : 0.0;
        gs[k] = (k < dl) ? h2p[k] : 0.0;
        accs[k] = 0.0;
    }
    __syncthreads();
    const double hl = dl >= 0 ? hs[dl] : 0.0;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int cl = dl >= 0 ? dl / 128 : -1, ll = dl >= 0 ? (dl % 128) / 2 : -1, hlf = dl >= 0 ? dl % 2 : 0;
    const int yb = dl >= 0 ? (dl & ~7) : 0;
    const bool blk = dl >= 0 && (dl & 7) == 7;
    const int ju = lane >> 3, jj = lane & 7;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min(m, r0 + (int64_t)rows_per_blk);
    double acc[KC2][2];
#pragma unroll
    for (int c = 0; c < KC2; ++c) acc[c][0] = acc[c][1] = 0.0;
    double accl = 0.0;                              // the deferred column's products (see cgs1_lag_kernel)
    double nacc = 0.0;
    for (int64_t rb = r0 + (int64_t)w * RU; rb < r1; rb += (int64_t)nw * RU) {
        const int64_t rl = rb + lane;
        const bool okl = lane < RU && rl < r1;
        const double xl = okl ? xp[rl] : 0.0;
        const double vl = (okl && dl >= 0) ? v1p[rl] : 0.0;
        const bool okb = blk && ju < RU && rb + ju < r1;
        const double sv = (okb && jj < 7) ? ys[(int64_t)jj * m + rb + ju] : 0.0;
        double y[RU][KC2][2];
        double dots[2 * RU];
        load_y32_rows<NT, RU, KC2, true>(y, Y, ldy, ys, m, rb, r1, lane, dl, yb);
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int c = 0; c < KC2; ++c)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int k = 2 * lane + 128 * c + h;
                    a = fma(y[u][c][h], gs[k], a);
                    b = fma(y[u][c][h], hs[k], b);
                }
            dots[u] = a;
            dots[RU + u] = b;
        }
        wave_sum_n<2 * RU>(dots);
        double vo = 0.0, yo = 0.0, yb7 = 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const double yl = dl >= 0 ? (double)(float)((lane_bcast(vl, u) - dots[u]) * invp) : 0.0;
            const double v = lane_bcast(xl, u) - dots[RU + u] - yl * hl;
#pragma unroll
            for (int c = 0; c < KC2; ++c)
#pragma unroll
                for (int h = 0; h < 2; ++h) acc[c][h] = fma(y[u][c][h], v, acc[c][h]);
            accl = fma(lane == ll ? yl : 0.0, v, accl);
            if (lane == u) { vo = v; yo = yl; }
            if (ju == u) yb7 = yl;
        }
        if (okl) {
            v1[rl] = vo;
            nacc = fma(vo, vo, nacc);
            if (dl >= 0) ys[(int64_t)(dl - yb) * m + rl] = yo;
        }
        if (okb) Y[(rb + ju) * ldy + yb + jj] = (float)(jj < 7 ? sv : yb7);
    }
#pragma unroll
    for (int c = 0; c < KC2; ++c)
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (c == cl && h == hlf) acc[c][h] += accl;
    const double nn = block_sum(nacc, sred);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * ldp + d] = nn;
    if (d == 0) return;
    for (int q = 0; q < nw; ++q) {
        if (w == q) {
#pragma unroll
            for (int c = 0; c < KC2; ++c)
#pragma unroll
                for (int h = 0; h < 2; ++h) accs[2 * lane + 128 * c + h] += acc[c][h];
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < d; k += blockDim.x) part[(int64_t)blockIdx.x * ldp + k] = accs[k];
}

// ycol for an FP32 basis (see ycol_kernel): the deferred column into Y and
// the staged columns [8 floor(col / 8), col) from their slots.
template <int KC2, int RU, bool FINAL, bool NT>
__global__ __launch_bounds__(256) void ycol32_kernel(float* __restrict__ Y, int64_t ldy, int64_t m,
                                                      const State* __restrict__ st, int d, int rows_per_blk,
                                                      const double* __restrict__ v1a, const double* __restrict__ v1b,
                                                      const double* __restrict__ h2a, const double* __restrict__ h2b,
                                                      const double* __restrict__ ys) {
    int col;
    if (FINAL) {                 // d: only a final column at or above d is written here
        if (st->stop == kStopError) return;
        col = st->d - 1;
        if (col < 0 || col < d) return;
    } else {
        if (st->stop || st->nflag == 0) return;
        col = d;
    }
    const double* v1 = (col & 1) ? v1b : v1a;
    const double* h2 = (col & 1) ? h2b : h2a;
    constexpr int KW = 128 * KC2;
    __shared__ double hs[KW];
    for (int k = threadIdx.x; k < KW; k += blockDim.x) hs[k] = (k < col) ? h2[k] : 0.0;
    __syncthreads();
    const double inv = st->inv_nu;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int yb = col & ~7;
    const int ju = lane >> 3, jj = lane & 7;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = min(m, r0 + (int64_t)rows_per_blk);
    for (int64_t rb = r0 + (int64_t)wv * RU; rb < r1; rb += (int64_t)nw * RU) {
        double y[RU][KC2][2];
        load_y32_rows<NT, RU, KC2>(y, Y, ldy, ys, m, rb, r1, lane, col, yb);
        double dot[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            dot[u] = 0.0;
#pragma unroll
            for (int c = 0; c < KC2; ++c)
#pragma unroll
                for (int h = 0; h < 2; ++h) dot[u] = fma(y[u][c][h], hs[2 * lane + 128 * c + h], dot[u]);
        }
        wave_sum_n<RU>(dot);
#pragma unroll
        for (int u = 0; u < RU; ++u)
            if (lane == u && rb + u < r1) Y[(rb + u) * ldy + col] = (float)((v1[rb + u] - dot[u]) * inv);
        if (ju < RU && rb + ju < r1 && yb + jj < col) Y[(rb + ju) * ldy + yb + jj] = (float)ys[(int64_t)jj * m + rb + ju];
    }
}

// ---------------------------------------------------------------------------
// reduce_rows: out[g * ldo + c] = sum over rows r of group g (rows g*per ..
// g*per+per-1, ascending) of part[r * ldp + c], for c < len.  Grid
// (ceil(len / blockDim), groups).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_rows_kernel(const State* __restrict__ st,
                                                           const double* __restrict__ part, int64_t ldp,
                                                           int rows, int per, int64_t len,
                                                           double* __restrict__ out, int64_t ldo) {
    if (st && st->stop) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= len) return;
    const int r0 = blockIdx.y * per, r1 = min(rows, r0 + per);
    double s = 0.0;
#pragma unroll 8
    for (int r = r0; r < r1; ++r) s += part[(int64_t)r * ldp + c];
    out[(int64_t)blockIdx.y * ldo + c] = s;
}

// ---------------------------------------------------------------------------
// resid_mfma: partial squared residual norms of listed columns (STORE:
// the residual entries themselves, R[i * ldr + jj], instead of any sums),
//   part[s * ldp + jj] = sum_{i in slab s} w_i (X[i, c] - sum_{k<K} Y[i, k] C[k, c])^2,
// c = J ? J[jj] : jj, w_i = 1 without weights, for jj < count (count =
// *count_dev when given, else count_host).  Work items (column tile, slab)
// are strided over a fixed grid, each writing its own partial.  The product
// Y(:, 0:K) C(0:K, cols) runs on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64; lane l supplies A(l % 16, l / 16) and
// B(l / 16, l % 16), accumulator register r of lane l holds C(4r + l / 16,
// l % 16)).  Workgroup tile 128 rows x 64 columns, four waves of 32 x 64;
// k staged through LDS 16 deep, the next chunk's global loads in flight
// while the current chunk is multiplied.  Partial sums are combined in a
// fixed order (lanes, then waves), so results are deterministic.
// ---------------------------------------------------------------------------
typedef double f64x4_t __attribute__((ext_vector_type(4)));
constexpr bool kResidPrefetchX = false;    // load the tile's X entries before the products (measured: slower, spills)
#define RBD_RESID_MIN_BLOCKS 2                // workgroups per CU the register budget is sized for

template <typename Tx, bool STORE = false, typename Ty = double>
__global__ __launch_bounds__(256, RBD_RESID_MIN_BLOCKS) void resid_mfma_kernel(const Tx* __restrict__ X, int64_t ldx, int64_t m,
                                                          const Ty* __restrict__ Y, int64_t ldy, int K,
                                                          const double* __restrict__ C, int64_t ldc,
                                                          const int* __restrict__ J,
                                                          const int* __restrict__ count_dev, int count_host,
                                                          int rows_per_slab, int nslab, double* __restrict__ part,
                                                          int64_t ldp, const double* __restrict__ w,
                                                          double* __restrict__ R = nullptr, int64_t ldr = 0,
                                                          int count_off = 0, int count_cap = INT32_MAX) {
    // the queue entries [count_off, count_off + count_cap) of a device-side count
    const int cnt = count_dev ? min(max(*count_dev - count_off, 0), count_cap) : count_host;
    if (cnt <= 0) return;
    constexpr int TM = 128, TN = 64, KB = 16;
    constexpr int YQ = TM * KB / 256, CQ = KB * TN / 256;
    __shared__ double Ys[TM][KB + 1];
    __shared__ double Cs[KB][TN + 1];
    __shared__ double red[4][TN];
    __shared__ int cols[TN];
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int lr = lane % 16, lk = lane / 16;
    const int ntiles = (cnt + TN - 1) / TN;
    const int nwork = ntiles * nslab;
    for (int wk = blockIdx.x; wk < nwork; wk += gridDim.x) {
        const int t = wk % ntiles, s = wk / ntiles;
        __syncthreads();
        if (tid < TN) {
            const int jj = t * TN + tid;
            cols[tid] = (jj < cnt) ? (J ? J[jj] : jj) : -1;
        }
        __syncthreads();
        const int64_t rbeg = (int64_t)s * rows_per_slab;
        const int64_t rend = min(m, rbeg + (int64_t)rows_per_slab);
        double rs[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t row0 = rbeg; row0 < rend; row0 += TM) {
            // this tile's entries of X, loaded first so that the gather's
            // latency is covered by the products
            Tx xr[2][4][4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int col = cols[16 * b + lr];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = row0 + 32 * wv + 16 * a + 4 * r + lk;
                        xr[a][b][r] = (kResidPrefetchX && row < rend && col >= 0) ? X[row * ldx + col] : Tx{};
                    }
            }
            f64x4_t acc[2][4];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = (f64x4_t){0.0, 0.0, 0.0, 0.0};
            double yr[YQ], cr[CQ];
            auto load = [&](int k0) {
#pragma unroll
                for (int q = 0; q < YQ; ++q) {
                    const int e = tid + 256 * q;
                    const int rr = e / KB, kk = e % KB;
                    const int64_t row = row0 + rr;
                    const int k = k0 + kk;
                    if constexpr (sizeof(Ty) == 8) {
                        yr[q] = (row < rend && k < K) ? Y[row * ldy + k] : 0.0;
                    } else {
                        // clamped and unconditional, masked by a product (basis entries are
                        // finite): a selected load would become a branch that waits for it
                        const double v = (double)Y[min(row, rend - 1) * ldy + min(k, K - 1)];
                        yr[q] = v * ((row < rend && k < K) ? 1.0 : 0.0);
                    }
                }
#pragma unroll
                for (int q = 0; q < CQ; ++q) {
                    const int e = tid + 256 * q;
                    const int kk = e / TN, cc = e % TN;
                    const int k = k0 + kk;
                    const int col = cols[cc];
                    cr[q] = (k < K && col >= 0) ? C[(int64_t)k * ldc + col] : 0.0;
                }
            };
            load(0);
            for (int k0 = 0; k0 < K; k0 += KB) {
                __syncthreads();
#pragma unroll
                for (int q = 0; q < YQ; ++q) {
                    const int e = tid + 256 * q;
                    Ys[e / KB][e % KB] = yr[q];
                }
#pragma unroll
                for (int q = 0; q < CQ; ++q) {
                    const int e = tid + 256 * q;
                    Cs[e / TN][e % TN] = cr[q];
                }
                __syncthreads();
                if (k0 + KB < K) load(k0 + KB);
#pragma unroll
                for (int ks = 0; ks < KB; ks += 4) {
                    if (k0 + ks >= K) break;       // the last chunk's padding
                    double af[2], bf[4];
#pragma unroll
                    for (int a = 0; a < 2; ++a) af[a] = Ys[32 * wv + 16 * a + lr][ks + lk];
#pragma unroll
                    for (int b = 0; b < 4; ++b) bf[b] = Cs[ks + lk][16 * b + lr];
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
                }
            }
            // r = X - Y C, squared and summed per column.  Every entry is loaded
            // before any is used, from a clamped address (row rbeg, column
            // cols[0] stand in outside the tile) and without a branch: a guarded
            // load used at once waits for its data before the next one issues.
            if (!kResidPrefetchX) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int col = cols[16 * b + lr];
                    const int colc = col >= 0 ? col : cols[0];
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int64_t row = row0 + 32 * wv + 16 * a + 4 * r + lk;
                            xr[a][b][r] = X[(row < rend ? row : rbeg) * ldx + colc];
                        }
                }
            }
            double wt[2][4];         // row weights, loaded the same way
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row0 + 32 * wv + 16 * a + 4 * r + lk;
                    wt[a][r] = (!STORE && w) ? w[row < rend ? row : rbeg] : 1.0;
                }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int col = cols[16 * b + lr];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t row = row0 + 32 * wv + 16 * a + 4 * r + lk;
                        const bool in = row < rend && col >= 0;
                        const double d = in ? Ld<Tx>::from(xr[a][b][r]) - acc[a][b][r] : 0.0;
                        if (STORE) {
                            if (in) R[row * ldr + t * TN + 16 * b + lr] = d;
                        } else {
                            // outside the tile d = 0 adds exactly nothing
                            rs[b] = w ? fma(wt[a][r] * d, d, rs[b]) : fma(d, d, rs[b]);
                        }
                    }
            }
        }
        if (STORE) continue;
        // column cc = 16 b + lane % 16: sum the four lane groups, then the four waves
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            double v = rs[b];
            v += __shfl_xor(v, 16, kWave);
            v += __shfl_xor(v, 32, kWave);
            if (lk == 0) red[wv][16 * b + lr] = v;
        }
        __syncthreads();
        if (tid < TN) {
            const double sum = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
            const int jj = t * TN + tid;
            if (jj < cnt) part[(int64_t)s * ldp + jj] = sum;
        }
    }
}

// ---------------------------------------------------------------------------
// resid_finish: exact errors replace the downdated ones, then argmax + stop.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void resid_finish_kernel(State* __restrict__ st, const double* __restrict__ part,
                                                            int64_t ldp, int nslab, const int* __restrict__ J,
                                                            double* __restrict__ e2, double* __restrict__ base2,
                                                            int64_t n, unsigned* __restrict__ tickets,
                                                            int64_t* __restrict__ pivots,
                                                            double* __restrict__ err_hist, int d) {
    const int cnt = st->nflag;
    if (cnt == 0) return;
    __shared__ double sv[4];
    __shared__ int64_t si[4];
    const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj < cnt) {
        double s = 0.0;
#pragma unroll 8
        for (int q = 0; q < nslab; ++q) s += part[(int64_t)q * ldp + jj];
        const int j = J[jj];
        e2[j] = s;
        base2[j] = s;
    }
    if (!last_to_arrive(&tickets[0], gridDim.x)) return;
    double v = -1.0;
    int64_t i = INT64_MAX;
    for (int64_t c = threadIdx.x; c < n; c += blockDim.x) argmax_merge(v, i, e2[c], c);
    block_argmax(v, i, sv, si);
    if (threadIdx.x == 0) {
        finish_step(st, d, v, i, pivots, err_hist);
        st->nflag = 0;
    }
}

// ---------------------------------------------------------------------------
// General SPD A (section 3.2), A in CSR form (indptr int64, indices int32,
// values FP64).  Every index is checked: a column index outside [0, m) or a
// row range outside [0, nnz) is skipped; the set-up step, which reads every
// row range and entry once, raises bad_index for these and for a decreasing
// indptr (reported as RBD_EMATRIX, and the loop does not start).
// ---------------------------------------------------------------------------
struct Csr {
    const int64_t* __restrict__ ip;
    const int32_t* __restrict__ ix;
    const double* __restrict__ av;
    int64_t nnz;
};

__device__ __forceinline__ void csr_row(const Csr& A, int64_t i, int64_t& e0, int64_t& e1) {
    e0 = max((int64_t)0, A.ip[i]);
    e1 = min(A.nnz, A.ip[i + 1]);
}

// csr_xax: per row slab, part[slab * n + j] = sum_{i in slab} x_ij (A x_j)_i,
// so that summing the slabs gives x_j' A x_j (the pre-computation of
// diag(X'AX) in section 3.3).  One column per thread; all lanes walk the same
// row of A (uniform loads).
template <typename Tx>
__global__ __launch_bounds__(256) void csr_xax_kernel(const Tx* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                                                       Csr A, int rows_per_slab, double* __restrict__ part,
                                                       State* __restrict__ st) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t jc = j < n ? j : n - 1;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_slab, r1 = min(m, r0 + (int64_t)rows_per_slab);
    double acc = 0.0;
    bool bad = false;
    for (int64_t i = r0; i < r1; ++i) {
        int64_t e0, e1;
        csr_row(A, i, e0, e1);
        if (A.ip[i] < 0 || A.ip[i + 1] > A.nnz || A.ip[i + 1] < A.ip[i]) bad = true;
        double y = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t k = A.ix[e];
            if (k < 0 || k >= m) { bad = true; continue; }
            y = fma(A.av[e], Ld<Tx>::one(X + k * ldx + jc), y);
        }
        acc = fma(Ld<Tx>::one(X + i * ldx + jc), y, acc);
    }
    if (bad && threadIdx.x == 0) atomicOr(&st->bad_index, 1);
    if (j < n) part[(int64_t)blockIdx.y * n + j] = acc;
}

// spmv: u = A v, or u = (A v) / nu with SCALED (one row per thread)
template <bool SCALED>
__global__ __launch_bounds__(256) void spmv_kernel(const State* __restrict__ st, Csr A, int64_t m,
                                                    const double* __restrict__ v, double* __restrict__ u) {
    if (st->stop) return;
    const double sc = SCALED ? st->inv_nu : 1.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        int64_t e0, e1;
        csr_row(A, i, e0, e1);
        double y = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t k = A.ix[e];
            if (k >= 0 && k < m) y = fma(A.av[e], v[k], y);
        }
        u[i] = SCALED ? y * sc : y;
    }
}

// csr_quad: part[slab * ldp + c0 + jj] = sum_{i in slab} r_i,jj (A r_jj)_i for
// the residual columns jj < cnt held in R (m x cnt, leading dimension ldr).
// The sum runs over the slab's nonzeros, r' A r = sum_e a_e r_row(e) r_col(e),
// so every entry is independent and several are in flight per wave.  The
// slab's entries are staged in LDS in chunks with the row of each entry
// (rows of a well-formed CSR matrix own consecutive ranges of entries);
// lanes run along the 64 columns of the block, so each access to R reads one
// contiguous row segment.  The kQuadGroups waves take interleaved entries and
// are combined in LDS in a fixed order.
constexpr int kQuadGroups = 4;
constexpr int kQuadChunk = 2048;
__global__ __launch_bounds__(64 * kQuadGroups) void csr_quad_kernel(const double* __restrict__ R, int64_t ldr, int64_t m,
                                                                    const int* __restrict__ count_dev, int cap, Csr A,
                                                                    int rows_per_slab, double* __restrict__ part,
                                                                    int64_t ldp, int c0) {
    // the chunk holds queue entries [c0, c0 + cnt): cnt from the device-side queue length
    const int cnt = min(max(*count_dev - c0, 0), cap);
    if (blockIdx.x * 64 >= cnt) return;
    __shared__ int s_row[kQuadChunk];
    __shared__ int s_col[kQuadChunk];
    __shared__ double s_val[kQuadChunk];
    __shared__ double red[kQuadGroups][64];
    const int lane = threadIdx.x % 64, grp = threadIdx.x / 64;
    const int jj = blockIdx.x * 64 + lane;
    const int jc = jj < cnt ? jj : cnt - 1;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_slab, r1 = min(m, r0 + (int64_t)rows_per_slab);
    const int64_t eb = min(A.nnz, max((int64_t)0, A.ip[r0]));
    const int64_t ee = max(eb, min(A.nnz, A.ip[r1]));
    const double* __restrict__ Rc = R + jc;
    double acc = 0.0;
    for (int64_t cb = eb; cb < ee; cb += kQuadChunk) {
        const int ne = (int)min((int64_t)kQuadChunk, ee - cb);
        for (int t = threadIdx.x; t < ne; t += blockDim.x) {
            const int64_t k = A.ix[cb + t];
            s_row[t] = -1;
            s_col[t] = (k >= 0 && k < m) ? (int)k : -1;
            s_val[t] = A.av[cb + t];
        }
        __syncthreads();
        for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            int64_t e0, e1;
            csr_row(A, i, e0, e1);
            e0 = max(e0, cb);
            e1 = min(e1, cb + ne);
            for (int64_t e = e0; e < e1; ++e) s_row[e - cb] = (int)(i - r0);
        }
        __syncthreads();
        constexpr int G = kQuadGroups, U = 4;
        int t = grp;
        for (; t + (U - 1) * G < ne; t += U * G) {
            double a[U], x[U], y[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int rr = s_row[t + u * G], k = s_col[t + u * G];
                const bool ok = rr >= 0 && k >= 0;
                a[u] = ok ? s_val[t + u * G] : 0.0;
                x[u] = ok ? Rc[(r0 + rr) * ldr] : 0.0;
                y[u] = ok ? Rc[(int64_t)k * ldr] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc = fma(a[u] * x[u], y[u], acc);
        }
        for (; t < ne; t += G) {
            const int rr = s_row[t], k = s_col[t];
            if (rr >= 0 && k >= 0) acc = fma(s_val[t] * Rc[(r0 + rr) * ldr], Rc[(int64_t)k * ldr], acc);
        }
        __syncthreads();
    }
    red[grp][lane] = acc;
    __syncthreads();
    if (grp == 0 && jj < cnt) {
        double sum = red[0][lane];
        for (int g = 1; g < kQuadGroups; ++g) sum += red[g][lane];
        part[(int64_t)blockIdx.y * ldp + c0 + jj] = sum;
    }
}

// ---------------------------------------------------------------------------
// read_stream: every 16-byte vector of a buffer read once (the X-scan's loads,
// non-temporal when NT), values folded into a register and discarded.  The
// bandwidth a scan of that buffer can reach.  Workgroups own contiguous
// chunks; eight loads in flight per thread.
// ---------------------------------------------------------------------------
template <bool NT>
__global__ __launch_bounds__(256) void read_stream_kernel(const u32x4* __restrict__ v, int64_t nvec,
                                                          unsigned key, unsigned* __restrict__ sink) {
    const int64_t per = (nvec + gridDim.x - 1) / gridDim.x;
    const int64_t a = (int64_t)blockIdx.x * per, b = min(nvec, a + per);
    unsigned acc = 0u;
    constexpr int U = 8;
    int64_t i = a + threadIdx.x;
    for (; i + (U - 1) * (int64_t)blockDim.x < b; i += U * (int64_t)blockDim.x) {
        u32x4 r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const u32x4* q = v + i + u * (int64_t)blockDim.x;
            r[u] = NT ? __builtin_nontemporal_load(q) : *q;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= r[u].x ^ r[u].y ^ r[u].z ^ r[u].w;
    }
    for (; i < b; i += blockDim.x) {
        const u32x4 r = v[i];
        acc ^= r.x ^ r.y ^ r.z ^ r.w;
    }
    if (acc == key) *sink = acc;     // keeps the loads; practically never taken
}

// ---------------------------------------------------------------------------
// y32_switch: rbd_fit_basis runs its first steps on the FP64 basis in Y and,
// once the fit passes that many columns, rounds the complete columns
// [0, ncols) into the FP32 basis (the rest of the open block is staged and
// reaches the FP32 basis through the next pass).  Nothing when the fit has
// stopped.
// ---------------------------------------------------------------------------
// Two rows per workgroup of 256 threads, one column per thread (ncols <= 128).
__global__ __launch_bounds__(256) void y32_switch_kernel(const State* __restrict__ st, const double* __restrict__ Y,
                                                          int64_t ldy, float* __restrict__ Yf, int64_t ldyf,
                                                          int64_t m, int ncols) {
    if (st->stop) return;
    const int64_t i = 2 * (int64_t)blockIdx.x + threadIdx.x / 128;
    const int k = threadIdx.x % 128;
    if (i < m && k < ncols) Yf[i * ldyf + k] = (float)Y[i * ldy + k];
}

// ---------------------------------------------------------------------------
// epilogue: col_err = sqrt(e^2), zero unused columns/rows, publish d and status.
// ---------------------------------------------------------------------------
__global__ void epilogue_kernel(const State* __restrict__ st, const double* __restrict__ e2,
                                double* __restrict__ col_err, int64_t n, double* __restrict__ Y, int64_t m,
                                int d_max, double* __restrict__ T, int64_t* __restrict__ pivots,
                                double* __restrict__ err_hist, int32_t* d_out, int32_t* status,
                                int32_t* stop_reason, const float* __restrict__ Yf = nullptr, int64_t ldyf = 0,
                                int ysw = 0) {
    const int d = st->d;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = gid; j < n; j += stride) col_err[j] = sqrt(e2[j]);
    const bool from_f = Yf && d > ysw;   // the FP32 basis was in use (the fit passed column ysw)
    if (from_f) {             // the output is its FP64 copy, zero beyond column d
        const int64_t tot = m * (int64_t)d_max;
        for (int64_t e = gid; e < tot; e += stride) {
            const int64_t i = e / d_max, k = e % d_max;
            Y[e] = k < d ? (double)Yf[i * ldyf + k] : 0.0;
        }
    }
    if (d < d_max) {
        if (!from_f)
            for (int64_t i = gid; i < m; i += stride)
                for (int k = d; k < d_max; ++k) Y[i * d_max + k] = 0.0;
        const int64_t tot = (int64_t)(d_max - d) * n;
        for (int64_t e = gid; e < tot; e += stride) T[(int64_t)d * n + e] = 0.0;
    }
    for (int64_t k = gid; k < d_max; k += stride)
        if (k >= d) pivots[k] = -1;
    for (int64_t k = gid; k <= d_max; k += stride)
        if (k > d) err_hist[k] = 0.0;
    if (gid == 0) {
        *d_out = d;
        *status = st->status;
        if (stop_reason) *stop_reason = (st->stop == kStopError) ? 0 : st->stop;
    }
}

// ---------------------------------------------------------------------------
// fixed-order sums of per-slab partials
// ---------------------------------------------------------------------------
// out[e] = f(sum_{s < S} part[s * len + e]) with f = identity or sqrt.
__global__ void sum_rows_kernel(const double* __restrict__ part, int S, int64_t len, double* __restrict__ out,
                                int take_sqrt) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll 8
        for (int q = 0; q < S; ++q) s += part[(int64_t)q * len + e];      // eight loads in flight, ascending q
        out[e] = take_sqrt ? sqrt(s) : s;
    }
}

}  // namespace rbd
