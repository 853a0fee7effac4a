// Batched Reduced Basis Decomposition: many independent, uneven matrices in one
// persistent launch.  Each workgroup takes the next matrix from a device queue
// (matrices are queued longest first) and runs the whole greedy loop of
// Algorithm 1 (section 3.1) on it with workgroup barriers only, so no grid-wide
// synchronisation is ever needed; every workgroup leaves the loop once the
// queue is drained.
//
// Per matrix b (m x n, row-major, leading dimension n) the workgroup keeps
//   v        the working vector, in LDS (m <= kBatchMaxM)
//   Yt       the basis transposed (D x m, one basis vector per row), its
//            first KL = ycap / m vectors in LDS and the rest in the workspace,
//            so every Gram-Schmidt access is coalesced (or an LDS access);
//            Y_b is written row-major at the end
//   e2, b2   downdated and last exact squared errors (workspace)
// and applies the same certified refresh as rbd_fit: a column whose downdated
// error falls below 2^-20 of its last exact value is re-evaluated exactly
// before the step's argmax and stop test.
#pragma once

#include "rbd_device.h"

namespace rbd {

constexpr int kBatchMaxM = 4096;
constexpr int kBatchMaxD = 256;

// per-matrix descriptor (int64 x 8), built on the host by rbd_batch_plan
enum { kDescM = 0, kDescN, kDescX, kDescY, kDescT, kDescC, kDescW, kDescD, kDescWords };

template <int TPB>
__device__ __forceinline__ double bsum(double v, double* sred) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    constexpr int nw = TPB / kWave;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sred[w] = v;
    __syncthreads();
    double s = sred[0];
#pragma unroll
    for (int k = 1; k < nw; ++k) s += sred[k];
    __syncthreads();
    return s;
}

template <int TPB>
__device__ __forceinline__ void bargmax(double& v, int64_t& i, double* sv, int64_t* si) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    constexpr int nw = TPB / kWave;
    wave_argmax(v, i);
    __syncthreads();
    if (lane == 0) { sv[w] = v; si[w] = i; }
    __syncthreads();
    v = sv[0];
    i = si[0];
#pragma unroll
    for (int k = 1; k < nw; ++k) argmax_merge(v, i, sv[k], si[k]);
    __syncthreads();
}

constexpr int kCPL = 4;   // columns per lane in one pass over the rows
constexpr int kRG = 8;    // queued columns re-evaluated together

// Per-thread partial column sums over this wave's rows (rows w, w+NW, ...):
// t[c] = sum_i w_i x_{i, j0 + lane + 64 c}   (SQR: sum_i x^2).
template <typename Tx, int TPB, bool SQR>
__device__ __forceinline__ void col_pass(const Tx* __restrict__ Xb, int m, int n, int j0,
                                         const double* __restrict__ wts, double (&t)[kCPL]) {
    using L = Ld<Tx>;
    constexpr int NW = TPB / kWave;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < kCPL; ++c) t[c] = 0.0;
    bool ok[kCPL];
#pragma unroll
    for (int c = 0; c < kCPL; ++c) ok[c] = j0 + lane + kWave * c < n;
    // Loads without branches: a lane past the last column reads column 0 of
    // the same row and drops the value.  (A load guarded by a branch, with its
    // conversion in the same branch, waits for its data before the next load
    // issues.)
    int off[kCPL];
#pragma unroll
    for (int c = 0; c < kCPL; ++c) off[c] = ok[c] ? j0 + lane + kWave * c : 0;
    int i = w;
    for (; i + 3 * NW < m; i += 4 * NW) {
        Tx xr[4][kCPL];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const Tx* r = Xb + (int64_t)(i + u * NW) * n;
#pragma unroll
            for (int c = 0; c < kCPL; ++c) xr[u][c] = r[off[c]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double wu = SQR ? 0.0 : wts[i + u * NW];
#pragma unroll
            for (int c = 0; c < kCPL; ++c) {
                const double x = ok[c] ? L::from(xr[u][c]) : 0.0;
                t[c] = SQR ? fma(x, x, t[c]) : fma(wu, x, t[c]);
            }
        }
    }
    for (; i < m; i += NW) {
        const Tx* r0 = Xb + (int64_t)i * n;
        const double w0 = SQR ? 0.0 : wts[i];
        Tx xr[kCPL];
#pragma unroll
        for (int c = 0; c < kCPL; ++c) xr[c] = r0[off[c]];
#pragma unroll
        for (int c = 0; c < kCPL; ++c) {
            const double x = ok[c] ? L::from(xr[c]) : 0.0;
            t[c] = SQR ? fma(x, x, t[c]) : fma(w0, x, t[c]);
        }
    }
}

// red[lane + 64 c] = sum over waves (in order) of the waves' t[c].
template <int TPB>
__device__ __forceinline__ void combine_waves(const double (&t)[kCPL], double* red) {
    constexpr int NW = TPB / kWave;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    double* stage = red + kWave * kCPL;            // NW x (64 kCPL)
#pragma unroll
    for (int c = 0; c < kCPL; ++c) stage[w * kWave * kCPL + lane + kWave * c] = t[c];
    __syncthreads();
    for (int col = threadIdx.x; col < kWave * kCPL; col += TPB) {
        double s = 0.0;
        for (int q = 0; q < NW; ++q) s += stage[q * kWave * kCPL + col];
        red[col] = s;
    }
    __syncthreads();
}

// Block sums of R values per thread, fixed order; results in red[0..R).
template <int TPB, int R>
__device__ __forceinline__ void bsum_n(double (&v)[R], double* red) {
    constexpr int NW = TPB / kWave;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    wave_sum_n<R>(v);
    double* stage = red + R;
    if (lane == 0)
#pragma unroll
        for (int g = 0; g < R; ++g) stage[w * R + g] = v[g];
    __syncthreads();
    if (threadIdx.x < R) {
        double s = 0.0;
        for (int q = 0; q < NW; ++q) s += stage[q * R + threadIdx.x];
        red[threadIdx.x] = s;
    }
    __syncthreads();
}

// sum_{k0<=k<k1} Yt[k*m + i] * h[k] with 8 independent loads in flight (Yt in
// LDS or in global memory; the caller splits the range between the two)
__device__ __forceinline__ double yt_dot(const double* __restrict__ Yt, int64_t m, int i, const double* h, int k0,
                                         int k1) {
    double s0 = 0.0, s1 = 0.0;
    int k = k0;
    for (; k + 8 <= k1; k += 8) {
        double y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) y[u] = Yt[(int64_t)(k + u) * m + i];
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
            s0 = fma(y[u], h[k + u], s0);
            s1 = fma(y[u + 1], h[k + u + 1], s1);
        }
    }
    for (; k < k1; ++k) s0 = fma(Yt[(int64_t)k * m + i], h[k], s0);
    return s0 + s1;
}

__global__ void batch_queue_reset_kernel(unsigned* queue) {
    if (threadIdx.x == 0) *queue = 0u;
}

template <typename Tx, int TPB>
__global__ __launch_bounds__(TPB) void batched_fit_kernel(
    const Tx* __restrict__ X, const int64_t* __restrict__ desc, const int* __restrict__ order, int nitems,
    int stride, unsigned* __restrict__ queue, double tol, int rel, int d_max, double* __restrict__ Yout,
    double* __restrict__ Tout, int64_t* __restrict__ pivots, double* __restrict__ col_err,
    double* __restrict__ err_hist, int32_t* __restrict__ d_out, int32_t* __restrict__ status,
    double* __restrict__ wsd, int vcap, int ycap) {
    using L = Ld<Tx>;
    constexpr int NW = TPB / kWave;
    extern __shared__ double lds[];
    double* vs = lds;                       // m <= vcap
    double* ylds = lds + vcap;              // the first KL basis vectors (KL * m <= ycap)
    __shared__ double h1[kBatchMaxD];
    __shared__ double h2[kBatchMaxD];
    __shared__ double sred[NW];
    __shared__ int64_t sidx[NW];
    __shared__ int s_item, s_nf;
    __shared__ int flist[kWave * kCPL];
    __shared__ double red[kWave * kCPL * (TPB / kWave + 1)];
    __shared__ double tq[(kBatchMaxD + 1) * kRG];     // T(0:d+1, queued group), k-major
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;

    for (;;) {
        if (tid == 0) s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= nitems) break;
        const int b = order[(int64_t)it * stride];
        const int64_t* dsc = desc + (int64_t)b * kDescWords;
        const int m = (int)dsc[kDescM], n = (int)dsc[kDescN], D = (int)dsc[kDescD];
        const Tx* Xb = X + dsc[kDescX];
        double* Yb = Yout + dsc[kDescY];
        double* Tb = Tout + dsc[kDescT];
        double* ceb = col_err + dsc[kDescC];
        double* Yt = wsd + dsc[kDescW];
        double* e2 = Yt + (int64_t)D * m;
        const int KL = min(D, ycap / max(m, 1));    // basis vectors kept in LDS
        // basis vector k (transposed layout, m contiguous values)
        auto ycol = [&](int k) -> double* { return k < KL ? ylds + (int64_t)k * m : Yt + (int64_t)k * m; };
        double* b2 = e2 + n;
        int64_t* pvb = pivots + (int64_t)b * d_max;
        double* ehb = err_hist + (int64_t)b * (d_max + 1);

        // ---- pre-computation: e_j^2 = ||x_j||^2, E_0, first column
        double best = -1.0;
        int64_t bi = INT64_MAX;
        int nonfinite = 0;
        for (int j0 = 0; j0 < n; j0 += kWave * kCPL) {
            double t[kCPL];
            col_pass<Tx, TPB, true>(Xb, m, n, j0, nullptr, t);
            combine_waves<TPB>(t, red);
            for (int c = tid; c < kWave * kCPL; c += TPB) {
                const int j = j0 + c;
                if (j >= n) continue;
                const double s = red[c];
                e2[j] = s;
                b2[j] = s;
                if (!isfinite(s)) nonfinite = 1;
                argmax_merge(best, bi, s, j);
            }
            __syncthreads();
        }
        const double nf = bsum<TPB>((double)nonfinite, sred);
        bargmax<TPB>(best, bi, sred, sidx);
        int d = 0, stop = 0, p = (int)bi;
        int st_code = RBD_OK;
        double tau = 0.0;
        if (nf > 0.0) {
            st_code = RBD_ENONFINITE;
            stop = kStopError;
            if (tid == 0) ehb[0] = NAN;
        } else {
            const double E0 = sqrt(best);
            tau = rel ? tol * E0 : tol;
            if (tid == 0) ehb[0] = E0;
        }

        // ---- greedy loop
        while (!stop && d < D) {
            // step 2.1 + first Gram-Schmidt pass: v = x_p - Y h1, h1 = T(0:d, p)
            for (int k = tid; k < d; k += TPB) h1[k] = Tb[(int64_t)k * n + p];
            __syncthreads();
            for (int i = tid; i < m; i += TPB)
                vs[i] = L::one(Xb + (int64_t)i * n + p) - yt_dot(ylds, m, i, h1, 0, min(d, KL)) -
                        yt_dot(Yt, m, i, h1, min(d, KL), d);
            __syncthreads();
            // h2 = Y' v1: one wave per basis vector
            auto col_dot = [&](const double* __restrict__ yk) {
                double s0 = 0.0, s1 = 0.0;
                int i = lane;
                for (; i + 3 * kWave < m; i += 4 * kWave) {
                    const double a0 = yk[i], a1 = yk[i + kWave], a2 = yk[i + 2 * kWave], a3 = yk[i + 3 * kWave];
                    s0 = fma(a0, vs[i], s0);
                    s1 = fma(a1, vs[i + kWave], s1);
                    s0 = fma(a2, vs[i + 2 * kWave], s0);
                    s1 = fma(a3, vs[i + 3 * kWave], s1);
                }
                for (; i < m; i += kWave) s0 = fma(yk[i], vs[i], s0);
                return wave_sum(s0 + s1);
            };
            for (int k = w; k < d; k += NW) {
                const double sw = k < KL ? col_dot(ylds + (int64_t)k * m) : col_dot(Yt + (int64_t)k * m);
                if (lane == 0) h2[k] = sw;
            }
            __syncthreads();
            // second pass and its norm
            double acc = 0.0;
            for (int i = tid; i < m; i += TPB) {
                const double v = vs[i] - yt_dot(ylds, m, i, h2, 0, min(d, KL)) - yt_dot(Yt, m, i, h2, min(d, KL), d);
                vs[i] = v;
                acc = fma(v, v, acc);
            }
            const double nu = sqrt(bsum<TPB>(acc, sred));
            if (nu < tau || nu == 0.0) {      // step 2.2: keep the d vectors found so far
                stop = RBD_STOP_BREAK;
                break;
            }
            const double inv = 1.0 / nu;
            for (int i = tid; i < m; i += TPB) {
                const double xi = vs[i] * inv;
                vs[i] = xi;
                ycol(d)[i] = xi;
            }
            __syncthreads();
            // T(d, :) = xi' X, downdate, queue columns for exact evaluation
            if (tid == 0) s_nf = 0;
            __syncthreads();
            for (int j0 = 0; j0 < n; j0 += kWave * kCPL) {
                double t[kCPL];
                col_pass<Tx, TPB, false>(Xb, m, n, j0, vs, t);
                combine_waves<TPB>(t, red);
                for (int c = tid; c < kWave * kCPL; c += TPB) {
                    const int j = j0 + c;
                    if (j >= n) continue;
                    const double tj = red[c];
                    Tb[(int64_t)d * n + j] = tj;
                    double e = e2[j] - tj * tj;
                    if (!(e > 0.0)) e = 0.0;
                    double bb = b2[j];
                    if (j == p) {
                        e = 0.0;
                        bb = 0.0;
                        b2[j] = 0.0;
                    }
                    e2[j] = e;
                    if (e < kRefresh * bb) flist[atomicAdd(&s_nf, 1)] = j;   // at most 64*kCPL per pass
                }
                __syncthreads();
                // exact ||x_j - Y T(:, j)||^2 for the queued columns, kRG at a time
                const int nq = s_nf;
                for (int q0 = 0; q0 < nq; q0 += kRG) {
                    double r2[kRG];
#pragma unroll
                    for (int g = 0; g < kRG; ++g) r2[g] = 0.0;
                    // the group's columns of T(0:d+1, :) into LDS once (every row reads all of them)
                    for (int e = tid; e < (d + 1) * kRG; e += TPB)
                        tq[e] = Tb[(int64_t)(e / kRG) * n + flist[min(q0 + e % kRG, nq - 1)]];
                    __syncthreads();
                    for (int i = tid; i < m; i += TPB) {
                        double acc[kRG];
#pragma unroll
                        for (int g = 0; g < kRG; ++g) acc[g] = 0.0;
                        auto part_sum = [&](const double* __restrict__ Yp, int k0, int k1) {
                            int k = k0;
                            for (; k + 4 <= k1; k += 4) {
                                double y[4];
#pragma unroll
                                for (int u = 0; u < 4; ++u) y[u] = Yp[(int64_t)(k + u) * m + i];
#pragma unroll
                                for (int u = 0; u < 4; ++u)
#pragma unroll
                                    for (int g = 0; g < kRG; ++g) acc[g] = fma(y[u], tq[(k + u) * kRG + g], acc[g]);
                            }
                            for (; k < k1; ++k) {
                                const double y = Yp[(int64_t)k * m + i];
#pragma unroll
                                for (int g = 0; g < kRG; ++g) acc[g] = fma(y, tq[k * kRG + g], acc[g]);
                            }
                        };
                        part_sum(ylds, 0, min(d + 1, KL));
                        part_sum(Yt, min(d + 1, KL), d + 1);
                        Tx xr[kRG];      // past the queue's end: a repeat of its first entry, unused
#pragma unroll
                        for (int g = 0; g < kRG; ++g) xr[g] = Xb[(int64_t)i * n + flist[q0 + g < nq ? q0 + g : q0]];
#pragma unroll
                        for (int g = 0; g < kRG; ++g)
                            if (q0 + g < nq) {
                                const double r = L::from(xr[g]) - acc[g];
                                r2[g] = fma(r, r, r2[g]);
                            }
                    }
                    bsum_n<TPB, kRG>(r2, red);
                    if (tid < kRG && q0 + tid < nq) {
                        const int j = flist[q0 + tid];
                        e2[j] = red[tid];
                        b2[j] = red[tid];
                    }
                    __syncthreads();
                }
                if (tid == 0) s_nf = 0;
                __syncthreads();
            }
            // step 2.3: E_cur and the next column (lowest index on ties)
            best = -1.0;
            bi = INT64_MAX;
            for (int j = tid; j < n; j += TPB) argmax_merge(best, bi, e2[j], j);
            bargmax<TPB>(best, bi, sred, sidx);
            const double E = sqrt(best);
            if (tid == 0) {
                pvb[d] = p;
                ehb[d + 1] = E;
            }
            ++d;
            p = (int)bi;
            if (E <= tau) stop = RBD_STOP_TOL;       // step 2.4
            else if (d >= D) stop = RBD_STOP_DMAX;
            __syncthreads();
        }

        // ---- outputs: col_err, Y (row-major, zero past d), T rows past d, history
        for (int j = tid; j < n; j += TPB) ceb[j] = sqrt(e2[j]);
        for (int64_t e = tid; e < (int64_t)m * d_max; e += TPB) {
            const int i = (int)(e / d_max), k = (int)(e % d_max);
            Yb[e] = k < d ? (k < KL ? ylds[(int64_t)k * m + i] : Yt[(int64_t)k * m + i]) : 0.0;
        }
        for (int64_t e = (int64_t)d * n + tid; e < (int64_t)d_max * n; e += TPB) Tb[e] = 0.0;
        for (int k = d + tid; k < d_max; k += TPB) pvb[k] = -1;
        for (int k = d + 1 + tid; k <= d_max; k += TPB) ehb[k] = 0.0;
        if (tid == 0) {
            d_out[b] = d;
            status[b] = st_code;
        }
        __syncthreads();
    }
}

}  // namespace rbd
