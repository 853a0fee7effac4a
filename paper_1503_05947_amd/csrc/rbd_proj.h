// Projection onto the basis on the FP64 matrix cores: C = Y(:, 0:d)' V.
// This is the compression of out-of-sample data of section 3.1 (the
// coefficients of each column of V in the orthonormal basis Y); it serves the
// out-of-sample projection and the recognition of section 4.
#pragma once

#include <algorithm>
#include <cstdint>

#include "rbd_gemm.h"

namespace rbd {

inline int64_t proj_cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// proj_mfma: C = Y(:, 0:d)' V (d x N result) on the FP64 matrix cores.  Y
// is m x d FP64 row-major (ldy), V is m x N row-major (ldv) stored as Tv.  A
// workgroup owns MT*16 <= 64 rows of C (grid.y) and 256 columns (grid.x, 64
// per wave); grid.z splits the k range (rows of Y and V), writing partials
// when it is larger than 1.  MFMA operands (16x16x4): lane l supplies
// A(l % 16, l / 16) = Y(k0 + l/16, i0 + l % 16) and, for the e-th 16-column
// tile, B(l / 16, l % 16) = V(k0 + l/16, j0 + 4 (l % 16) + e): each lane
// reads four adjacent columns of V with one vector load, and the results are
// written back through the same column permutation.
// ---------------------------------------------------------------------------
// Four adjacent stored values of V, kept in their storage format until use.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
template <typename Tv> struct Raw4;
template <> struct Raw4<float> {
    f32x4 v;
    __device__ __forceinline__ void load(const float* p) { v = *reinterpret_cast<const f32x4*>(p); }
    __device__ __forceinline__ void load_some(const float* p, int cnt) {
        v = (f32x4){cnt > 0 ? p[0] : 0.f, cnt > 1 ? p[1] : 0.f, cnt > 2 ? p[2] : 0.f, cnt > 3 ? p[3] : 0.f};
    }
    __device__ __forceinline__ void zero() { v = (f32x4){0.f, 0.f, 0.f, 0.f}; }
    __device__ __forceinline__ double get(int e) const { return (double)v[e]; }
};
template <> struct Raw4<double> {
    f64x2 v0, v1;
    __device__ __forceinline__ void load(const double* p) {
        v0 = reinterpret_cast<const f64x2*>(p)[0];
        v1 = reinterpret_cast<const f64x2*>(p)[1];
    }
    __device__ __forceinline__ void load_some(const double* p, int cnt) {
        v0 = (f64x2){cnt > 0 ? p[0] : 0.0, cnt > 1 ? p[1] : 0.0};
        v1 = (f64x2){cnt > 2 ? p[2] : 0.0, cnt > 3 ? p[3] : 0.0};
    }
    __device__ __forceinline__ void zero() { v0 = v1 = (f64x2){0.0, 0.0}; }
    __device__ __forceinline__ double get(int e) const { return e < 2 ? v0[e] : v1[e - 2]; }
};
template <typename H> struct Raw4Half {       // BF16 / FP16: four 16-bit values in two words
    u32x2_t v;
    __device__ __forceinline__ void load(const H* p) { v = *reinterpret_cast<const u32x2_t*>(p); }
    __device__ __forceinline__ void load_some(const H* p, int cnt) {
        const unsigned a = cnt > 0 ? p[0].u : 0u, b = cnt > 1 ? p[1].u : 0u;
        const unsigned c = cnt > 2 ? p[2].u : 0u, d = cnt > 3 ? p[3].u : 0u;
        v = (u32x2_t){a | (b << 16), c | (d << 16)};
    }
    __device__ __forceinline__ void zero() { v = (u32x2_t){0u, 0u}; }
};
template <> struct Raw4<bf16_t> : Raw4Half<bf16_t> {
    __device__ __forceinline__ double get(int e) const { return e & 1 ? bf16_hi(v[e >> 1]) : bf16_lo(v[e >> 1]); }
};
template <> struct Raw4<f16_t> : Raw4Half<f16_t> {
    __device__ __forceinline__ double get(int e) const { return e & 1 ? f16_hi(v[e >> 1]) : f16_lo(v[e >> 1]); }
};

typedef double f64x4_t __attribute__((ext_vector_type(4)));
constexpr int kProjCols = 256;      // columns per workgroup
// Waves per SIMD: three where the accumulators leave room (up to 32 rows of C,
// or 48 for FP32 queries: 6.35 -> 5.2-5.3 ms for a batch of 262,144 FP32
// queries of 10,304 entries against two per SIMD), two otherwise (one wave per SIMD left the
// matrix cores idle most of the time) ...
template <typename Tv, int MT> constexpr int proj_occupancy() {
    return (MT <= 2 || (sizeof(Tv) == 4 && MT == 3)) ? 3 : 2;
}
// ... and the k-steps of operands held in registers within that budget ...
template <typename Tv, int MT> constexpr int proj_regs() {
    return proj_occupancy<Tv, MT>() == 3 ? 4
                                          : ((sizeof(Tv) == 8 && MT == 4) ? 2 : ((sizeof(Tv) == 8 || MT == 4) ? 4 : 8));
}
// ... held as B buffers of G k-steps (B * G = proj_regs): while one buffer is
// multiplied, B - 1 are in flight
template <typename Tv, int MT> constexpr int proj_group() { return proj_regs<Tv, MT>() >= 8 ? 2 : 1; }
template <typename Tv, int MT> constexpr int proj_bufs() { return proj_regs<Tv, MT>() / proj_group<Tv, MT>(); }
constexpr int kProjStepMax = 16;    // row chunks of a k-split are a multiple of this

template <typename Tv, int MT>
__global__ __launch_bounds__(256, (proj_occupancy<Tv, MT>())) void proj_mfma_kernel(const double* __restrict__ Y, int64_t ldy, int64_t m, int d,
                                                         const Tv* __restrict__ V, int64_t ldv, int64_t N,
                                                         int64_t kchunk, int vec_ok, double* __restrict__ C,
                                                         int64_t ldc, double* __restrict__ part) {
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int lr = lane % 16, lk = lane / 16;
    const int i0 = blockIdx.y * 64;
    const int64_t j0 = (int64_t)blockIdx.x * kProjCols + wv * 64;
    const int64_t jl = j0 + 4 * lr;                 // this lane's four columns jl .. jl + 3
    const bool full = vec_ok && jl + 3 < N;
    const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = min(m, kb + kchunk);
    if (j0 >= N) return;                            // no columns for this wave (no barriers below)
    f64x4_t acc[MT][4];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[t][e] = (f64x4_t){0.0, 0.0, 0.0, 0.0};
    constexpr int kProjGroup = proj_group<Tv, MT>(), kBufs = proj_bufs<Tv, MT>();
    double a[kBufs][kProjGroup][MT];
    Raw4<Tv> b[kBufs][kProjGroup];
    auto load = [&](double (&a)[kProjGroup][MT], Raw4<Tv> (&b)[kProjGroup], int64_t k0) {
#pragma unroll
        for (int g = 0; g < kProjGroup; ++g) {
            const int64_t k = k0 + 4 * g + lk;
            const bool okk = k < ke;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const int i = i0 + 16 * t + lr;
                a[g][t] = (okk && i < d) ? Y[k * ldy + i] : 0.0;
            }
            if (okk && full) b[g].load(V + k * ldv + jl);
            else if (okk && jl < N) b[g].load_some(V + k * ldv + jl, (int)min((int64_t)4, N - jl));
            else b[g].zero();
        }
    };
    auto mult = [&](const double (&a)[kProjGroup][MT], const Raw4<Tv> (&b)[kProjGroup]) {
#pragma unroll
        for (int g = 0; g < kProjGroup; ++g)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double be = b[g].get(e);
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    acc[t][e] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[g][t], be, acc[t][e], 0, 0, 0);
            }
    };
    // B groups per iteration, the buffers in rotation, and a single exit (an
    // exit inside the rotation made the compiler keep two sets of
    // accumulators: 1 wave per SIMD).  Loads past the end of the chunk give
    // zeros, so a group count that is not a multiple of B costs up to B - 1
    // groups of products with zeros.
    constexpr int kStep = 4 * kProjGroup;
#pragma unroll
    for (int q = 0; q + 1 < kBufs; ++q) load(a[q], b[q], kb + q * kStep);
    for (int64_t k0 = kb; k0 < ke; k0 += kBufs * kStep) {
#pragma unroll
        for (int q = 0; q < kBufs; ++q) {
            load(a[(q + kBufs - 1) % kBufs], b[(q + kBufs - 1) % kBufs], k0 + (q + kBufs - 1) * kStep);
            mult(a[q], b[q]);
        }
    }
    double* out = part ? part + (int64_t)blockIdx.z * d * N : C;
    const int64_t ldo = part ? N : ldc;
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 16 * t + 4 * r + lk;
            if (i >= d) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (jl + e < N) out[(int64_t)i * ldo + jl + e] = acc[t][e][r];
        }
}

template <typename Tv>
inline hipError_t proj_mfma(const double* Y, int64_t ldy, int64_t m, int d, const Tv* V, int64_t ldv, int64_t N, double* C,
                     int64_t ldc, double* part, size_t part_elems, hipStream_t s) {
    const int64_t ctiles = proj_cdiv(N, kProjCols), rtiles = proj_cdiv(d, 64);
    int64_t splits = 1;
    while (ctiles * rtiles * splits < 1024 && m / (splits * 2) >= 1024 && (size_t)(splits * 2) * d * N <= part_elems)
        splits *= 2;
    const int64_t kchunk = proj_cdiv(proj_cdiv(m, splits), kProjStepMax) * kProjStepMax;
    splits = std::max<int64_t>(1, proj_cdiv(m, kchunk));
    const int vec_ok = (ldv % 4 == 0) && (reinterpret_cast<uintptr_t>(V) % (4 * sizeof(Tv)) == 0);
    const dim3 grid((unsigned)ctiles, (unsigned)rtiles, (unsigned)splits);
    double* pp = splits > 1 ? part : nullptr;
    // row tiles of 64 (MT = 4) except a last, narrower one
    const int mt_last = (int)proj_cdiv(d - 64 * (rtiles - 1), 16);
    auto launch = [&](int mt, dim3 g, int i0_tiles) {
        (void)i0_tiles;
        switch (mt) {
            case 1: proj_mfma_kernel<Tv, 1><<<g, 256, 0, s>>>(Y, ldy, m, d, V, ldv, N, kchunk, vec_ok, C, ldc, pp); break;
            case 2: proj_mfma_kernel<Tv, 2><<<g, 256, 0, s>>>(Y, ldy, m, d, V, ldv, N, kchunk, vec_ok, C, ldc, pp); break;
            case 3: proj_mfma_kernel<Tv, 3><<<g, 256, 0, s>>>(Y, ldy, m, d, V, ldv, N, kchunk, vec_ok, C, ldc, pp); break;
            default: proj_mfma_kernel<Tv, 4><<<g, 256, 0, s>>>(Y, ldy, m, d, V, ldv, N, kchunk, vec_ok, C, ldc, pp); break;
        }
    };
    // one launch: rows past d are skipped inside, so MT = 4 serves every full row tile and
    // the narrower last tile only matters when it is the only one
    launch(rtiles == 1 ? mt_last : 4, grid, 0);
    if (splits > 1) launch_split_sum(d, N, (int)splits, 1.0, part, 0.0, C, ldc, s);
    return hipGetLastError();
}

}  // namespace rbd
