// FP64 GEMM on the matrix cores (v_mfma_f64_16x16x4f64) for the dense
// contractions of the reconstruction Y T and its backward:
//   C = alpha * op(A) op(B) + beta * C      (op = identity or transpose)
// A and B are row-major with leading dimensions lda / ldb and may be stored
// in FP64, FP32, BF16 or FP16 (widened exactly to FP64 when staged).
//
// Tiling: 128 x 128 output tile per workgroup (4 waves, 64 x 64 each, i.e.
// 4 x 4 MFMA tiles of 16 x 16), k staged through LDS 16 deep with the next
// chunk's loads in flight while the current one is multiplied.  Two waves per
// SIMD: the launch bound keeps the kernel within 256 registers (the
// accumulators then live in the unified VGPR file); at one wave per SIMD the
// matrix cores idled during every chunk's LDS phase.  MFMA operand
// layout (16x16x4, wave64): lane l supplies A(l % 16, l / 16) and
// B(l / 16, l % 16); accumulator register r of lane l holds C(4 r + l / 16,
// l % 16).  With `splits` > 1 the k range is divided over blockIdx.z and each
// split writes its own partial tile to `part` (split-major, M x N each), to be
// summed in a fixed order by gemm_split_sum_kernel.
#pragma once

#include <algorithm>
#include <type_traits>

#include "rbd_device.h"

namespace rbd {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kGN = 128, kGK = 16;
constexpr int64_t kShortK = 256;      // k ranges up to this use the 64-row tiles when they make >= 1024 tiles

// WM: rows of each wave's sub-tile (64, or 32 for short k ranges: half the
// accumulators, so three workgroups per CU instead of two hide the prologue
// and the epilogue of each other's tiles).
template <int WM>
struct GemmShape {
    static constexpr int GM = 2 * WM;              // workgroup tile rows
    static constexpr int MT = WM / 16;             // MFMA tiles per wave along M
    static constexpr int WG_PER_CU = WM == 64 ? 2 : 3;
};

// Optional extra columns of the product (single-split products only):
// C += A2 E, where E (n2 x N) is one in row colrank[j] of column j when
// colrank[j] >= 0 and zero elsewhere, i.e. output column j gains column
// colrank[j] of A2 (M x n2, leading dimension ld2).  colrank has N + 1 entries
// and is increasing in the sense that a column's rank, or -1 - (its insertion
// point) for columns that gain nothing, never decreases with j, so a wave's
// 64 columns gain the contiguous range of A2's columns [lo_w, hi_w) decoded
// from colrank at its first column and the one past its last: they run as
// extra k-steps of the wave, with E generated in place.  Products by exact
// zeros and ones add nothing else (each column has at most one rank), so each
// gaining entry is (A B)(i, j) + A2(i, colrank[j]) with one rounding.
struct GemmColAdd {
    const double* a2 = nullptr;
    int64_t ld2 = 0;
    const int* colrank = nullptr;
};

template <bool TA, bool TB, typename TAe, typename TBe, int WM = 64, bool ADD = false>
__global__ __launch_bounds__(256, GemmShape<WM>::WG_PER_CU) void gemm_f64_kernel(
    int64_t M, int64_t N, int64_t K, double alpha, const TAe* __restrict__ A, int64_t lda,
    const TBe* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C, int64_t ldc, int64_t kchunk,
    double* __restrict__ part, GemmColAdd add) {
    constexpr int kGM = GemmShape<WM>::GM, MT = GemmShape<WM>::MT;
    __shared__ double As[kGK][kGM + 1];
    __shared__ double Bs[kGK][kGN + 1];
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
    const int wr = (w >> 1) * WM, wc = (w & 1) * 64;       // this wave's WM x 64 sub-tile
    const int64_t row0 = (int64_t)blockIdx.y * kGM, col0 = (int64_t)blockIdx.x * kGN;
    const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    f64x4 acc[MT][4];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};

    // the next chunk's operands are loaded into registers while the current
    // chunk, already in LDS, is multiplied; they stay in their storage format
    // until they go to LDS (a conversion right after a guarded load would make
    // each load wait for its data before the next one issues)
    constexpr int QA = (kGM * kGK) / 256, QB = (kGN * kGK) / 256;
    TAe ra[QA];
    TBe rb[QB];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + 256 * q;
            int i, k;
            if (TA) { k = e / kGM; i = e % kGM; }     // A stored K x M: rows of A are k
            else { i = e / kGK; k = e % kGK; }        // A stored M x K
            const int64_t gi = row0 + i, gk = k0 + k;
            ra[q] = (gi < M && gk < ke) ? (TA ? A[gk * lda + gi] : A[gi * lda + gk]) : TAe{};
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + 256 * q;
            int j, k;
            if (TB) { j = e / kGK; k = e % kGK; }     // B stored N x K
            else { k = e / kGN; j = e % kGN; }        // B stored K x N
            const int64_t gj = col0 + j, gk = k0 + k;
            rb[q] = (gj < N && gk < ke) ? (TB ? B[gj * ldb + gk] : B[gk * ldb + gj]) : TBe{};
        }
    };
    // the extra columns (see GemmColAdd): each wave adds A2's columns
    // [lo_w, hi_w), those its own 64 columns gain, as extra k-steps taken from
    // registers, with no LDS and no barrier: each lane loads its MFMA operands of
    // A2 itself (the first kAddPre k-steps during the tile's last chunk) and
    // forms E's from the rank of its column
    auto dec = [](int r) { return r >= 0 ? r : -1 - r; };
    int lo_w = 0, hi_w = 0;
    if (ADD) {
        lo_w = dec(add.colrank[min(col0 + wc, N)]);
        hi_w = dec(add.colrank[min(col0 + wc + 64, N)]);
    }
    constexpr int kAddPre = 2;
    double pa[kAddPre][MT];
    int cr[4];
    auto load_add = [&](int s, double (&v)[MT]) {      // k-step s: ranks lo_w + 4 s + (0 .. 3)
        const int r = lo_w + 4 * s + lane / 16;
#pragma unroll
        for (int a = 0; a < MT; ++a) {
            const int64_t gi = row0 + wr + a * 16 + lane % 16;
            v[a] = (gi < M && r < hi_w) ? add.a2[gi * add.ld2 + r] : 0.0;
        }
    };
    auto prefetch_add = [&]() {
#pragma unroll
        for (int q = 0; q < kAddPre; ++q) load_add(q, pa[q]);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t gj = col0 + wc + b * 16 + lane % 16;
            cr[b] = gj < N ? add.colrank[gj] : -1;
        }
    };
    // one chunk: stage the operands loaded one chunk earlier, then load the
    // next chunk's (LAST: the extra columns' instead) while multiplying
    auto chunk = [&](int64_t k0, auto last) {
        __syncthreads();      // the previous chunk's products are done with LDS
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + 256 * q;
            if (TA) As[e / kGM][e % kGM] = Ld<TAe>::from(ra[q]);
            else As[e % kGK][e / kGK] = Ld<TAe>::from(ra[q]);
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + 256 * q;
            if (TB) Bs[e % kGK][e / kGK] = Ld<TBe>::from(rb[q]);
            else Bs[e / kGN][e % kGN] = Ld<TBe>::from(rb[q]);
        }
        __syncthreads();
        if constexpr (!decltype(last)::value) load(k0 + kGK);
        else if (ADD && lo_w < hi_w) prefetch_add();
#pragma unroll
        for (int ks = 0; ks < kGK; ks += 4) {
            double af[MT], bf[4];
#pragma unroll
            for (int a = 0; a < MT; ++a) af[a] = As[ks + lane / 16][wr + a * 16 + lane % 16];
#pragma unroll
            for (int b = 0; b < 4; ++b) bf[b] = Bs[ks + lane / 16][wc + b * 16 + lane % 16];
#pragma unroll
            for (int a = 0; a < MT; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
    };
    // the last chunk peeled off, so that what it prefetches for the extra
    // columns is not live across the loop
    int64_t k0 = kb;
    if (kb < ke) load(kb);
    for (; k0 + kGK < ke; k0 += kGK) chunk(k0, std::false_type{});
    if (k0 < ke) chunk(k0, std::true_type{});
    if (ADD && lo_w < hi_w) {
        if (!(kb < ke)) prefetch_add();               // no chunk of the product to hide it behind
        auto mul = [&](const double (&af)[MT], int s) {
            const int r = lo_w + 4 * s + lane / 16;
            double bf[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) bf[b] = cr[b] == r ? 1.0 : 0.0;
#pragma unroll
            for (int a = 0; a < MT; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        };
        const int nsteps = (hi_w - lo_w + 3) / 4;
#pragma unroll
        for (int q = 0; q < kAddPre; ++q)
            if (q < nsteps) mul(pa[q], q);
        for (int q = kAddPre; q < nsteps; ++q) {
            double af[MT];
            load_add(q, af);
            mul(af, q);
        }
    }
    double* out = part ? part + (int64_t)blockIdx.z * M * N : nullptr;
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = row0 + wr + a * 16 + 4 * r + lane / 16;
                const int64_t gj = col0 + wc + b * 16 + lane % 16;
                if (gi < M && gj < N) {
                    if (out) {
                        out[gi * N + gj] = acc[a][b][r];
                    } else {
                        const double prev = beta != 0.0 ? C[gi * ldc + gj] : 0.0;
                        C[gi * ldc + gj] = alpha * acc[a][b][r] + beta * prev;
                    }
                }
            }
}

// C = alpha * sum_{s < splits} part[s] + beta * C in a fixed order: eight
// interleaved chains (split q goes to chain q % 8, eight loads in flight per
// thread), then the chains in order.
static __global__ __launch_bounds__(256) void gemm_split_sum_kernel(int64_t M, int64_t N, int splits, double alpha,
                                                              const double* __restrict__ part, double beta,
                                                              double* __restrict__ C, int64_t ldc) {
    const int64_t tot = M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        double g[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int q = 0;
        for (; q + 8 <= splits; q += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) g[u] += part[(int64_t)(q + u) * tot + e];
        }
        for (int u = 0; q < splits; ++q, ++u) g[u] += part[(int64_t)q * tot + e];
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) s += g[u];
        const int64_t i = e / N, j = e % N;
        const double prev = beta != 0.0 ? C[i * ldc + j] : 0.0;
        C[i * ldc + j] = alpha * s + beta * prev;
    }
}

// The same sums for outputs too small to fill the GPU with one thread per
// entry: the eight chains of an entry run on eight adjacent threads, and the
// chain sums are added in the same order from LDS (bit-identical results).
static __global__ __launch_bounds__(256) void gemm_split_sum8_kernel(int64_t M, int64_t N, int splits, double alpha,
                                                               const double* __restrict__ part, double beta,
                                                               double* __restrict__ C, int64_t ldc) {
    __shared__ double gs[256];
    const int64_t tot = M * N;
    const int u = threadIdx.x % 8;
    const int64_t e = (int64_t)blockIdx.x * 32 + threadIdx.x / 8;
    double g = 0.0;
    if (e < tot) {
#pragma unroll 4
        for (int q = u; q < splits; q += 8) g += part[(int64_t)q * tot + e];
    }
    gs[threadIdx.x] = g;
    __syncthreads();
    if (u == 0 && e < tot) {
        double sum = 0.0;
#pragma unroll
        for (int v = 0; v < 8; ++v) sum += gs[threadIdx.x + v];
        const int64_t i = e / N, j = e % N;
        const double prev = beta != 0.0 ? C[i * ldc + j] : 0.0;
        C[i * ldc + j] = alpha * sum + beta * prev;
    }
}

// C = alpha * sum of the split partials + beta * C (either kernel above)
inline void launch_split_sum(int64_t M, int64_t N, int splits, double alpha, const double* part, double beta,
                             double* C, int64_t ldc, hipStream_t s) {
    const int64_t tot = M * N;
    if (tot <= 65536)
        gemm_split_sum8_kernel<<<(unsigned)((tot + 31) / 32), 256, 0, s>>>(M, N, splits, alpha, part, beta, C, ldc);
    else
        gemm_split_sum_kernel<<<(unsigned)std::min<int64_t>(4096, (tot + 255) / 256), 256, 0, s>>>(
            M, N, splits, alpha, part, beta, C, ldc);
}

constexpr size_t kPartElems = (size_t)8 << 20;   // split-k partials: 64 MB

// Host side: C = alpha op(A) op(B) + beta C.  The k range is split (partials
// in `part`, at most part_elems doubles, summed in a fixed order) while the
// output tiles alone would leave the GPU mostly idle.
template <bool TA, bool TB, typename TAe, typename TBe>
inline hipError_t gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const TAe* A, int64_t lda, const TBe* B,
                           int64_t ldb, double beta, double* C, int64_t ldc, double* part, size_t part_elems,
                           hipStream_t s, GemmColAdd add = {}) {
    auto cdiv = [](int64_t a, int64_t b) { return (a + b - 1) / b; };
    constexpr int kGM = GemmShape<64>::GM;
    const int64_t tiles = cdiv(M, kGM) * cdiv(N, kGN);
    int64_t splits = 1;
    while (part && !add.a2 && tiles * splits < 512 && K / (splits * 2) >= 256 && (size_t)(splits * 2) * M * N <= part_elems)
        splits *= 2;
    const int64_t kchunk = cdiv(cdiv(K, splits), kGK) * kGK;
    splits = std::max<int64_t>(1, cdiv(K, kchunk));
    if (splits == 1 && K <= kShortK && tiles >= 1024) {
        // a short k range over many tiles: 64 x 128 tiles, three workgroups per CU
        constexpr int gm = GemmShape<32>::GM;
        const dim3 grid((unsigned)cdiv(N, kGN), (unsigned)cdiv(M, gm), 1u);
        if (add.a2)
            gemm_f64_kernel<TA, TB, TAe, TBe, 32, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                                          ldc, kchunk, nullptr, add);
        else
            gemm_f64_kernel<TA, TB, TAe, TBe, 32><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                                                        kchunk, nullptr, add);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)cdiv(N, kGN), (unsigned)cdiv(M, kGM), (unsigned)splits);
    if (add.a2)
        gemm_f64_kernel<TA, TB, TAe, TBe, 64, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                                                      kchunk, nullptr, add);
    else
        gemm_f64_kernel<TA, TB, TAe, TBe><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk,
                                                                splits > 1 ? part : nullptr, add);
    if (splits > 1) launch_split_sum(M, N, (int)splits, alpha, part, beta, C, ldc, s);
    return hipGetLastError();
}

}  // namespace rbd
