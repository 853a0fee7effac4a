// Reconstruction Z = Y T (section 3.1, "Uncompress") and its backward with
// the pivots held fixed.
//
// With the pivots P fixed, the basis is the Q factor of A = X(:, P) = Y R
// (Gram-Schmidt of the pivot columns in order; R = T(:, P) is upper
// triangular with positive diagonal), and T = Y'X.  For L = <G, Y Y' X>:
//   dL/dX        = Y (Y'G)                       (through T)
//              + scatter_P( (Ybar + Y copyltu(M)) R^{-T} )   (through Y)
// (scatter_P adds column k of its argument to column piv[k]; it runs inside
// the product that writes Y (Y'G), so dX is written once.)
//   Ybar = dL/dY = G T' + X (G'Y),   M = -Ybar' Y,
//   copyltu(M)   = tril(M) + tril(M, -1)'
// i.e. the standard adjoint of the QR factorisation with Rbar = 0.  Every
// product is an FP64 GEMM on the matrix cores (rbd_gemm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/rbd.h"
#include "rbd_gemm.h"

namespace {

using namespace rbd;

int64_t cd(int64_t a, int64_t b) { return (a + b - 1) / b; }
size_t al(size_t x) { return (x + 255) / 256 * 256; }

template <bool TA, bool TB, typename TAe, typename TBe>
hipError_t gemm(int64_t M, int64_t N, int64_t K, double alpha, const TAe* A, int64_t lda, const TBe* B, int64_t ldb,
                double beta, double* C, int64_t ldc, double* part, size_t part_elems, hipStream_t s) {
    return gemm_f64<TA, TB, TAe, TBe>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, part_elems, s);
}

// Pivot ranks.  colrank[j], j = 0..n: the rank of column j among the pivots
// ordered by column index when j is a pivot, else -1 - (the number of pivots
// below j), so that the pivots among columns [a, b) have the ranks
// [dec(colrank[a]), dec(colrank[b])) with dec(r) = r >= 0 ? r : -1 - r;
// rank[k] = the rank of pivot k (ties, which distinct pivots never have, are
// broken by position, so ranks are distinct).  One thread per column and per
// pivot, the pivots staged in LDS.
// With Rp, the same launch also gathers R's upper triangle packed by columns
// (column i holds R(0..i, i) at i (i + 1) / 2) and the reciprocals of its
// diagonal after it, once, for the inverse below.
__global__ __launch_bounds__(256) void pivot_rank_kernel(const int64_t* __restrict__ piv, int d, int64_t n,
                                                         int* __restrict__ colrank, int* __restrict__ rank,
                                                         const double* __restrict__ T, int64_t ldt,
                                                         double* __restrict__ Rp) {
    __shared__ int64_t ps[RBD_MAX_D];
    for (int k = threadIdx.x; k < d; k += blockDim.x) ps[k] = piv[k];
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (Rp) {
        const int64_t tri = (int64_t)d * (d + 1) / 2;
        for (int64_t e = j; e < tri; e += (int64_t)gridDim.x * blockDim.x) {
            int64_t i = (int64_t)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);      // column: i (i + 1) / 2 <= e
            while (i * (i + 1) / 2 > e) --i;
            while ((i + 1) * (i + 2) / 2 <= e) ++i;
            const int64_t k = e - i * (i + 1) / 2;
            const double v = T[k * ldt + ps[i]];
            Rp[e] = v;
            if (k == i) Rp[tri + i] = 1.0 / v;
        }
    }
    if (j <= n) {
        int lb = 0;
        bool hit = false;
        for (int i = 0; i < d; ++i) {
            lb += ps[i] < j;
            hit |= ps[i] == j;
        }
        colrank[j] = (hit && j < n) ? lb : -1 - lb;
    }
    if (j < d) {
        const int64_t pj = ps[j];
        int r = 0;
        for (int i = 0; i < d; ++i) r += (ps[i] < pj) || (ps[i] == pj && i < j);
        rank[j] = r;
    }
}

// Rinv' = R^{-1} with its rows in pivot-rank order: row rank[k] holds row k
// of R^{-1} (R upper triangular, d x d, R(i, k) = T(i, piv[k]) for i <= k).
// Then column rank[k] of Ybar Rinv'^T is column k of Ybar R^{-T}, so the
// columns that a tile of dX gains are contiguous.
__global__ void rinv_kernel(const double* __restrict__ T, int64_t ldt, const int64_t* __restrict__ piv, int d,
                            const int* __restrict__ rank, double* __restrict__ Rinv) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d) return;
    for (int i = j + 1; i < d; ++i) Rinv[(int64_t)rank[i] * d + j] = 0.0;
    Rinv[(int64_t)rank[j] * d + j] = 1.0 / T[(int64_t)j * ldt + piv[j]];
    for (int i = j - 1; i >= 0; --i) {
        double s = 0.0;
        for (int k = i + 1; k <= j; ++k) s = fma(T[(int64_t)i * ldt + piv[k]], Rinv[(int64_t)rank[k] * d + j], s);
        Rinv[(int64_t)rank[i] * d + j] = -s / T[(int64_t)i * ldt + piv[i]];
    }
}

// The same inverse for d <= kRinvLds: one wave per column j of R^{-1}, solving
// R x = e_j by column-oriented back substitution: for i = j down to 0,
// x_i = b_i / R(i, i), then b_k -= R(k, i) x_i for k < i.  Lane l keeps rows l
// and l + 64 of b (then x) in registers; a step is one lane broadcast and one
// multiply-add per row, with no cross-lane sum.  R's upper triangle is staged
// in LDS once per workgroup, packed by columns (column i holds rows 0..i at
// i (i + 1) / 2), with the reciprocals of its diagonal after it, copied from
// the packed form pivot_rank_kernel gathered once.
constexpr int kRinvLds = 128;
__global__ __launch_bounds__(256) void rinv_lds_kernel(const double* __restrict__ Rp, int d,
                                                       const int* __restrict__ rank, double* __restrict__ Rinv) {
    extern __shared__ double Rc[];           // packed R by columns: d (d + 1) / 2, then 1 / R(i, i): d
    double* rd = Rc + d * (d + 1) / 2;
    const int tot = d * (d + 1) / 2 + d;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) Rc[e] = Rp[e];     // contiguous, all in flight
    __syncthreads();
    const int lane = threadIdx.x % kWave;
    const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (j >= d) return;                      // whole waves leave together
    const int k0 = lane, k1 = lane + kWave;
    double x0 = (k0 == j) ? 1.0 : 0.0;
    double x1 = (k1 == j) ? 1.0 : 0.0;
    for (int i = j; i >= 0; --i) {
        const double* ci = Rc + i * (i + 1) / 2;               // ci[k] = R(k, i), k <= i
        const double src = i < kWave ? x0 : x1;                // i is uniform
        const int lo = __builtin_amdgcn_readlane(__double2loint(src), i % kWave);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(src), i % kWave);
        const double xi = __hiloint2double(hi, lo) * rd[i];
        const double r0 = ci[min(k0, i)], r1 = ci[min(k1, i)];
        x0 = k0 == i ? xi : (k0 < i ? fma(-r0, xi, x0) : x0);
        x1 = k1 == i ? xi : (k1 < i ? fma(-r1, xi, x1) : x1);
    }
    if (k0 < d) Rinv[(int64_t)rank[k0] * d + j] = x0;
    if (k1 < d) Rinv[(int64_t)rank[k1] * d + j] = x1;
}

// S = tril(M) + tril(M, -1)'
__global__ void copyltu_kernel(const double* __restrict__ Mm, int d, double* __restrict__ S) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)d * d) return;
    const int i = (int)(e / d), j = (int)(e % d);
    S[e] = Mm[(int64_t)max(i, j) * d + min(i, j)];
}

struct BwdPlan {
    size_t o_c1, o_ybar, o_m, o_s, o_rinv, o_abar, o_colrank, o_rank, o_rp, o_part, total;
};

bool make_bwd_plan(int64_t m, int64_t n, int32_t d, BwdPlan* P) {
    if (m < 1 || n < 1 || d < 1 || d > RBD_MAX_D || d > std::min(m, n)) return false;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = al(o + bytes);
        return at;
    };
    P->o_c1 = take(8 * (size_t)d * n);
    P->o_ybar = take(8 * (size_t)m * d);
    P->o_m = take(8 * (size_t)d * d);
    P->o_s = take(8 * (size_t)d * d);
    P->o_rinv = take(8 * (size_t)d * d);
    P->o_abar = take(8 * (size_t)m * d);
    P->o_colrank = take(4 * ((size_t)n + 1));
    P->o_rank = take(4 * (size_t)d);
    P->o_rp = take(8 * ((size_t)d * (d + 1) / 2 + d));
    P->o_part = take(8 * kPartElems);
    P->total = o;
    return true;
}

template <typename Tx, typename Tg>
int backward_typed(const BwdPlan& P, const Tx* X, int64_t ldx, const Tg* G, int64_t ldg, const double* Y, int64_t ldy,
                   const double* T, int64_t ldt, const int64_t* piv, int64_t m, int64_t n, int d, double* dX,
                   int64_t lddx, char* ws, hipStream_t s) {
    double* C1 = reinterpret_cast<double*>(ws + P.o_c1);
    double* Ybar = reinterpret_cast<double*>(ws + P.o_ybar);
    double* Mm = reinterpret_cast<double*>(ws + P.o_m);
    double* S = reinterpret_cast<double*>(ws + P.o_s);
    double* Rinv = reinterpret_cast<double*>(ws + P.o_rinv);
    double* Abar = reinterpret_cast<double*>(ws + P.o_abar);
    double* part = reinterpret_cast<double*>(ws + P.o_part);
    int* colrank = reinterpret_cast<int*>(ws + P.o_colrank);
    int* rank = reinterpret_cast<int*>(ws + P.o_rank);
    double* Rp = reinterpret_cast<double*>(ws + P.o_rp);
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    // C1 = Y'G (d x n)
    ok(gemm<true, false, double, Tg>(d, n, m, 1.0, Y, ldy, G, ldg, 0.0, C1, n, part, kPartElems, s));
    // Ybar = G T' + X C1'  (m x d)
    ok(gemm<false, true, Tg, double>(m, d, n, 1.0, G, ldg, T, ldt, 0.0, Ybar, d, part, kPartElems, s));
    ok(gemm<false, true, Tx, double>(m, d, n, 1.0, X, ldx, C1, n, 1.0, Ybar, d, part, kPartElems, s));
    // M = -Ybar' Y (d x d);  S = copyltu(M);  Ybar += Y S
    ok(gemm<true, false, double, double>(d, d, m, -1.0, Ybar, d, Y, ldy, 0.0, Mm, d, part, kPartElems, s));
    copyltu_kernel<<<(unsigned)cd((int64_t)d * d, 256), 256, 0, s>>>(Mm, d, S);
    ok(hipGetLastError());
    ok(gemm<false, false, double, double>(m, d, d, 1.0, Y, ldy, S, d, 1.0, Ybar, d, nullptr, 0, s));
    // Rinv' = R^{-1}, rows in pivot-rank order (R gathered once by pivot_rank_kernel when d <= kRinvLds)
    const bool lds_inv = d <= kRinvLds;
    // one thread per column rank, pivot rank and (with the LDS inverse) entry of the packed R
    const int64_t rank_threads =
        std::max<int64_t>(std::max<int64_t>(n + 1, d), lds_inv ? (int64_t)d * (d + 1) / 2 : 0);
    pivot_rank_kernel<<<(unsigned)cd(rank_threads, 256), 256, 0, s>>>(piv, d, n, colrank, rank, T, ldt,
                                                                       lds_inv ? Rp : nullptr);
    ok(hipGetLastError());
    if (lds_inv) {
        const size_t lds = sizeof(double) * ((size_t)d * (d + 1) / 2 + d);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rinv_lds_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        rinv_lds_kernel<<<(unsigned)cd(d, 4), 256, lds, s>>>(Rp, d, rank, Rinv);
    } else {
        rinv_kernel<<<(unsigned)cd(d, 64), 64, 0, s>>>(T, ldt, piv, d, rank, Rinv);
    }
    ok(hipGetLastError());
    // Abar' = Ybar R^{-T} with its columns in pivot-rank order
    ok(gemm<false, true, double, double>(m, d, d, 1.0, Ybar, d, Rinv, d, 0.0, Abar, d, nullptr, 0, s));
    // dX = Y C1 + scatter_P(Abar): each tile of dX adds the Abar' columns of the pivots among its
    // columns as extra k-steps of its own product (dX is written once)
    ok(gemm_f64<false, false, double, double>(m, n, d, 1.0, Y, ldy, C1, n, 0.0, dX, lddx, nullptr, 0, s,
                                              GemmColAdd{Abar, d, colrank}));
    return e == hipSuccess ? RBD_OK : RBD_EDEVICE;
}

template <typename Tx>
int backward_g(rbd_dtype gt, const BwdPlan& P, const Tx* X, int64_t ldx, const void* G, int64_t ldg, const double* Y,
               int64_t ldy, const double* T, int64_t ldt, const int64_t* piv, int64_t m, int64_t n, int d, double* dX,
               int64_t lddx, char* ws, hipStream_t s) {
    switch (gt) {
        case RBD_F64:
            return backward_typed<Tx, double>(P, X, ldx, static_cast<const double*>(G), ldg, Y, ldy, T, ldt, piv, m,
                                              n, d, dX, lddx, ws, s);
        case RBD_F32:
            return backward_typed<Tx, float>(P, X, ldx, static_cast<const float*>(G), ldg, Y, ldy, T, ldt, piv, m, n,
                                             d, dX, lddx, ws, s);
        default:
            return RBD_EINVAL;
    }
}

}  // namespace

extern "C" {

int rbd_reconstruct(const double* Y, int64_t ldy, int64_t m, int32_t d, const double* T, int64_t ldt, int64_t n,
                    double* Z, int64_t ldz, void* stream) {
    if (!Y || !T || !Z || m < 1 || n < 1 || d < 1 || ldy < d || ldt < n || ldz < n) return RBD_EINVAL;
    const hipError_t e = gemm<false, false, double, double>(m, n, d, 1.0, Y, ldy, T, ldt, 0.0, Z, ldz, nullptr, 0,
                                                            reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RBD_OK : RBD_EDEVICE;
}

int rbd_reconstruct_backward_workspace_size(int64_t m, int64_t n, int32_t d, size_t* bytes) {
    BwdPlan P;
    if (!bytes || !make_bwd_plan(m, n, d, &P)) return RBD_EINVAL;
    *bytes = P.total;
    return RBD_OK;
}

int rbd_reconstruct_backward(const void* X, rbd_dtype xt, int64_t ldx, const void* G, rbd_dtype gt, int64_t ldg,
                             const double* Y, int64_t ldy, const double* T, int64_t ldt, const int64_t* pivots,
                             int64_t m, int64_t n, int32_t d, double* dX, int64_t lddx, void* workspace,
                             size_t workspace_bytes, void* stream) {
    BwdPlan P;
    if (!make_bwd_plan(m, n, d, &P)) return RBD_EINVAL;
    if (!X || !G || !Y || !T || !pivots || !dX || !workspace) return RBD_EINVAL;
    if (ldx < n || ldg < n || ldy < d || ldt < n || lddx < n) return RBD_EINVAL;
    if (gt != RBD_F64 && gt != RBD_F32) return RBD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return RBD_EINVAL;
    if (workspace_bytes < P.total) return RBD_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    switch (xt) {
        case RBD_F32:
            return backward_g<float>(gt, P, static_cast<const float*>(X), ldx, G, ldg, Y, ldy, T, ldt, pivots, m, n,
                                     d, dX, lddx, ws, s);
        case RBD_F64:
            return backward_g<double>(gt, P, static_cast<const double*>(X), ldx, G, ldg, Y, ldy, T, ldt, pivots, m, n,
                                      d, dX, lddx, ws, s);
        case RBD_BF16:
            return backward_g<bf16_t>(gt, P, static_cast<const bf16_t*>(X), ldx, G, ldg, Y, ldy, T, ldt, pivots, m,
                                      n, d, dX, lddx, ws, s);
        case RBD_F16:
            return backward_g<f16_t>(gt, P, static_cast<const f16_t*>(X), ldx, G, ldg, Y, ldy, T, ldt, pivots, m, n,
                                     d, dX, lddx, ws, s);
    }
    return RBD_EINVAL;
}

}  // extern "C"
