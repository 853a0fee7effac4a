// Reconstruction Z = Y T (section 3.1, "Uncompress") and its backward with
// the pivots held fixed.
//
// With the pivots P fixed, the basis is the Q factor of A = X(:, P) = Y R
// (Gram-Schmidt of the pivot columns in order; R = T(:, P) is upper
// triangular with positive diagonal), and T = Y'X.  For L = <G, Y Y' X>:
//   dL/dX        = Y (Y'G)                       (through T)
//              + scatter_P( (Ybar + Y copyltu(M)) R^{-T} )   (through Y)
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

// Rinv = R^{-1} (upper triangular, d x d row-major), R(i, k) = T(i, piv[k]) for i <= k.
__global__ void rinv_kernel(const double* __restrict__ T, int64_t ldt, const int64_t* __restrict__ piv, int d,
                            double* __restrict__ Rinv) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d) return;
    for (int i = j + 1; i < d; ++i) Rinv[(int64_t)i * d + j] = 0.0;
    Rinv[(int64_t)j * d + j] = 1.0 / T[(int64_t)j * ldt + piv[j]];
    for (int i = j - 1; i >= 0; --i) {
        double s = 0.0;
        for (int k = i + 1; k <= j; ++k) s = fma(T[(int64_t)i * ldt + piv[k]], Rinv[(int64_t)k * d + j], s);
        Rinv[(int64_t)i * d + j] = -s / T[(int64_t)i * ldt + piv[i]];
    }
}

// The same inverse for d <= kRinvLds: one wave per column j of Rinv, solving
// R x = e_j by back substitution.  Lane l keeps x(l) and x(l + 64) in
// registers; each step i is one wave sum of R(i, k) x(k) over k in (i, j],
// times 1 / R(i, i).  R's upper triangle is staged in LDS once per workgroup,
// packed by rows (row i holds columns i..d-1 at tri_off(i)), with the
// reciprocals of its diagonal after it.
constexpr int kRinvLds = 128;
__device__ __forceinline__ int tri_off(int i, int d) { return i * d - i * (i - 1) / 2; }
__global__ __launch_bounds__(256) void rinv_lds_kernel(const double* __restrict__ T, int64_t ldt,
                                                       const int64_t* __restrict__ piv, int d,
                                                       double* __restrict__ Rinv) {
    extern __shared__ double Rp[];           // packed R: d (d + 1) / 2, then 1 / R(i, i): d
    double* rd = Rp + d * (d + 1) / 2;
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) {      // independent loads, all in flight
        const int i = e / d, k = e % d;
        if (k >= i) {
            const double v = T[(int64_t)i * ldt + piv[k]];
            Rp[tri_off(i, d) + k - i] = v;
            if (k == i) rd[i] = 1.0 / v;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x % kWave;
    const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (j >= d) return;                      // whole waves leave together
    const int k0 = lane, k1 = lane + kWave;
    double x0 = (k0 == j) ? rd[j] : 0.0;
    double x1 = (k1 == j) ? rd[j] : 0.0;
    for (int i = j - 1; i >= 0; --i) {
        const double* ri = Rp + tri_off(i, d) - i;             // ri[k] = R(i, k), k >= i
        double sum = 0.0;
        if (k0 > i && k0 <= j) sum = ri[k0] * x0;
        if (k1 > i && k1 <= j) sum = fma(ri[k1], x1, sum);
        sum = wave_sum(sum);
        const double v = -sum * rd[i];
        if (k0 == i) x0 = v;
        if (k1 == i) x1 = v;
    }
    if (k0 < d) Rinv[(int64_t)k0 * d + j] = x0;
    if (k1 < d) Rinv[(int64_t)k1 * d + j] = x1;
}

// dX(:, piv[k]) += Abar(:, k)   (pivots are distinct; one outside [0, n) is skipped)
__global__ void scatter_add_cols_kernel(const double* __restrict__ Abar, int64_t m, int d,
                                        const int64_t* __restrict__ piv, int64_t n, double* __restrict__ dX,
                                        int64_t lddx) {
    const int64_t tot = m * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / d;
        const int k = (int)(e % d);
        const int64_t c = piv[k];
        if (c >= 0 && c < n) dX[i * lddx + c] += Abar[e];
    }
}

// S = tril(M) + tril(M, -1)'
__global__ void copyltu_kernel(const double* __restrict__ Mm, int d, double* __restrict__ S) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)d * d) return;
    const int i = (int)(e / d), j = (int)(e % d);
    S[e] = Mm[(int64_t)max(i, j) * d + min(i, j)];
}

struct BwdPlan {
    size_t o_c1, o_ybar, o_m, o_s, o_rinv, o_abar, o_part, total;
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
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    // C1 = Y'G (d x n);  dX = Y C1
    ok(gemm<true, false, double, Tg>(d, n, m, 1.0, Y, ldy, G, ldg, 0.0, C1, n, part, kPartElems, s));
    ok(gemm<false, false, double, double>(m, n, d, 1.0, Y, ldy, C1, n, 0.0, dX, lddx, nullptr, 0, s));
    // Ybar = G T' + X C1'  (m x d)
    ok(gemm<false, true, Tg, double>(m, d, n, 1.0, G, ldg, T, ldt, 0.0, Ybar, d, part, kPartElems, s));
    ok(gemm<false, true, Tx, double>(m, d, n, 1.0, X, ldx, C1, n, 1.0, Ybar, d, part, kPartElems, s));
    // M = -Ybar' Y (d x d);  S = copyltu(M);  Ybar += Y S
    ok(gemm<true, false, double, double>(d, d, m, -1.0, Ybar, d, Y, ldy, 0.0, Mm, d, part, kPartElems, s));
    copyltu_kernel<<<(unsigned)cd((int64_t)d * d, 256), 256, 0, s>>>(Mm, d, S);
    ok(hipGetLastError());
    ok(gemm<false, false, double, double>(m, d, d, 1.0, Y, ldy, S, d, 1.0, Ybar, d, nullptr, 0, s));
    // Abar = Ybar R^{-T};  dX(:, P) += Abar
    if (d <= kRinvLds) {
        const size_t lds = sizeof(double) * ((size_t)d * (d + 1) / 2 + d);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rinv_lds_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        rinv_lds_kernel<<<(unsigned)cd(d, 4), 256, lds, s>>>(T, ldt, piv, d, Rinv);
    } else {
        rinv_kernel<<<(unsigned)cd(d, 64), 64, 0, s>>>(T, ldt, piv, d, Rinv);
    }
    ok(hipGetLastError());
    ok(gemm<false, true, double, double>(m, d, d, 1.0, Ybar, d, Rinv, d, 0.0, Abar, d, nullptr, 0, s));
    scatter_add_cols_kernel<<<(unsigned)std::min<int64_t>(4096, cd(m * d, 256)), 256, 0, s>>>(Abar, m, d, piv, n, dX,
                                                                                              lddx);
    ok(hipGetLastError());
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
