// Recognition of out-of-sample data in the compressed coordinates.
//
// Each query v is compressed as c = Y'v (section 3.1, the
// compression of out-of-sample data), and matched to the training sample
// whose coordinates T(:, j) are nearest in the Euclidean norm of R^d -- the
// use of the compressed representation for face recognition in section 4.
// The only work that depends on the entry length m is the product Y'V (an
// FP64 GEMM on the matrix cores); the search is m-independent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/rbd.h"
#include "rbd_proj.h"

namespace {

using namespace rbd;

int64_t cdv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// nn: for query q (column q of C, d x k, leading dimension ldc), the training
// column j of T (d x n, leading dimension ldt) minimising
// sum_i (C[i, q] - T[i, j])^2, accumulated term by term in ascending i; the
// lowest index wins ties.  One query per thread; every lane of a wave reads
// the same T entries, so those loads are uniform (scalar) loads.
constexpr int kNnJ = 16;

__global__ __launch_bounds__(256) void nn_kernel(const double* __restrict__ C, int64_t ldc, int64_t k,
                                                  const double* __restrict__ T, int64_t ldt, int64_t n, int d,
                                                  const int32_t* __restrict__ labels, int64_t* __restrict__ nn_index,
                                                  int32_t* __restrict__ nn_label, double* __restrict__ nn_dist2) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t qc = q < k ? q : k - 1;        // lanes past the end repeat the last query, unwritten
    double best = INFINITY;
    int64_t bi = -1;
    for (int64_t j0 = 0; j0 < n; j0 += kNnJ) {
        double acc[kNnJ];
#pragma unroll
        for (int jj = 0; jj < kNnJ; ++jj) acc[jj] = 0.0;
        if (j0 + kNnJ <= n) {
            for (int i = 0; i < d; ++i) {
                const double c = C[(int64_t)i * ldc + qc];
                const double* t = T + (int64_t)i * ldt + j0;
#pragma unroll
                for (int jj = 0; jj < kNnJ; ++jj) {
                    const double e = c - t[jj];
                    acc[jj] = fma(e, e, acc[jj]);
                }
            }
        } else {
            const int jn = (int)(n - j0);
            for (int i = 0; i < d; ++i) {
                const double c = C[(int64_t)i * ldc + qc];
                const double* t = T + (int64_t)i * ldt + j0;
#pragma unroll
                for (int jj = 0; jj < kNnJ; ++jj) {
                    const double e = jj < jn ? c - t[jj] : 0.0;
                    acc[jj] = fma(e, e, acc[jj]);
                }
            }
#pragma unroll
            for (int jj = 0; jj < kNnJ; ++jj)
                if (jj >= jn) acc[jj] = INFINITY;
        }
#pragma unroll
        for (int jj = 0; jj < kNnJ; ++jj)
            if (acc[jj] < best) {
                best = acc[jj];
                bi = j0 + jj;
            }
    }
    if (q < k) {
        nn_index[q] = bi;
        nn_label[q] = bi < 0 ? -1 : (labels ? labels[bi] : (int32_t)bi);
        nn_dist2[q] = bi < 0 ? NAN : best;
    }
}

template <typename Tv>
int classify_typed(const double* Y, int64_t ldy, int64_t m, int d, const double* T, int64_t ldt, int64_t n,
                   const int32_t* labels, const Tv* V, int64_t k, int64_t ldv, double* C, int64_t* nn_index,
                   int32_t* nn_label, double* nn_dist2, double* part, size_t part_elems, hipStream_t s) {
    // C = Y' V: Y is stored m x d (row-major, ldy), V is m x k (ldv)
    if (proj_mfma<Tv>(Y, ldy, m, d, V, ldv, k, C, k, part, part_elems, s) != hipSuccess) return RBD_EDEVICE;
    nn_kernel<<<(unsigned)cdv(k, 256), 256, 0, s>>>(C, k, k, T, ldt, n, d, labels, nn_index, nn_label, nn_dist2);
    return hipGetLastError() == hipSuccess ? RBD_OK : RBD_EDEVICE;
}

bool classify_args_ok(int64_t m, int32_t d, int64_t k) {
    return m >= 1 && d >= 1 && d <= RBD_MAX_D && k >= 1 && k < (int64_t)INT32_MAX;
}

}  // namespace

extern "C" {

int rbd_classify_workspace_size(int64_t m, int32_t d, int64_t k, size_t* bytes) {
    if (!bytes || !classify_args_ok(m, d, k)) return RBD_EINVAL;
    *bytes = 8 * kPartElems;
    return RBD_OK;
}

int rbd_classify(const double* Y, int64_t ldy, int64_t m, int32_t d, const double* T, int64_t ldt, int64_t n,
                 const int32_t* labels, const void* V, rbd_dtype vt, int64_t k, int64_t ldv, double* C,
                 int64_t* nn_index, int32_t* nn_label, double* nn_dist2, void* workspace, size_t workspace_bytes,
                 void* stream) {
    if (!classify_args_ok(m, d, k) || n < 1) return RBD_EINVAL;
    if (!Y || !T || !V || !C || !nn_index || !nn_label || !nn_dist2 || !workspace) return RBD_EINVAL;
    if (ldy < d || ldt < n || ldv < k) return RBD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return RBD_EINVAL;
    if (workspace_bytes < 8 * kPartElems) return RBD_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double* part = static_cast<double*>(workspace);
    switch (vt) {
        case RBD_F32:
            return classify_typed<float>(Y, ldy, m, d, T, ldt, n, labels, static_cast<const float*>(V), k, ldv, C,
                                         nn_index, nn_label, nn_dist2, part, kPartElems, s);
        case RBD_F64:
            return classify_typed<double>(Y, ldy, m, d, T, ldt, n, labels, static_cast<const double*>(V), k, ldv, C,
                                          nn_index, nn_label, nn_dist2, part, kPartElems, s);
        case RBD_BF16:
            return classify_typed<bf16_t>(Y, ldy, m, d, T, ldt, n, labels, static_cast<const bf16_t*>(V), k, ldv,
                                          C, nn_index, nn_label, nn_dist2, part, kPartElems, s);
        case RBD_F16:
            return classify_typed<f16_t>(Y, ldy, m, d, T, ldt, n, labels, static_cast<const f16_t*>(V), k, ldv, C,
                                         nn_index, nn_label, nn_dist2, part, kPartElems, s);
    }
    return RBD_EINVAL;
}

}  // extern "C"
