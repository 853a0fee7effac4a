// Device-side building blocks shared by the RBD kernels (gfx950, wave64).
//
// Nothing here depends on torch.  All floating-point reductions are done in a
// fixed order so that results are bitwise reproducible: partial results are
// written per workgroup, and the last workgroup to arrive (detected with an
// integer ticket counter) combines them in index order.  There are no
// floating-point atomics.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rbd.h"

namespace rbd {

constexpr int kWave = 64;
constexpr int kStopError = 4;           // internal stop code: non-finite input
constexpr double kRefresh = 0x1p-20;    // kappa: re-evaluate a column exactly when e^2 < kappa * (last exact e^2)
constexpr double kRefreshEager = 0x1p-15;   // once any column needs it, also refresh those below this fraction

// ---------------------------------------------------------------------------
// loop state kept in device memory (one per rbd_fit call)
// ---------------------------------------------------------------------------
struct State {
    int d;          // basis vectors accepted so far
    int p;          // column to orthonormalise at the next step
    int stop;       // 0 while running, else an RBD_STOP_* value
    int status;     // RBD_OK, RBD_ENONFINITE or RBD_EMATRIX
    int nflag;      // columns queued for an exact error evaluation this step
    int D;          // min(d_max, m, n)
    int nonfinite;  // set while the column norms are formed
    int bad_index;  // set when a sparse A holds an index out of range
    double tau;     // eps_R after the relative/absolute reading
    double E0;      // max_j ||x_j||
    double nu;      // ||v|| after the second Gram-Schmidt pass
    double inv_nu;  // 1 / nu
    double wxx;     // ||xi||_A^2 = sum_i w_i xi_i^2 (diagonal A only)
    double pad1;
};

// ---------------------------------------------------------------------------
// storage types and 16-byte vector loads
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t u; };
struct f16_t { uint16_t u; };

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double bf16_lo(unsigned w) { return (double)__uint_as_float(w << 16); }
__device__ __forceinline__ double bf16_hi(unsigned w) { return (double)__uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ double f16_lo(unsigned w) {
    return (double)(float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
}
__device__ __forceinline__ double f16_hi(unsigned w) {
    return (double)(float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
}

template <typename Tx> struct Ld;

template <> struct Ld<float> {
    static constexpr int N = 4;
    using raw = f32x4;
    static __device__ __forceinline__ void cvt(raw r, double* o) {
        o[0] = r.x; o[1] = r.y; o[2] = r.z; o[3] = r.w;
    }
    static __device__ __forceinline__ double one(const float* p) { return (double)*p; }
    static __device__ __forceinline__ double from(float v) { return (double)v; }
};
template <> struct Ld<double> {
    static constexpr int N = 2;
    using raw = f64x2;
    static __device__ __forceinline__ void cvt(raw r, double* o) { o[0] = r.x; o[1] = r.y; }
    static __device__ __forceinline__ double one(const double* p) { return *p; }
    static __device__ __forceinline__ double from(double v) { return v; }
};
template <> struct Ld<bf16_t> {
    static constexpr int N = 8;
    using raw = u32x4;
    static __device__ __forceinline__ void cvt(raw r, double* o) {
        o[0] = bf16_lo(r.x); o[1] = bf16_hi(r.x); o[2] = bf16_lo(r.y); o[3] = bf16_hi(r.y);
        o[4] = bf16_lo(r.z); o[5] = bf16_hi(r.z); o[6] = bf16_lo(r.w); o[7] = bf16_hi(r.w);
    }
    static __device__ __forceinline__ double one(const bf16_t* p) {
        return (double)__uint_as_float((unsigned)p->u << 16);
    }
    static __device__ __forceinline__ double from(bf16_t v) { return (double)__uint_as_float((unsigned)v.u << 16); }
};
template <> struct Ld<f16_t> {
    static constexpr int N = 8;
    using raw = u32x4;
    static __device__ __forceinline__ void cvt(raw r, double* o) {
        o[0] = f16_lo(r.x); o[1] = f16_hi(r.x); o[2] = f16_lo(r.y); o[3] = f16_hi(r.y);
        o[4] = f16_lo(r.z); o[5] = f16_hi(r.z); o[6] = f16_lo(r.w); o[7] = f16_hi(r.w);
    }
    static __device__ __forceinline__ double one(const f16_t* p) {
        return (double)(float)__builtin_bit_cast(_Float16, p->u);
    }
    static __device__ __forceinline__ double from(f16_t v) { return (double)(float)__builtin_bit_cast(_Float16, v.u); }
};

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
// One step of a DPP reduction: v += v[lane given by CTRL] on the rows in ROW_MASK
// (other rows add 0).  Doubles move as two 32-bit halves.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return v + __hiloint2double(hi, lo);
}

// Sums of R independent values over the 64 lanes of a wave, interleaved step
// by step; the result is uniform (read from lane 63).  Fixed order: quads,
// half rows, rows of 16, then rows 0+1 and 2+3, then the two halves.
// Every lane of the wave must be active.
template <int R>
__device__ __forceinline__ void wave_sum_n(double (&v)[R]) {
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = dpp_add<0xB1, 0xf>(v[u]);   // quad_perm [1,0,3,2]
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = dpp_add<0x4E, 0xf>(v[u]);   // quad_perm [2,3,0,1]
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = dpp_add<0x141, 0xf>(v[u]);  // row_half_mirror
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = dpp_add<0x140, 0xf>(v[u]);  // row_mirror
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = dpp_add<0x142, 0xa>(v[u]);  // row_bcast:15
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = dpp_add<0x143, 0xc>(v[u]);  // row_bcast:31
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(v[u]), 63);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v[u]), 63);
        v[u] = __hiloint2double(hi, lo);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    double a[1] = {v};
    wave_sum_n<1>(a);
    return a[0];
}

// (value, index) maximum; ties go to the lower index.  NaN never wins.
__device__ __forceinline__ void argmax_merge(double& v, int64_t& i, double v2, int64_t i2) {
    if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

__device__ __forceinline__ void wave_argmax(double& v, int64_t& i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double v2 = __shfl_xor(v, off, kWave);
        int64_t i2 = __shfl_xor(i, off, kWave);
        argmax_merge(v, i, v2, i2);
    }
}

// Block-wide argmax over all threads; result valid in every thread.
// `sv`/`si` must hold blockDim.x / kWave entries.
__device__ __forceinline__ void block_argmax(double& v, int64_t& i, double* sv, int64_t* si) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    wave_argmax(v, i);
    __syncthreads();
    if (lane == 0) { sv[w] = v; si[w] = i; }
    __syncthreads();
    v = sv[0]; i = si[0];
    for (int k = 1; k < nw; ++k) argmax_merge(v, i, sv[k], si[k]);
    __syncthreads();
}

// Block-wide sum in a fixed order (waves combined in index order).
__device__ __forceinline__ double block_sum(double v, double* sv) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sv[w] = v;
    __syncthreads();
    double s = sv[0];
    for (int k = 1; k < nw; ++k) s += sv[k];
    __syncthreads();
    return s;
}

// Take a ticket on `counter`; returns true in every thread of the block that
// arrives last out of `expected`.  That block resets the counter to 0 so the
// next launch can reuse it, and issues an acquire fence before returning.
__device__ __forceinline__ bool last_to_arrive(unsigned* counter, unsigned expected) {
    __shared__ unsigned s_ticket;
    __threadfence();  // release this block's partial results
    __syncthreads();
    if (threadIdx.x == 0) s_ticket = atomicAdd(counter, 1u);
    __syncthreads();
    const bool last = (s_ticket == expected - 1);
    if (last) {
        if (threadIdx.x == 0) atomicExch(counter, 0u);
        __threadfence();  // acquire the other blocks' results
    }
    __syncthreads();
    return last;
}

}  // namespace rbd
