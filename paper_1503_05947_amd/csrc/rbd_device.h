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

// ---------------------------------------------------------------------------
// loop state kept in device memory (one per rbd_fit call)
// ---------------------------------------------------------------------------
struct State {
    int d;          // basis vectors accepted so far
    int p;          // column to orthonormalise at the next step
    int stop;       // 0 while running, else an RBD_STOP_* value
    int status;     // RBD_OK or RBD_ENONFINITE
    int nflag;      // columns queued for an exact error evaluation this step
    int D;          // min(d_max, m, n)
    int nonfinite;  // set while the column norms are formed
    int pad0;
    double tau;     // eps_R after the relative/absolute reading
    double E0;      // max_j ||x_j||
    double nu;      // ||v|| after the second Gram-Schmidt pass
    double inv_nu;  // 1 / nu
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
};
template <> struct Ld<double> {
    static constexpr int N = 2;
    using raw = f64x2;
    static __device__ __forceinline__ void cvt(raw r, double* o) { o[0] = r.x; o[1] = r.y; }
    static __device__ __forceinline__ double one(const double* p) { return *p; }
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
};

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
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

// Two-level deterministic reduction of per-block rows.
//   part  : nblk rows of `len` doubles (row stride ldp); block `blk` wrote row blk
//   l2    : ceil(nblk / group) rows (stride ldp) of scratch
//   out   : len doubles, written by the single block for which this returns true
// Order: out[k] = sum_g ( sum_{b in group g, ascending} part[b][k] ), g ascending.
// Uses tickets[0 .. ngroups] (ngroups + 1 counters).
__device__ __forceinline__ bool grid_reduce_rows(const double* part, int64_t ldp, int nblk, int len,
                                                 double* l2, int group, unsigned* tickets, double* out,
                                                 int blk) {
    const int ngroups = (nblk + group - 1) / group;
    const int g = blk / group;
    const int gsz = min(group, nblk - g * group);
    if (!last_to_arrive(&tickets[g], (unsigned)gsz)) return false;
    for (int k = threadIdx.x; k < len; k += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < gsz; ++b) s += part[(int64_t)(g * group + b) * ldp + k];
        l2[(int64_t)g * ldp + k] = s;
    }
    if (!last_to_arrive(&tickets[ngroups], (unsigned)ngroups)) return false;
    for (int k = threadIdx.x; k < len; k += blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < ngroups; ++q) s += l2[(int64_t)q * ldp + k];
        out[k] = s;
    }
    __threadfence();
    __syncthreads();
    return true;
}

}  // namespace rbd
