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

// One element of Y in a pass over its rows.  NT: a non-temporal load, for
// passes whose Y is larger than the caches (Y is read once per greedy step,
// so nothing it would keep in the caches is used again).
template <bool NT, typename T>
__device__ __forceinline__ T ld_y(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

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
typedef float f32x2 __attribute__((ext_vector_type(2)));
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

// A DPP move of a double (two 32-bit halves); every lane of the row receives.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Butterfly steps across rows with the gfx950 lane swaps.  bfly32: lanes 0-31
// get a(l) + a(l + 32), lanes 32-63 get b(l - 32) + b(l).  bfly16: rows 0 and
// 2 get a summed over the row pairs (0, 1) and (2, 3), rows 1 and 3 get b.
__device__ __forceinline__ double bfly32(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double bfly16(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
// Within rows: lanes whose bit B is 0 keep a, the others b, and each adds its
// partner's copy (CTRL pairs every lane with one whose bit B differs).
template <int CTRL, int B>
__device__ __forceinline__ double bfly_row(double a, double b, int lane) {
    const bool up = (lane >> B) & 1;
    const double keep = up ? b : a, send = up ? a : b;
    return keep + dpp_mov<CTRL>(send);
}

// Sums of R independent values (R = 1, 2, 4, 8 or 16) over the 64 lanes of a
// wave, results uniform.  A transposing butterfly: each of the first log2(R)
// levels halves the values a lane carries (lanes 32 apart, then 16, 8, 4), so
// the step count does not grow with R; value u ends up in lanes
// [u * 64 / R, (u + 1) * 64 / R).  The pairing order (bit 5, 4, 3, then the
// half-row mirror, then bits 1 and 0) is the same for every value and every R,
// so a value's sum does not depend on how many are reduced with it.
// Every lane of the wave must be active.
template <int R>
__device__ __forceinline__ void wave_sum_n(double (&v)[R]) {
    static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 16, "R must be a power of two up to 16");
    const int lane = __lane_id();
    if constexpr (R >= 2) {
#pragma unroll
        for (int j = 0; j < R / 2; ++j) v[j] = bfly32(v[j], v[j + R / 2]);
    } else {
        v[0] = bfly32(v[0], v[0]);
    }
    if constexpr (R >= 4) {
#pragma unroll
        for (int j = 0; j < R / 4; ++j) v[j] = bfly16(v[j], v[j + R / 4]);
    } else {
        v[0] = bfly16(v[0], v[0]);
    }
    if constexpr (R >= 8) {
#pragma unroll
        for (int j = 0; j < R / 8; ++j) v[j] = bfly_row<0x128, 3>(v[j], v[j + R / 8], lane);   // row_ror:8
    } else {
        v[0] = dpp_add<0x128, 0xf>(v[0]);
    }
    if constexpr (R >= 16) v[0] = bfly_row<0x141, 2>(v[0], v[1], lane);                       // row_half_mirror
    else v[0] = dpp_add<0x141, 0xf>(v[0]);
    v[0] = dpp_add<0x4E, 0xf>(v[0]);   // quad_perm [2,3,0,1]
    v[0] = dpp_add<0xB1, 0xf>(v[0]);   // quad_perm [1,0,3,2]
    const double s = v[0];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(s), u * (64 / R));
        const int hi = __builtin_amdgcn_readlane(__double2hiint(s), u * (64 / R));
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
