// Device helpers shared by the QEM kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "qem_internal.h"

namespace qemk {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;

template <typename T> __device__ __forceinline__ T neg_inf();
template <> __device__ __forceinline__ float neg_inf<float>() { return -__builtin_inff(); }
template <> __device__ __forceinline__ double neg_inf<double>() { return -__builtin_inf(); }
template <typename T> __device__ __forceinline__ T pos_inf() { return -neg_inf<T>(); }

__device__ __forceinline__ float fexp(float x) { return __expf(x); }
__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ float flog(float x) { return __logf(x); }
__device__ __forceinline__ double flog(double x) { return log(x); }

// Reductions inside aligned groups of `width` lanes (power of two <= 64); every
// lane of the group ends with the result.  FP32 groups of up to 16 lanes use
// DPP lane moves (quad permutations, then the 8- and 16-lane mirrors), which
// pair every lane with one from the other half at each stage; wider groups
// and FP64 use cross-lane shuffles.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int DPP_QUAD_1032 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_2301 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;

__device__ __forceinline__ float group_max(float v, int width) {
    if (width >= 2) v = fmaxf(v, dpp_mov<DPP_QUAD_1032>(v));
    if (width >= 4) v = fmaxf(v, dpp_mov<DPP_QUAD_2301>(v));
    if (width >= 8) v = fmaxf(v, dpp_mov<DPP_ROW_HALF_MIRROR>(v));
    if (width >= 16) v = fmaxf(v, dpp_mov<DPP_ROW_MIRROR>(v));
    if (width >= 32) v = fmaxf(v, __shfl_xor(v, 16, WAVE));
    if (width >= 64) v = fmaxf(v, __shfl_xor(v, 32, WAVE));
    return v;
}
__device__ __forceinline__ float group_sum(float v, int width) {
    if (width >= 2) v += dpp_mov<DPP_QUAD_1032>(v);
    if (width >= 4) v += dpp_mov<DPP_QUAD_2301>(v);
    if (width >= 8) v += dpp_mov<DPP_ROW_HALF_MIRROR>(v);
    if (width >= 16) v += dpp_mov<DPP_ROW_MIRROR>(v);
    if (width >= 32) v += __shfl_xor(v, 16, WAVE);
    if (width >= 64) v += __shfl_xor(v, 32, WAVE);
    return v;
}
__device__ __forceinline__ double group_max(double v, int width) {
    for (int off = width >> 1; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, width));
    return v;
}
__device__ __forceinline__ double group_sum(double v, int width) {
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, width);
    return v;
}

// Max of row[0..K) over the whole workgroup; every thread must call it.
// scratch: LDS of at least blockDim.x / WAVE doubles.
__device__ __forceinline__ double block_max(const double* row, int K, double* scratch) {
    double mx = -__builtin_inf();
    for (int k = threadIdx.x; k < K; k += blockDim.x) mx = fmax(mx, row[k]);
    mx = group_max(mx, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) scratch[threadIdx.x / WAVE] = mx;
    __syncthreads();
    double r = scratch[0];
    for (int w = 1; w < static_cast<int>(blockDim.x / WAVE); ++w) r = fmax(r, scratch[w]);
    __syncthreads();
    return r;
}

// Sets FLAG_NEG_INF_ROW (qem_internal.h) in the status word; called by the
// lanes that write a row whose log-sum-exp is -inf (divergent, so a vector
// atomic).
__device__ __forceinline__ void flag_neg_inf_row(uint32_t* status) {
    if (status) atomicOr(status, FLAG_NEG_INF_ROW);
}

// The shift applied to a row of log-weights before reduced-precision
// arithmetic: its maximum, or 0 when every entry is -inf.
__device__ __forceinline__ double finite_or_zero(double mx) { return mx == -__builtin_inf() ? 0.0 : mx; }

// 16-byte vector access for rows whose length is a multiple of the vector width.
template <typename T, int VEC> struct Vec { T v[VEC]; };

template <typename T, int VEC>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, T (&out)[VEC]) {
    if constexpr (VEC == 4 && sizeof(T) == 4) {
        float4 q = *reinterpret_cast<const float4*>(p);
        out[0] = q.x; out[1] = q.y; out[2] = q.z; out[3] = q.w;
    } else if constexpr (VEC == 2 && sizeof(T) == 8) {
        double2 q = *reinterpret_cast<const double2*>(p);
        out[0] = q.x; out[1] = q.y;
    } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) out[i] = p[i];
    }
}

// Streaming (nontemporal) variants for tensors that are read or written once
// per pass: they do not displace reusable data from the caches.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));

template <typename T, int VEC>
__device__ __forceinline__ void load_vec_nt(const T* __restrict__ p, T (&out)[VEC]) {
    if constexpr (VEC == 4 && sizeof(T) == 4) {
        const f32x4_t q = __builtin_nontemporal_load(reinterpret_cast<const f32x4_t*>(p));
        out[0] = q[0]; out[1] = q[1]; out[2] = q[2]; out[3] = q[3];
    } else if constexpr (VEC == 2 && sizeof(T) == 8) {
        const f64x2_t q = __builtin_nontemporal_load(reinterpret_cast<const f64x2_t*>(p));
        out[0] = q[0]; out[1] = q[1];
    } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) out[i] = __builtin_nontemporal_load(p + i);
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec_nt(T* __restrict__ p, const T (&in)[VEC]) {
    if constexpr (VEC == 4 && sizeof(T) == 4) {
        const f32x4_t q = {in[0], in[1], in[2], in[3]};
        __builtin_nontemporal_store(q, reinterpret_cast<f32x4_t*>(p));
    } else if constexpr (VEC == 2 && sizeof(T) == 8) {
        const f64x2_t q = {in[0], in[1]};
        __builtin_nontemporal_store(q, reinterpret_cast<f64x2_t*>(p));
    } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) __builtin_nontemporal_store(in[i], p + i);
    }
}

// Tensors larger than the Infinity Cache are streamed with nontemporal
// hints; smaller ones keep normal caching so a tensor written by one kernel
// can be read back from the cache by the next.
constexpr size_t STREAM_BYTES = size_t(256) << 20;

template <typename T, int VEC>
__device__ __forceinline__ void load_vec_hint(const T* __restrict__ p, T (&out)[VEC], bool nt) {
    if (nt) load_vec_nt<T, VEC>(p, out);
    else load_vec<T, VEC>(p, out);
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec_hint(T* __restrict__ p, const T (&in)[VEC], bool nt);

template <typename T, int VEC>
__device__ __forceinline__ void store_vec(T* __restrict__ p, const T (&in)[VEC]) {
    if constexpr (VEC == 4 && sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(in[0], in[1], in[2], in[3]);
    } else if constexpr (VEC == 2 && sizeof(T) == 8) {
        *reinterpret_cast<double2*>(p) = make_double2(in[0], in[1]);
    } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) p[i] = in[i];
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec_hint(T* __restrict__ p, const T (&in)[VEC], bool nt) {
    if (nt) store_vec_nt<T, VEC>(p, in);
    else store_vec<T, VEC>(p, in);
}

}  // namespace qemk
