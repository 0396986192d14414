// Device helpers shared by the QEM kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

namespace qemk {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;

template <typename T> __device__ __forceinline__ T neg_inf();
template <> __device__ __forceinline__ float neg_inf<float>() { return -__builtin_inff(); }
template <> __device__ __forceinline__ double neg_inf<double>() { return -__builtin_inf(); }

__device__ __forceinline__ float fexp(float x) { return __expf(x); }
__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ float flog(float x) { return __logf(x); }
__device__ __forceinline__ double flog(double x) { return log(x); }

// Butterfly reductions inside aligned groups of `width` lanes (power of two <= 64).
template <typename T>
__device__ __forceinline__ T group_max(T v, int width) {
    for (int off = width >> 1; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, width));
    return v;
}
template <typename T>
__device__ __forceinline__ T group_sum(T v, int width) {
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, width);
    return v;
}

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

}  // namespace qemk
