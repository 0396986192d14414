// The linear-Gaussian pairwise log-factor of a (parent sample, child sample)
// pair, shared by the pair-table kernels and the plate forward kernel that
// evaluates the table on the fly, so that every path produces the same bits:
//   mean_j = a * zp_j + b
//   F      = c0 - hp * sum_j (zc_j - mean_j)^2,   c0 = -d/2 log(2 pi var), hp = 1/(2 var)
// with every multiply-add an explicit fused multiply-add.
#pragma once
#include <hip/hip_runtime.h>

namespace qemk {

template <typename T>
__device__ __forceinline__ T pair_mean(T a, T zp, T b) { return fma(a, zp, b); }

// D > 0: compile-time dimension; D = 0: d read at run time.
template <typename T, int D>
__device__ __forceinline__ T normal_pair_value(const T* zc, const T* mean, int d, T c0, T hp) {
    const int n = D > 0 ? D : d;
    T s = 0;
#pragma unroll
    for (int j = 0; j < n; ++j) {
        const T e = zc[j] - mean[j];
        s = fma(e, e, s);
    }
    return fma(-hp, s, c0);
}

}  // namespace qemk
