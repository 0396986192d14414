// Moments (Eq. mmp with m = (z, z^2), or (z, log z) for the exponential-family
// Gamma), EMA of mean parameters (Eq. ema) and the closed-form M-step of
// Algorithm 1, all in FP64.
//   Gaussian: mean = m1, var = max(m2 - m1^2, floor)
//   Gamma (moment matching): v = max(m2 - m1^2, floor), shape = m1^2/v, rate = m1/v
//   Gamma (exponential family): shape from log a - psi(a) = max(log m1 - m2, floor), rate = shape/m1
// The EMA is skipped when the status word says this iteration's log P_MP was
// not finite; variance-floor hits are counted.
#include <algorithm>

#include "qem_internal.h"
#include "dev_common.h"
#include "dev_finish.h"

namespace qemk {

namespace {

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_moments(const T* __restrict__ z, const T* __restrict__ w,
                                                   double* __restrict__ mone, long n, int K, int d, bool logz) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * d) return;
    const long i = t / d;
    double s1, s2;
    moment_sums(z + i * K * d, w + i * K, static_cast<int>(t % d), K, d, s1, s2, logz);
    mone[t * 2 + 0] = s1;
    mone[t * 2 + 1] = s2;
}

// Dirichlet nodes: the first thread of each instance (t a multiple of d)
// updates its d components together.
__global__ void __launch_bounds__(BLOCK) k_mstep(double* __restrict__ mema, const double* __restrict__ mone,
                                                 double* __restrict__ qp, long count, int qfamily, double lam,
                                                 uint32_t* __restrict__ status, int d) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const bool skip = (status[0] & 0x1u) != 0u;
    if (qfamily == QF_DIRICHLET) {
        if (t % d == 0) mstep_dirichlet(mema + t * 2, mone + t * 2, qp + t * 2, d, 1.0, lam, skip, status);
        return;
    }
    mstep_entry(mema, mone, qp, t, qfamily, lam, skip, status);
}

__global__ void __launch_bounds__(BLOCK) k_mstep_multi(MstepTable tb, double lam, uint32_t* __restrict__ status,
                                                       uint64_t* __restrict__ iter_dev) {
    long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (iter_dev && t == 0) *iter_dev = *iter_dev + 1;
    const double l = tb.lam_dev ? *tb.lam_dev : lam;
    const double rho = tb.lp_z ? exp(*tb.lp_z - *tb.lp_new) : 1.0;
    const bool skip = (status[0] & 0x1u) != 0u;
    for (int v = 0; v < tb.n; ++v) {
        if (t < tb.count[v]) {
            const double* o = tb.mone[v];
            if (tb.qfamily[v] == QF_DIRICHLET) {
                const int d = tb.dim[v];
                if (t % d == 0) mstep_dirichlet(tb.mema[v] + t * 2, o + t * 2, tb.qp[v] + t * 2, d, rho, l, skip, status);
                return;
            }
            mstep_update(tb.mema[v], tb.qp[v], t, tb.mema[v][t * 2], tb.mema[v][t * 2 + 1], rho * o[t * 2],
                         rho * o[t * 2 + 1], tb.qfamily[v], l, skip, status);
            return;
        }
        t -= tb.count[v];
    }
}

__global__ void k_copy_scalar(const double* __restrict__ src, double* __restrict__ dst) {
    if (threadIdx.x == 0) *dst = *src;
}

__global__ void __launch_bounds__(BLOCK) k_init_q(double* __restrict__ qp, double* __restrict__ mema, long count,
                                                  int qfamily, int set_q, double q0a, double q0b, int d) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= count) return;
    if (qfamily == QF_DIRICHLET) {
        // (E z_c, E log z_c) = (alpha_c / alpha_0, psi(alpha_c) - psi(alpha_0)); with set_q every
        // component takes q0a (other threads write the instance's entries meanwhile)
        double a0 = 0.0;
        if (set_q) {
            qp[t * 2] = q0a;
            qp[t * 2 + 1] = 1.0;
            a0 = d * q0a;
        } else {
            const long i0 = (t / d) * d;
            for (int j = 0; j < d; ++j) a0 += qp[(i0 + j) * 2];
        }
        const double a = set_q ? q0a : qp[t * 2];
        mema[t * 2] = a / a0;
        mema[t * 2 + 1] = digamma_d(a) - digamma_d(a0);
        return;
    }
    if (set_q) { qp[t * 2] = q0a; qp[t * 2 + 1] = q0b; }
    const double a = qp[t * 2], b = qp[t * 2 + 1];
    if (qfamily == 0) {
        mema[t * 2] = a;
        mema[t * 2 + 1] = a * a + b;
    } else if (qfamily == QF_GAMMA_EF) {
        mema[t * 2] = a / b;
        mema[t * 2 + 1] = digamma_d(a) - log(b);
    } else if (qfamily == QF_BERNOULLI || qfamily == QF_CATEGORICAL) {
        mema[t * 2] = a;
        mema[t * 2 + 1] = a;
    } else {
        mema[t * 2] = a / b;
        mema[t * 2 + 1] = a * (a + 1.0) / (b * b);
    }
}

// Marginal effective sample size of instance i, 1 / sum_k w[i,k]^2 (FP64, k in
// lane-strided order, then the wave's shuffle tree), one wave per instance.
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_ess(const T* __restrict__ w, long n, int K, double* __restrict__ ess) {
    const long i = static_cast<long>(blockIdx.x) * (BLOCK / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (i >= n) return;
    double s = 0.0;
    for (int k = lane; k < K; k += WAVE) {
        const double x = static_cast<double>(w[i * K + k]);
        s += x * x;
    }
    s = group_sum(s, WAVE);
    if (lane == 0) ess[i] = 1.0 / s;
}

// out = the mean of v[0..n): per-thread strided sums in index order, then a
// fixed tree over the workgroup.
__global__ void __launch_bounds__(BLOCK) k_mean(const double* __restrict__ v, long n, double* __restrict__ out) {
    __shared__ double red[BLOCK];
    double s = 0.0;
    for (long i = threadIdx.x; i < n; i += BLOCK) s += v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] / static_cast<double>(n);
}

__global__ void k_iter_set(uint64_t* it, uint64_t v) {
    if (threadIdx.x == 0) *it = v;
}
__global__ void k_reset_status(uint32_t* status) {
    if (threadIdx.x < 4) status[threadIdx.x] = 0u;
}

}  // namespace

hipError_t moments(hipStream_t s, bool f64, const void* z, const void* w, double* mone, long n, int K, int d,
                   bool logz) {
    const long total = n * d;
    const dim3 grid((total + BLOCK - 1) / BLOCK);
    if (f64) hipLaunchKernelGGL(k_moments<double>, grid, dim3(BLOCK), 0, s, (const double*)z, (const double*)w, mone, n, K, d, logz);
    else hipLaunchKernelGGL(k_moments<float>, grid, dim3(BLOCK), 0, s, (const float*)z, (const float*)w, mone, n, K, d, logz);
    return hipGetLastError();
}

hipError_t mstep(hipStream_t s, double* mema, const double* mone, double* qp, long count, int qfamily, double lam,
                 uint32_t* status, int d) {
    hipLaunchKernelGGL(k_mstep, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, mema, mone, qp, count, qfamily,
                       lam, status, d);
    return hipGetLastError();
}

hipError_t init_q(hipStream_t s, double* qp, double* mema, long count, int qfamily, int set_q, double q0a,
                  double q0b, int d) {
    hipLaunchKernelGGL(k_init_q, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, qp, mema, count, qfamily, set_q,
                       q0a, q0b, d);
    return hipGetLastError();
}

hipError_t ess(hipStream_t s, bool f64, const void* w, long n, int K, double* ess_out, double* mean_out) {
    const dim3 grid(static_cast<unsigned>((n + BLOCK / WAVE - 1) / (BLOCK / WAVE)));
    if (f64) hipLaunchKernelGGL(k_ess<double>, grid, dim3(BLOCK), 0, s, (const double*)w, n, K, ess_out);
    else hipLaunchKernelGGL(k_ess<float>, grid, dim3(BLOCK), 0, s, (const float*)w, n, K, ess_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !mean_out) return e;
    hipLaunchKernelGGL(k_mean, dim3(1), dim3(BLOCK), 0, s, ess_out, n, mean_out);
    return hipGetLastError();
}

hipError_t iter_set(hipStream_t s, uint64_t* it, uint64_t v) {
    hipLaunchKernelGGL(k_iter_set, dim3(1), dim3(WAVE), 0, s, it, v);
    return hipGetLastError();
}

hipError_t mstep_multi(hipStream_t s, const MstepTable& tb, double lam, uint32_t* status, uint64_t* iter_dev) {
    long total = 0;
    for (int v = 0; v < tb.n; ++v) total += tb.count[v];
    const long blocks = std::max(1L, (total + BLOCK - 1) / BLOCK);   // one block still advances the counter
    hipLaunchKernelGGL(k_mstep_multi, dim3(blocks), dim3(BLOCK), 0, s, tb, lam, status, iter_dev);
    return hipGetLastError();
}

hipError_t copy_scalar(hipStream_t s, const double* src, double* dst) {
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(WAVE), 0, s, src, dst);
    return hipGetLastError();
}

hipError_t reset_status(hipStream_t s, uint32_t* status) {
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(WAVE), 0, s, status);
    return hipGetLastError();
}

}  // namespace qemk
