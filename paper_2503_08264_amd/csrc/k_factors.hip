// Log-factor tensors of log r_k (Eq. rmp), split by the latents each term
// touches:
//   unary  u_v[i,k]    = own observations + root prior - log Q(z) - log K
//   pair   F_v[i,kp,k] = prior / likelihood terms linking instance i to its
//                        factor parent's sample kp.
// The -log K per latent instance carries the 1/K^n of Eq. Prmp.
// Gaussian observations enter through (mean, centred sum of squares) per
// instance and dimension: sum_o (x_o - z)^2 = ss + J (xbar - z)^2.
#include "qem_internal.h"
#include "dev_common.h"
#include "dev_unary.h"
#include "dev_pair.h"

namespace qemk {

namespace {

__global__ void __launch_bounds__(BLOCK) k_stats_gauss(const double* __restrict__ x, int n, int J, int d,
                                                       double* __restrict__ xbar, double* __restrict__ ss) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<long>(n) * d) return;
    const long i = t / d, j = t % d;
    double s = 0.0;
    for (int o = 0; o < J; ++o) s += x[(i * J + o) * d + j];
    const double mean = s / J;
    double q = 0.0;
    for (int o = 0; o < J; ++o) {
        const double e = x[(i * J + o) * d + j] - mean;
        q += e * e;
    }
    xbar[t] = mean;
    ss[t] = q;
}

__global__ void __launch_bounds__(BLOCK) k_stats_poisson(const double* __restrict__ y, int n, int J,
                                                         double* __restrict__ sy, double* __restrict__ slg) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = 0.0, b = 0.0;
    for (int o = 0; o < J; ++o) {
        const double v = y[i * J + o];
        a += v;
        b += lgamma(v + 1.0);
    }
    sy[i] = a;
    slg[i] = b;
}

__global__ void __launch_bounds__(BLOCK) k_stats_mixture(const double* __restrict__ y, const double* __restrict__ mu,
                                                         int n, int J, int C, double c0, double hp,
                                                         double* __restrict__ lik) {
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<long>(n) * C) return;
    const long i = e / C;
    const double m = mu[e % C];
    double s = 0.0;
    for (int o = 0; o < J; ++o) {
        const double d = y[i * J + o] - m;
        s += c0 - hp * d * d;
    }
    lik[e] = s;
}

// One block per child instance i: its samples' categories are staged in LDS,
// then F[i, kp, k] = log pi^kp[c_k] is written row by row (coalesced).  With
// TABLE the Kp x C logarithms of the parent's samples are formed once in LDS
// (CATP_TABLE_MAX entries at most) and every entry is a lookup.
constexpr int CATP_TABLE_MAX = 4096;

template <typename T, bool TABLE>
__global__ void __launch_bounds__(BLOCK) k_pair_categorical(T* __restrict__ F, const T* __restrict__ zc,
                                                            const T* __restrict__ zp, const int32_t* __restrict__ pidx,
                                                            int K, int Kp, int C) {
    __shared__ int s_cat[512];
    __shared__ T s_lp[TABLE ? CATP_TABLE_MAX : 1];
    const long i = blockIdx.x;
    const T* pi = zp + static_cast<long>(pidx ? pidx[i] : 0) * Kp * C;
    for (int k = threadIdx.x; k < K; k += BLOCK) {
        const T* z = zc + (i * K + k) * C;
        int cat = C - 1;
        for (int c = C - 1; c >= 0; --c)
            if (z[c] != T(0)) cat = c;
        s_cat[k] = cat;
    }
    if constexpr (TABLE)
        for (int e = threadIdx.x; e < Kp * C; e += BLOCK) s_lp[e] = static_cast<T>(log(static_cast<double>(pi[e])));
    __syncthreads();
    T* Fi = F + i * Kp * K;
    for (int r = threadIdx.x; r < Kp * K; r += BLOCK) {
        const int kp = r / K, k = r - kp * K;
        if constexpr (TABLE) Fi[r] = s_lp[kp * C + s_cat[k]];
        else Fi[r] = static_cast<T>(log(static_cast<double>(pi[kp * C + s_cat[k]])));
    }
}

__global__ void __launch_bounds__(BLOCK) k_stats_categorical(const double* __restrict__ y, int n, int J, int C,
                                                             double* __restrict__ cnt) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double c[MAX_DIM];
    for (int j = 0; j < C; ++j) c[j] = 0.0;
    for (int o = 0; o < J; ++o) {
        const double v = y[i * J + o];
        for (int j = 0; j < C; ++j) c[j] += (v == static_cast<double>(j)) ? 1.0 : 0.0;
    }
    for (int j = 0; j < C; ++j) cnt[i * C + j] = c[j];
}

template <typename T, int D>
__global__ void __launch_bounds__(BLOCK) k_unary(UnaryArgs a) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<long>(a.n) * a.K) return;
    const int d = D > 0 ? D : a.d;
    const long i = t / a.K;
    const T* z = static_cast<const T*>(a.z) + t * d;
    double zd[D > 0 ? D : MAX_DIM];
#pragma unroll
    for (int j = 0; j < d; ++j) zd[j] = static_cast<double>(z[j]);
    static_cast<T*>(a.u)[t] = static_cast<T>(unary_value<D>(a, i, zd));
}

// One block per tile r; tile = Kp x K entries written as 16-byte vectors.
template <typename T, int VEC>
__global__ void __launch_bounds__(BLOCK) k_pair_normal(T* __restrict__ F, const T* __restrict__ zc,
                                                       const T* __restrict__ zp, const int32_t* __restrict__ pidx,
                                                       int K, int Kp, int d, T a, T b, T c0, T half_prec,
                                                       int chain_T, bool nt) {
    extern __shared__ unsigned char smem_raw[];
    T* s_mean = reinterpret_cast<T*>(smem_raw);   // [Kp, d]: a*zp + b
    T* s_c = s_mean + Kp * d;                      // [K, d]
    const long r = blockIdx.x;
    long ci, pi;
    if (chain_T > 1) {
        const long g = r / (chain_T - 1), t = r % (chain_T - 1) + 1;
        ci = g * chain_T + t;
        pi = ci - 1;
    } else {
        ci = r;
        pi = pidx ? pidx[r] : 0;
    }
    for (int e = threadIdx.x; e < Kp * d; e += blockDim.x) s_mean[e] = pair_mean(a, zp[pi * Kp * d + e], b);
    for (int e = threadIdx.x; e < K * d; e += blockDim.x) s_c[e] = zc[ci * K * d + e];
    __syncthreads();
    const long tile = static_cast<long>(Kp) * K;
    T* out = F + r * tile;
    for (long f0 = static_cast<long>(threadIdx.x) * VEC; f0 < tile; f0 += static_cast<long>(blockDim.x) * VEC) {
        T v[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            const long f = f0 + q;
            const int kp = static_cast<int>(f / K), k = static_cast<int>(f % K);
            v[q] = normal_pair_value<T, 0>(s_c + k * d, s_mean + kp * d, d, c0, half_prec);
        }
        store_vec_hint<T, VEC>(out + f0, v, nt);
    }
}

// Fast path when BLOCK*VEC is a multiple of K: each thread keeps the samples of
// its VEC columns in registers and walks the rows kp of the tile, writing
// 16-byte vectors; a wave writes whole consecutive rows.
template <typename T, int VEC, int D>
__global__ void __launch_bounds__(BLOCK) k_pair_normal_cols(T* __restrict__ F, const T* __restrict__ zc,
                                                            const T* __restrict__ zp, const int32_t* __restrict__ pidx,
                                                            int K, int Kp, T a, T b, T c0, T half_prec, int chain_T,
                                                            bool nt) {
    extern __shared__ unsigned char smem_raw[];
    T* s_mean = reinterpret_cast<T*>(smem_raw);   // [Kp, D]: a*zp + b
    const long r = blockIdx.x;
    long ci, pi;
    if (chain_T > 1) {
        const long g = r / (chain_T - 1), t = r % (chain_T - 1) + 1;
        ci = g * chain_T + t;
        pi = ci - 1;
    } else {
        ci = r;
        pi = pidx ? pidx[r] : 0;
    }
    for (int e = threadIdx.x; e < Kp * D; e += blockDim.x) s_mean[e] = pair_mean(a, zp[pi * Kp * D + e], b);
    const int k0 = (threadIdx.x * VEC) % K;
    const int row0 = (threadIdx.x * VEC) / K;
    const int rows_per_pass = (BLOCK * VEC) / K;
    T zr[VEC][D];
#pragma unroll
    for (int q = 0; q < VEC; ++q)
#pragma unroll
        for (int j = 0; j < D; ++j) zr[q][j] = zc[(ci * K + k0 + q) * D + j];
    __syncthreads();
    T* out = F + r * static_cast<long>(Kp) * K + k0;
    for (int kp = row0; kp < Kp; kp += rows_per_pass) {
        T mean[D];
#pragma unroll
        for (int j = 0; j < D; ++j) mean[j] = s_mean[kp * D + j];
        T v[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) v[q] = normal_pair_value<T, D>(zr[q], mean, D, c0, half_prec);
        store_vec_hint<T, VEC>(out + static_cast<long>(kp) * K, v, nt);
    }
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_pair_logscale(T* __restrict__ F, const T* __restrict__ zc,
                                                         const T* __restrict__ zp, long n, int K, int Kp) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * Kp * K) return;
    const long i = t / (static_cast<long>(Kp) * K);
    const int kp = static_cast<int>((t / K) % Kp), k = static_cast<int>(t % K);
    const double ls = static_cast<double>(zp[kp]);
    const double z = static_cast<double>(zc[i * K + k]);
    F[t] = static_cast<T>(-0.5 * LOG_2PI_D - ls - 0.5 * z * z * exp(-2.0 * ls));
}

// One block per instance i: s[kb][o] = cov[i,o,:] . beta[kb,:] in LDS, then
// F[i,kb,k] = sum_o y_o (s + z_k) - softplus(s + z_k).
// softplus(x) = max(x, 0) + log(1 + exp(-|x|)).  FP64: log1p.  FP32: the
// hardware exp and log; 1 + exp(-|x|) drops at most half an ulp of 1, an
// absolute error below 6e-8 per term.
__device__ __forceinline__ double softplus(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }
__device__ __forceinline__ float softplus(float x) { return fmaxf(x, 0.0f) + __logf(1.0f + __expf(-fabsf(x))); }

// Bernoulli-logit prior of a discrete child: F[i,kp,k] = z_k eta - softplus(eta),
// eta = a zp[p(i),kp] + b, in the arithmetic of T (softplus as above).
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_pair_bern_prior(T* __restrict__ F, const T* __restrict__ zc,
                                                           const T* __restrict__ zp, const int32_t* __restrict__ pidx,
                                                           long n, int K, int Kp, T a, T b) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * Kp * K) return;
    const long i = t / (static_cast<long>(Kp) * K);
    const int kp = static_cast<int>((t / K) % Kp), k = static_cast<int>(t % K);
    const long pi = pidx ? pidx[i] : 0;
    const T eta = a * zp[pi * Kp + kp] + b;
    const T sp = softplus(eta);
    F[t] = zc[i * K + k] != T(0) ? eta - sp : -sp;
}

// FP32 works in base 2 (the hardware exp2 and log2) and sums the log terms
// as the log of their product: each factor 1 + 2^-|x'| lies in (1, 2], so a
// product of 64 stays below 2^64 and is folded into the sum (one log) every
// 64 observations: one log per 64 terms instead of one per term, with the
// product's rounding (one fused multiply-add, about 6e-8 relative, per
// factor) in place of one log's per term.  The positive part max(x, 0) is
// taken as (x + |x|) / 2: the sum of the x over the observations is
// sum_o s_o + J z, which enters through the row's constant (sum_o y_o s_o -
// sum_o s_o / 2) and the coefficient of z (sum_o y_o - J / 2), so a term
// costs one add, one exp2, one add of |x'| and one fused multiply-add (the
// rounding of sum_o |x| and of the two separated sums, each at most
// J eps sum_o |x|, replaces that of the positive parts).  s holds each kb's
// row of J values padded to a multiple of 4, read four at a time.
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_pair_bernoulli(T* __restrict__ F, const T* __restrict__ zc,
                                                          const T* __restrict__ zbeta, const double* __restrict__ y,
                                                          const double* __restrict__ cov, int K, int Kb, int J, int D) {
    extern __shared__ unsigned char smem_raw[];
    const int Jp = (J + 3) & ~3;
    double* s_cov = reinterpret_cast<double*>(smem_raw);   // [J, D]: the instance's covariates
    double* s_beta = s_cov + J * D;                         // [Kb, D + 1]: the beta samples (padded rows)
    T* s_s = reinterpret_cast<T*>(s_beta + Kb * (D + 1));   // [Kb, Jp]
    T* s_y = s_s + Kb * Jp;                                 // [J]
    T* s_ys = s_y + J;                                      // [Kb]: sum_o y_o s[kb][o]
    const long i = blockIdx.x;
    // the covariates and the beta samples staged first (coalesced loads, all
    // in flight together); the dot products then read LDS
    for (int e = threadIdx.x; e < J * D; e += blockDim.x) s_cov[e] = cov[i * J * D + e];
    for (int e = threadIdx.x; e < Kb * D; e += blockDim.x)
        s_beta[(e / D) * (D + 1) + e % D] = static_cast<double>(zbeta[e]);
    for (int o = threadIdx.x; o < J; o += blockDim.x) s_y[o] = static_cast<T>(y[i * J + o]);
    __syncthreads();
    for (int e = threadIdx.x; e < J * Kb; e += blockDim.x) {
        const int o = e / Kb, kb = e % Kb;
        double acc = 0.0;
        for (int q = 0; q < D; ++q) acc += s_cov[o * D + q] * s_beta[kb * (D + 1) + q];
        s_s[kb * Jp + o] = static_cast<T>(acc);
    }
    __syncthreads();
    constexpr bool F32 = sizeof(T) == 4;
    double ysum = 0.0;
    for (int o = 0; o < J; ++o) ysum += static_cast<double>(s_y[o]);
    if constexpr (F32) ysum -= 0.5 * J;
    for (int kb = threadIdx.x; kb < Kb; kb += blockDim.x) {
        T acc = 0, rs = 0;
        for (int o = 0; o < J; ++o) {
            acc += s_y[o] * s_s[kb * Jp + o];
            if constexpr (F32) rs += s_s[kb * Jp + o];
        }
        s_ys[kb] = F32 ? acc - T(0.5) * rs : acc;
    }
    __syncthreads();
    const long tile = static_cast<long>(Kb) * K;
    for (long f = threadIdx.x; f < tile; f += blockDim.x) {
        const int kb = static_cast<int>(f / K), k = static_cast<int>(f % K);
        const T z = zc[i * K + k];
        const T* row = s_s + kb * Jp;
        T sp = 0;
        if constexpr (F32) {
            // base 2: x' = x log2(e); softplus(x) = ln 2 ((x' + |x'|) / 2 + log2(1 + 2^-|x'|)),
            // the x' / 2 part being in s_ys and ysum
            constexpr float L2E = 1.44269504088896341f, LN2 = 0.693147180559945309f;
            const float z2 = z * L2E;
            float abss = 0.0f, lsum = 0.0f, prod = 1.0f;
            const int J4 = J & ~3;
            for (int c0 = 0; c0 < J4; c0 += 64) {
                if (c0 > 0) {   // fold the previous 64 factors
                    lsum += __builtin_amdgcn_logf(prod);
                    prod = 1.0f;
                }
                const int ce = c0 + 64 < J4 ? c0 + 64 : J4;
#pragma unroll 4
                for (int o = c0; o < ce; o += 4) {
                    const float4 e4 = *reinterpret_cast<const float4*>(row + o);
                    const float eta[4] = {fmaf(e4.x, L2E, z2), fmaf(e4.y, L2E, z2), fmaf(e4.z, L2E, z2),
                                          fmaf(e4.w, L2E, z2)};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        abss += fabsf(eta[q]);
                        prod = fmaf(prod, __builtin_amdgcn_exp2f(-fabsf(eta[q])), prod);
                    }
                }
            }
            for (int o = J4; o < J; ++o) {   // at most 3 more factors: the product stays below 2^67
                const float eta = fmaf(row[o], L2E, z2);
                abss += fabsf(eta);
                prod = fmaf(prod, __builtin_amdgcn_exp2f(-fabsf(eta)), prod);
            }
            sp = LN2 * (0.5f * abss + (lsum + __builtin_amdgcn_logf(prod)));
        } else {
            for (int o = 0; o < J; ++o) sp += softplus(row[o] + z);
        }
        F[i * tile + f] = s_ys[kb] + z * static_cast<T>(ysum) - sp;
    }
}

}  // namespace

hipError_t stats_gauss(hipStream_t s, const double* x, int n, int J, int d, double* xbar, double* ss) {
    const long total = static_cast<long>(n) * d;
    hipLaunchKernelGGL(k_stats_gauss, dim3((total + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, x, n, J, d, xbar, ss);
    return hipGetLastError();
}

hipError_t stats_poisson(hipStream_t s, const double* y, int n, int J, double* sy, double* slg) {
    hipLaunchKernelGGL(k_stats_poisson, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, y, n, J, sy, slg);
    return hipGetLastError();
}

hipError_t stats_gauss_mixture(hipStream_t s, const double* y, const double* mu, int n, int J, int C, double var,
                               double* lik) {
    const long total = static_cast<long>(n) * C;
    hipLaunchKernelGGL(k_stats_mixture, dim3((total + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, y, mu, n, J, C,
                       -0.5 * (LOG_2PI_D + std::log(var)), 0.5 / var, lik);
    return hipGetLastError();
}

hipError_t pair_categorical(hipStream_t s, bool f64, void* F, const void* zc, const void* zp, const int32_t* pidx,
                            long n, int K, int Kp, int C) {
    if (K > 512) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(n));
    const bool table = Kp * C <= CATP_TABLE_MAX;
#define QEM_CATP(T, TB) \
    hipLaunchKernelGGL((k_pair_categorical<T, TB>), grid, dim3(BLOCK), 0, s, (T*)F, (const T*)zc, (const T*)zp, pidx, K, Kp, C)
    if (f64) { if (table) QEM_CATP(double, true); else QEM_CATP(double, false); }
    else { if (table) QEM_CATP(float, true); else QEM_CATP(float, false); }
#undef QEM_CATP
    return hipGetLastError();
}

hipError_t stats_categorical(hipStream_t s, const double* y, int n, int J, int C, double* cnt) {
    hipLaunchKernelGGL(k_stats_categorical, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, y, n, J, C, cnt);
    return hipGetLastError();
}

hipError_t stats_bernoulli(hipStream_t, const double*, const double*, int, int, int, double*, double*) {
    return hipSuccess;   // the Bernoulli factor reads raw (y, cov); nothing to precompute
}

template <typename T>
void launch_unary(hipStream_t s, dim3 grid, const UnaryArgs& a) {
    switch (a.d) {
        case 1: hipLaunchKernelGGL((k_unary<T, 1>), grid, dim3(BLOCK), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_unary<T, 2>), grid, dim3(BLOCK), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_unary<T, 4>), grid, dim3(BLOCK), 0, s, a); break;
        case 8: hipLaunchKernelGGL((k_unary<T, 8>), grid, dim3(BLOCK), 0, s, a); break;
        default: hipLaunchKernelGGL((k_unary<T, 0>), grid, dim3(BLOCK), 0, s, a); break;
    }
}

void unary_consts(UnaryArgs& a) {
    a.neg_log_K = -std::log(static_cast<double>(a.K));
    a.prior_c0 = 0.0;
    a.prior_hp = 0.0;
    if (a.prior_term == PT_NORMAL || a.prior_term == PT_CHAIN_START) {
        a.prior_c0 = -0.5 * (LOG_2PI_D + std::log(a.pvar));
        a.prior_hp = 0.5 / a.pvar;
    } else if (a.prior_term == PT_GAMMA) {
        a.prior_c0 = a.pshape * std::log(a.prate) - std::lgamma(a.pshape);
    } else if (a.prior_term == PT_CAT) {
        a.prior_c0 = -std::log(static_cast<double>(a.d));
    } else if (a.prior_term == PT_DIR) {
        a.prior_c0 = std::lgamma(a.d * a.pshape) - a.d * std::lgamma(a.pshape);
        a.prior_hp = a.pshape - 1.0;
    } else if (a.prior_term == PT_BERN) {
        // log sigmoid(+-b) = -softplus(-+b)
        const auto softplus_h = [](double x) { return std::max(x, 0.0) + std::log1p(std::exp(-std::fabs(x))); };
        a.prior_c0 = -softplus_h(-a.pb);
        a.prior_hp = -softplus_h(a.pb);
    }
    a.g_c0 = 0.0;
    a.g_hp = 0.0;
    if (a.g_xbar) {
        a.g_c0 = -0.5 * a.g_J * (LOG_2PI_D + std::log(a.g_var));
        a.g_hp = 0.5 / a.g_var;
    }
}

hipError_t unary(hipStream_t s, bool f64, const UnaryArgs& a) {
    const long total = static_cast<long>(a.n) * a.K;
    const dim3 grid((total + BLOCK - 1) / BLOCK);
    if (f64) launch_unary<double>(s, grid, a);
    else launch_unary<float>(s, grid, a);
    return hipGetLastError();
}

hipError_t pair_normal(hipStream_t s, bool f64, void* F, const void* zc, const void* zp,
                       const int32_t* pidx, long R, int K, int Kp, int d,
                       double a, double b, double var, int chain_T) {
    double c0, hp;
    normal_pair_consts(d, var, &c0, &hp);
    const int vf = f64 ? 2 : 4;
    const bool nt = static_cast<size_t>(R) * Kp * K * (f64 ? 8 : 4) > STREAM_BYTES;
    const bool cols = (K % vf == 0) && ((BLOCK * vf) % K == 0) && (d == 1 || d == 2 || d == 3 || d == 4 || d == 8);
    if (cols) {
        const size_t sm = static_cast<size_t>(Kp) * d * (f64 ? 8 : 4);
#define QEM_PN_COLS(TT, VV, DD)                                                                                 \
    hipLaunchKernelGGL((k_pair_normal_cols<TT, VV, DD>), dim3(R), dim3(BLOCK), sm, s, (TT*)F, (const TT*)zc,       \
                       (const TT*)zp, pidx, K, Kp, (TT)a, (TT)b, (TT)c0, (TT)hp, chain_T, nt)
#define QEM_PN_D(TT, VV)                     \
    switch (d) {                             \
        case 1: QEM_PN_COLS(TT, VV, 1); break; \
        case 2: QEM_PN_COLS(TT, VV, 2); break; \
        case 3: QEM_PN_COLS(TT, VV, 3); break; \
        case 4: QEM_PN_COLS(TT, VV, 4); break; \
        default: QEM_PN_COLS(TT, VV, 8); break; \
    }
        if (f64) { QEM_PN_D(double, 2) } else { QEM_PN_D(float, 4) }
#undef QEM_PN_D
#undef QEM_PN_COLS
        return hipGetLastError();
    }
    if (f64) {
        const size_t sm = static_cast<size_t>(Kp + K) * d * sizeof(double);
        if (K % 2 == 0)
            hipLaunchKernelGGL((k_pair_normal<double, 2>), dim3(R), dim3(BLOCK), sm, s, (double*)F, (const double*)zc,
                               (const double*)zp, pidx, K, Kp, d, a, b, c0, hp, chain_T, nt);
        else
            hipLaunchKernelGGL((k_pair_normal<double, 1>), dim3(R), dim3(BLOCK), sm, s, (double*)F, (const double*)zc,
                               (const double*)zp, pidx, K, Kp, d, a, b, c0, hp, chain_T, nt);
    } else {
        const size_t sm = static_cast<size_t>(Kp + K) * d * sizeof(float);
        if (K % 4 == 0)
            hipLaunchKernelGGL((k_pair_normal<float, 4>), dim3(R), dim3(BLOCK), sm, s, (float*)F, (const float*)zc,
                               (const float*)zp, pidx, K, Kp, d, (float)a, (float)b, (float)c0, (float)hp, chain_T, nt);
        else
            hipLaunchKernelGGL((k_pair_normal<float, 1>), dim3(R), dim3(BLOCK), sm, s, (float*)F, (const float*)zc,
                               (const float*)zp, pidx, K, Kp, d, (float)a, (float)b, (float)c0, (float)hp, chain_T, nt);
    }
    return hipGetLastError();
}

hipError_t pair_logscale(hipStream_t s, bool f64, void* F, const void* zc, const void* zp, long n, int K, int Kp) {
    const long total = n * Kp * K;
    const dim3 grid((total + BLOCK - 1) / BLOCK);
    if (f64) hipLaunchKernelGGL(k_pair_logscale<double>, grid, dim3(BLOCK), 0, s, (double*)F, (const double*)zc, (const double*)zp, n, K, Kp);
    else hipLaunchKernelGGL(k_pair_logscale<float>, grid, dim3(BLOCK), 0, s, (float*)F, (const float*)zc, (const float*)zp, n, K, Kp);
    return hipGetLastError();
}

hipError_t pair_bern_prior(hipStream_t s, bool f64, void* F, const void* zc, const void* zp, const int32_t* pidx,
                           long n, int K, int Kp, double a, double b) {
    const long total = n * Kp * K;
    const dim3 grid((total + BLOCK - 1) / BLOCK);
    if (f64) hipLaunchKernelGGL(k_pair_bern_prior<double>, grid, dim3(BLOCK), 0, s, (double*)F, (const double*)zc,
                                (const double*)zp, pidx, n, K, Kp, a, b);
    else hipLaunchKernelGGL(k_pair_bern_prior<float>, grid, dim3(BLOCK), 0, s, (float*)F, (const float*)zc,
                            (const float*)zp, pidx, n, K, Kp, static_cast<float>(a), static_cast<float>(b));
    return hipGetLastError();
}

hipError_t pair_bernoulli(hipStream_t s, bool f64, void* F, const void* zc, const void* zbeta,
                          const double* y, const double* cov, const double*, const double*,
                          long n, int K, int Kb, int J, int D) {
    // LDS: covariates [J, D] and padded beta samples [Kb, D + 1] in FP64, then
    // the dot products [Kb, Jp], the outcomes [J] and their sums [Kb] in T
    const size_t staged = static_cast<size_t>(J * D + Kb * (D + 1)) * sizeof(double);
    const size_t rows = static_cast<size_t>(((J + 3) & ~3) * Kb + J + Kb);
    if (f64) {
        hipLaunchKernelGGL(k_pair_bernoulli<double>, dim3(n), dim3(BLOCK), staged + rows * sizeof(double), s, (double*)F,
                           (const double*)zc, (const double*)zbeta, y, cov, K, Kb, J, D);
    } else {
        hipLaunchKernelGGL(k_pair_bernoulli<float>, dim3(n), dim3(BLOCK), staged + rows * sizeof(float), s, (float*)F,
                           (const float*)zc, (const float*)zbeta, y, cov, K, Kb, J, D);
    }
    return hipGetLastError();
}

}  // namespace qemk
