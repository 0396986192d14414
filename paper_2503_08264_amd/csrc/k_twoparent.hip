// Elimination of a plate whose instances have two factor parents (a, b), both
// single-instance roots, and the joint root over (a, b).  This is the
// contraction of Eq. Prmp when a child links to two sampled parents, so each
// child message carries K_a x K_b entries (the max |qa| = 2 case of the
// memory bound stated in section 6):
//
//   m[i,ka,kb] = C[ka,kb] + LSE_k (G[ka,k] + H[kb,k] + ut[i,k])
//   G[ka,k]    = ga0[ka] + ga1[ka] * gk[i,k]
//   H[kb,k]    = hb[kb] * hk[i,k]     or a materialised likelihood table hmat[i,kb,k]
//   L          = LSE_{ka,kb} (ut_a[ka] + ut_b[kb] + sum_i m[i,ka,kb])
//   W[ka,kb]   = exp(ut_a + ut_b + sum_i m - L),  w_a = sum_kb W,  w_b = sum_ka W
//   w[i,k]     = sum_{ka,kb} W[ka,kb] exp(G + H + C + ut[i,k] - m[i,ka,kb])
//
// Gamma(shape a, rate b) prior:  ga1 = a - 1, gk = log z, hb = -b, hk = z,
//                                C = a log b - lgamma(a).
// N(0, exp(a)^2) prior with a Bernoulli-logit likelihood on coefficients b:
//                                ga0 = -log(2 pi)/2 - a, ga1 = -exp(-2a)/2, gk = z^2,
//                                H = likelihood table, C = 0.
//
// The forward keeps every (ka, kb, k) term exact: a two-pass (max, then sum of
// exponentials) log-sum-exp on VALU in base 2, each thread owning a 4 x 4
// block of (ka, kb).  Each instance's ut is shifted by c_i = max_k ut[i,k] before
// the FP32 arithmetic and m = C + c_i + LSE is formed and stored in FP64.
// Sums over instances are FP64 in a fixed order.
#include <algorithm>

#include "qem_internal.h"
#include "dev_common.h"

namespace qemk {

namespace {

constexpr double LOG_2PI = 1.8378770664093454835606594728112;
constexpr double LOG2E = 1.4426950408889634073599246810019;
constexpr double LN2 = 0.69314718055994530941723212145818;
constexpr int TA = 4, TB = 4;
constexpr int PAIR_CHUNKS = 32;

__device__ __forceinline__ float fexp2(float x) { return exp2f(x); }
__device__ __forceinline__ double fexp2(double x) { return exp2(x); }
__device__ __forceinline__ float flog2(float x) { return log2f(x); }
__device__ __forceinline__ double flog2(double x) { return log2(x); }

// All per-block vectors are stored pre-scaled by log2(e).
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_tp_fwd(TwoParentArgs a) {
    if (a.flags && a.flags[blockIdx.x] != TP_FLAG_EXACT) return;   // done on MFMA
    extern __shared__ unsigned char smem_raw[];
    T* s_gk = reinterpret_cast<T*>(smem_raw);   // [K]
    T* s_hk = s_gk + a.K;                         // [K]   (separable H)
    T* s_ut = s_hk + a.K;                         // [K]
    T* s_H = s_ut + a.K;                          // [Kb, K] (materialised H) or unused
    const long i = blockIdx.x;
    const int K = a.K, Ka = a.Ka, Kb = a.Kb;
    const T* hmat = static_cast<const T*>(a.hmat);
    __shared__ double s_scr[BLOCK / WAVE];
    const double sh = finite_or_zero(block_max(a.ut + i * K, K, s_scr));
    for (int k = threadIdx.x; k < K; k += BLOCK) {
        s_gk[k] = static_cast<T>(a.gk[i * K + k]);
        s_hk[k] = a.hk ? static_cast<T>(a.hk[i * K + k] * LOG2E) : T(0);
        s_ut[k] = static_cast<T>((a.ut[i * K + k] - sh) * LOG2E);
    }
    if (hmat)
        for (int e = threadIdx.x; e < Kb * K; e += BLOCK)
            s_H[e] = hmat[i * static_cast<long>(Kb) * K + e] * static_cast<T>(LOG2E);
    __syncthreads();
    const int nta = (Ka + TA - 1) / TA, ntb = (Kb + TB - 1) / TB;
    double* mout = a.m + i * static_cast<long>(Ka) * Kb;
    for (int tile = threadIdx.x; tile < nta * ntb; tile += BLOCK) {
        const int ka0 = (tile / ntb) * TA, kb0 = (tile % ntb) * TB;
        T g0[TA], g1[TA], hb[TB];
#pragma unroll
        for (int x = 0; x < TA; ++x) {
            const int ka = std::min(ka0 + x, Ka - 1);
            g0[x] = static_cast<T>((a.ga0 ? a.ga0[ka] : 0.0) * LOG2E);
            g1[x] = static_cast<T>(a.ga1[ka] * LOG2E);
        }
#pragma unroll
        for (int y = 0; y < TB; ++y) hb[y] = a.hb ? static_cast<T>(a.hb[std::min(kb0 + y, Kb - 1)]) : T(0);
        T mx[TA][TB];
#pragma unroll
        for (int x = 0; x < TA; ++x)
#pragma unroll
            for (int y = 0; y < TB; ++y) mx[x][y] = neg_inf<T>();
        for (int k = 0; k < K; ++k) {
            const T gk = s_gk[k], hk = s_hk[k], ut = s_ut[k];
            T h[TB];
#pragma unroll
            for (int y = 0; y < TB; ++y)
                h[y] = (hmat ? s_H[std::min(kb0 + y, Kb - 1) * K + k] : hb[y] * hk) + ut;
#pragma unroll
            for (int x = 0; x < TA; ++x) {
                const T g = g0[x] + g1[x] * gk;
#pragma unroll
                for (int y = 0; y < TB; ++y) mx[x][y] = fmax(mx[x][y], g + h[y]);
            }
        }
        T sm[TA][TB];
#pragma unroll
        for (int x = 0; x < TA; ++x)
#pragma unroll
            for (int y = 0; y < TB; ++y) sm[x][y] = 0;
        for (int k = 0; k < K; ++k) {
            const T gk = s_gk[k], hk = s_hk[k], ut = s_ut[k];
            T h[TB];
#pragma unroll
            for (int y = 0; y < TB; ++y)
                h[y] = (hmat ? s_H[std::min(kb0 + y, Kb - 1) * K + k] : hb[y] * hk) + ut;
#pragma unroll
            for (int x = 0; x < TA; ++x) {
                const T g = g0[x] + g1[x] * gk;
#pragma unroll
                for (int y = 0; y < TB; ++y) sm[x][y] += fexp2(g + h[y] - mx[x][y]);
            }
        }
#pragma unroll
        for (int x = 0; x < TA; ++x) {
            const int ka = ka0 + x;
            if (ka >= Ka) continue;
#pragma unroll
            for (int y = 0; y < TB; ++y) {
                const int kb = kb0 + y;
                if (kb >= Kb) continue;
                const double c = a.C ? a.C[ka * Kb + kb] : 0.0;
                mout[ka * Kb + kb] = (mx[x][y] == neg_inf<T>())
                                         ? -__builtin_inf()
                                         : c + sh + static_cast<double>(mx[x][y] + flog2(sm[x][y])) * LN2;
            }
        }
    }
}

// One block per instance; threads own columns k (parts of the ka range when K < BLOCK).
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_tp_bwd(TwoParentArgs a, const double* __restrict__ W, T* __restrict__ w) {
    if (a.flags && a.flags[blockIdx.x] != TP_FLAG_EXACT) return;   // done on MFMA
    extern __shared__ unsigned char smem_raw[];
    constexpr int CH = 16;                          // ka rows per chunk
    T* s_A = reinterpret_cast<T*>(smem_raw);        // [CH, Kb]: log2 W - log2-LSE part
    T* s_hb = s_A + CH * a.Kb;                      // [Kb]
    T* s_H = s_hb + a.Kb;                           // [Kb, K] materialised H (log2 units)
    __shared__ T s_red[BLOCK];
    const long i = blockIdx.x;
    const int K = a.K, Ka = a.Ka, Kb = a.Kb;
    const T* hmat = static_cast<const T*>(a.hmat);
    const double* m = a.m + i * static_cast<long>(Ka) * Kb;
    __shared__ double s_scr[BLOCK / WAVE];
    const double sh = finite_or_zero(block_max(a.ut + i * K, K, s_scr));
    const int parts = std::max(1, BLOCK / K);
    const int k = threadIdx.x % K;
    const int part = threadIdx.x / K;
    const bool active = threadIdx.x < parts * K;
    for (int kb = threadIdx.x; kb < Kb; kb += BLOCK) s_hb[kb] = a.hb ? static_cast<T>(a.hb[kb]) : T(0);
    if (hmat)
        for (int e = threadIdx.x; e < Kb * K; e += BLOCK)
            s_H[e] = hmat[i * static_cast<long>(Kb) * K + e] * static_cast<T>(LOG2E);
    const T gk = active ? static_cast<T>(a.gk[i * K + k]) : T(0);
    const T hk = (active && a.hk) ? static_cast<T>(a.hk[i * K + k] * LOG2E) : T(0);
    const T ut = active ? static_cast<T>((a.ut[i * K + k] - sh) * LOG2E) : T(0);
    T acc = 0;
    for (int ka0 = 0; ka0 < Ka; ka0 += CH) {
        const int rows = std::min(CH, Ka - ka0);
        __syncthreads();
        for (int e = threadIdx.x; e < rows * Kb; e += BLOCK) {
            const int ka = ka0 + e / Kb, kb = e % Kb;
            const double Wv = W[ka * Kb + kb];
            const double c = a.C ? a.C[ka * Kb + kb] : 0.0;
            const double mm = m[ka * Kb + kb] - c - sh;
            s_A[e] = (Wv > 0.0) ? static_cast<T>(log2(Wv) - mm * LOG2E) : neg_inf<T>();
        }
        __syncthreads();
        if (active) {
            for (int x = part; x < rows; x += parts) {
                const int ka = ka0 + x;
                const T g = static_cast<T>((a.ga0 ? a.ga0[ka] : 0.0) * LOG2E) +
                            static_cast<T>(a.ga1[ka] * LOG2E) * gk + ut;
                const T* Arow = s_A + x * Kb;
                for (int kb = 0; kb < Kb; ++kb) {
                    const T h = hmat ? s_H[kb * K + k] : s_hb[kb] * hk;
                    acc += fexp2(g + h + Arow[kb]);
                }
            }
        }
    }
    s_red[threadIdx.x] = active ? acc : T(0);
    __syncthreads();
    if (threadIdx.x < K) {
        T s = 0;
        for (int p = 0; p < parts; ++p) s += s_red[p * K + threadIdx.x];
        w[i * K + threadIdx.x] = s;
    }
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_tp_prep(int prior, const T* __restrict__ za, const T* __restrict__ zb,
                                                   const T* __restrict__ zc, long n, int Ka, int Kb, int K,
                                                   double* ga0, double* ga1, double* gk, double* hb, double* hk,
                                                   double* C) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const long nK = n * K;
    if (t < nK) {
        const double z = static_cast<double>(zc[t]);
        if (prior == 2) { gk[t] = log(z); hk[t] = z; }   // Gamma(shape a, rate b)
        else { gk[t] = z * z; }                          // N(0, exp(a)^2)
    }
    if (t < Ka) {
        const double av = static_cast<double>(za[t]);
        if (prior == 2) { ga0[t] = 0.0; ga1[t] = av - 1.0; }
        else { ga0[t] = -0.5 * LOG_2PI - av; ga1[t] = -0.5 * exp(-2.0 * av); }
    }
    if (prior == 2) {
        if (t < Kb) hb[t] = -static_cast<double>(zb[t]);
        if (t < static_cast<long>(Ka) * Kb) {
            const double av = static_cast<double>(za[t / Kb]);
            const double bv = static_cast<double>(zb[t % Kb]);
            C[t] = av * log(bv) - lgamma(av);
        }
    }
}

// partial[c, ka, kb] = sum over instances of chunk c; then M = sum over chunks (fixed order).
// The instances of a chunk are added in index order, their loads issued 16 at
// a time before any of them is added (a chunk is hundreds of instances long,
// and one load in flight per thread left the kernel waiting on latency).
__global__ void __launch_bounds__(BLOCK) k_pair_partial(const double* __restrict__ m, long n, int KK, double* __restrict__ part) {
    constexpr int B = 16;
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (e >= KK) return;
    const long per = (n + PAIR_CHUNKS - 1) / PAIR_CHUNKS;
    const long i0 = c * per, i1 = std::min(n, i0 + per);
    double s = 0.0;
    long i = i0;
    for (; i + B <= i1; i += B) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = m[(i + u) * KK + e];
#pragma unroll
        for (int u = 0; u < B; ++u) s += v[u];
    }
    for (; i < i1; ++i) s += m[i * KK + e];
    part[static_cast<long>(c) * KK + e] = s;
}

__global__ void __launch_bounds__(BLOCK) k_pair_final(const double* __restrict__ part, int KK, double* __restrict__ M,
                                                      int accumulate) {
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= KK) return;
    double s = 0.0;
    for (int c = 0; c < PAIR_CHUNKS; ++c) s += part[static_cast<long>(c) * KK + e];
    M[e] = accumulate ? M[e] + s : s;
}

// The joint root's L = LSE over (ka, kb) by one workgroup of ROOT_NT threads
// (every entry's exponential is FP64; more threads shorten each one's chain);
// the max is exact in any order, the sum is a fixed tree over the threads'
// strided partial sums.
constexpr int ROOT_NT = 1024;
__global__ void __launch_bounds__(ROOT_NT) k_pair_root_fwd(const double* __restrict__ uta, const double* __restrict__ utb,
                                                           const double* __restrict__ M, int Ka, int Kb, double* __restrict__ L) {
    constexpr int B = 8;   // entries whose loads are issued together
    __shared__ double red[ROOT_NT];
    const int KK = Ka * Kb;
    double mx = -__builtin_inf();
    for (int e0 = threadIdx.x; e0 < KK; e0 += B * ROOT_NT) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int e = e0 + u * ROOT_NT;
            v[u] = e < KK ? uta[e / Kb] + utb[e % Kb] + M[e] : -__builtin_inf();
        }
#pragma unroll
        for (int u = 0; u < B; ++u) mx = fmax(mx, v[u]);
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int h = ROOT_NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    mx = red[0];
    __syncthreads();
    double s = 0.0;
    if (mx != -__builtin_inf())
        for (int e0 = threadIdx.x; e0 < KK; e0 += B * ROOT_NT) {
            double v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int e = e0 + u * ROOT_NT;
                v[u] = e < KK ? uta[e / Kb] + utb[e % Kb] + M[e] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (e0 + u * ROOT_NT < KK) s += exp(v[u] - mx);   // the strided entries in index order
        }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = ROOT_NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *L = (mx == -__builtin_inf()) ? mx : mx + log(red[0]);
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_pair_root_w(const double* __restrict__ uta, const double* __restrict__ utb,
                                                       const double* __restrict__ M, const double* __restrict__ L,
                                                       int Ka, int Kb, double* __restrict__ W,
                                                       const double* __restrict__ g) {
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<long>(Ka) * Kb) return;
    const double sc = g ? *g : 1.0;
    const double Lv = *L;
    W[e] = (Lv == -__builtin_inf()) ? 0.0 : sc * exp(uta[e / Kb] + utb[e % Kb] + M[e] - Lv);
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_pair_marg(const double* __restrict__ W, int Ka, int Kb,
                                                     T* __restrict__ wa, T* __restrict__ wb) {
    // row and column sums in index order, their loads issued 16 at a time
    constexpr int B = 16;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < Ka) {
        double s = 0.0;
        int kb = 0;
        for (; kb + B <= Kb; kb += B) {
            double v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) v[u] = W[t * Kb + kb + u];
#pragma unroll
            for (int u = 0; u < B; ++u) s += v[u];
        }
        for (; kb < Kb; ++kb) s += W[t * Kb + kb];
        wa[t] = static_cast<T>(s);
    }
    if (t < Kb) {
        double s = 0.0;
        int ka = 0;
        for (; ka + B <= Ka; ka += B) {
            double v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) v[u] = W[(ka + u) * Kb + t];
#pragma unroll
            for (int u = 0; u < B; ++u) s += v[u];
        }
        for (; ka < Ka; ++ka) s += W[ka * Kb + t];
        wb[t] = static_cast<T>(s);
    }
}

size_t fwd_smem(const TwoParentArgs& a, size_t eb) {
    return (3 * static_cast<size_t>(a.K) + (a.hmat ? static_cast<size_t>(a.Kb) * a.K : 0)) * eb;
}
size_t bwd_smem(const TwoParentArgs& a, size_t eb) {
    return (16 * static_cast<size_t>(a.Kb) + a.Kb + (a.hmat ? static_cast<size_t>(a.Kb) * a.K : 0)) * eb;
}

}  // namespace

hipError_t twoparent_fwd(hipStream_t s, bool f64, const TwoParentArgs& a) {
    if (a.flags) {
        const hipError_t e = twoparent_fwd_mfma(s, a);
        if (e != hipSuccess) return e;
    }
    if (f64) hipLaunchKernelGGL(k_tp_fwd<double>, dim3(a.n), dim3(BLOCK), fwd_smem(a, 8), s, a);
    else hipLaunchKernelGGL(k_tp_fwd<float>, dim3(a.n), dim3(BLOCK), fwd_smem(a, 4), s, a);
    return hipGetLastError();
}

hipError_t twoparent_bwd(hipStream_t s, bool f64, const TwoParentArgs& a, const double* W, void* w) {
    if (a.flags) {
        const hipError_t e = twoparent_bwd_mfma(s, a, W, w);
        if (e != hipSuccess) return e;
    }
    if (f64) hipLaunchKernelGGL(k_tp_bwd<double>, dim3(a.n), dim3(BLOCK), bwd_smem(a, 8), s, a, W, (double*)w);
    else hipLaunchKernelGGL(k_tp_bwd<float>, dim3(a.n), dim3(BLOCK), bwd_smem(a, 4), s, a, W, (float*)w);
    return hipGetLastError();
}

hipError_t twoparent_prep(hipStream_t s, bool f64, int prior, const void* za, const void* zb, const void* zc,
                          long n, int Ka, int Kb, int K, double* ga0, double* ga1, double* gk, double* hb,
                          double* hk, double* C) {
    const long total = std::max<long>(n * K, static_cast<long>(Ka) * Kb);
    const dim3 grid((total + BLOCK - 1) / BLOCK);
    if (f64)
        hipLaunchKernelGGL(k_tp_prep<double>, grid, dim3(BLOCK), 0, s, prior, (const double*)za, (const double*)zb,
                           (const double*)zc, n, Ka, Kb, K, ga0, ga1, gk, hb, hk, C);
    else
        hipLaunchKernelGGL(k_tp_prep<float>, grid, dim3(BLOCK), 0, s, prior, (const float*)za, (const float*)zb,
                           (const float*)zc, n, Ka, Kb, K, ga0, ga1, gk, hb, hk, C);
    return hipGetLastError();
}

hipError_t pair_sum(hipStream_t s, bool f64, const double* m, long n, int Ka, int Kb, double* M, double* scratch,
                    int accumulate) {
    const int KK = Ka * Kb;
    const dim3 grid((KK + BLOCK - 1) / BLOCK, PAIR_CHUNKS);
    (void)f64;
    hipLaunchKernelGGL(k_pair_partial, grid, dim3(BLOCK), 0, s, m, n, KK, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pair_final, dim3((KK + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, scratch, KK, M, accumulate);
    return hipGetLastError();
}

hipError_t pair_root_fwd(hipStream_t s, const double* uta, const double* utb, const double* M, int Ka, int Kb,
                         double* L) {
    hipLaunchKernelGGL(k_pair_root_fwd, dim3(1), dim3(ROOT_NT), 0, s, uta, utb, M, Ka, Kb, L);
    return hipGetLastError();
}

hipError_t pair_root_bwd(hipStream_t s, bool f64, const double* uta, const double* utb, const double* M,
                         const double* L, int Ka, int Kb, double* W, void* wa, void* wb, const double* g) {
    const long KK = static_cast<long>(Ka) * Kb;
    hipLaunchKernelGGL(k_pair_root_w<double>, dim3((KK + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, uta, utb, M, L, Ka,
                       Kb, W, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int mx = std::max(Ka, Kb);
    if (f64) hipLaunchKernelGGL(k_pair_marg<double>, dim3((mx + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, W, Ka, Kb, (double*)wa, (double*)wb);
    else hipLaunchKernelGGL(k_pair_marg<float>, dim3((mx + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, W, Ka, Kb, (float*)wa, (float*)wb);
    return hipGetLastError();
}

}  // namespace qemk
