// The two-parent contraction as exponential GEMMs on MFMA (FP32 mode, K = 64
// or 128, K_a = K_b = K).  For instance i,
//
//   m[i,ka,kb] = C[ka,kb] + LSE_k (G[ka,k] + H[kb,k] + ut[i,k]),  G = ga0 + ga1 gk[i,k],
//
// splits as exp(G + H + ut) = exp(G[ka,k] - g_ka) exp(H[kb,k] + ut'[k] - h_kb)
// exp(g_ka + h_kb + c_i) with c_i = max_k ut[i,k], ut' = ut - c_i,
// g_ka = max_k G[ka,k] (closed form: G is linear in gk, so the maximum sits at
// the largest or smallest gk) and h_kb = max_k (H[kb,k] + ut'[k]):
//
//   m = C + c_i + g_ka + h_kb + log D,   D = A' B'^T,
//   A'[ka,k] = exp(ga1[ka] (gk[k] - gk_ext(ka))),  B'[kb,k] = exp(H + ut' - h_kb),
//
// every entry of A' and B' in (0, 1].  D >= exp(-B_i) with
// B_i = max_ka |ga1[ka]| range_k(gk[i,k]): the k where B' = 1 keeps at least
// that much of A'.  Instances with B_i <= TP_F32_BOUND run here in FP32
// (expf, v_mfma_f32_16x16x4f32), those with B_i <= TP_F64_BOUND in FP64 (exp,
// v_mfma_f64_16x16x4f64): every term that carries the sum stays far above
// the format's smallest normal.  The others are flagged and left to the exact
// VALU kernels, which skip every instance handled here (flags hold each
// instance's tier).
//
// The reverse pass is the transposed product:
//   w[i,k] = sum_{ka,kb} W[ka,kb] exp(G + H + C + ut - m)
//          = sum_ka A'[ka,k] (P B')[ka,k],   P[ka,kb] = W[ka,kb] exp(C + g_ka + h_kb + c_i - m[i,ka,kb])
//          = W / D.
//
// Blocks: one per instance, one wave per 16-row output tile (K / 16 waves);
// wave w owns row tile w and every column tile.  The operands are staged in
// LDS in MFMA operand order, 32 contraction steps at a time in FP32 (16 in
// FP64: the two tiers share the buffer).  Short chunks keep the LDS and
// register footprint small enough for 6-7 waves per SIMD: at K = 64 the
// whole contraction in one chunk, and at K = 128 four waves with two row
// tiles each, left half as many waves resident and took 1.3-1.6x longer.  MFMA layout (16x16x4):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 (l / 16) + r][l % 16] (FP32) or D[l / 16 + 4 r][l % 16] (FP64), r = 0..3.
#include <algorithm>
#include <cmath>

#include "qem_internal.h"
#include "dev_common.h"

namespace qemk {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr double TP_F32_BOUND = 60.0;
constexpr double TP_F64_BOUND = 600.0;
enum TpTier { TP_F32 = 0, TP_F64 = 1, TP_EXACT = TP_FLAG_EXACT };

template <int K> struct TpShape {
    static constexpr int NT = K / 16;                  // tiles per dimension
    static constexpr int KC32 = 32;                    // FP32 contraction chunk
    static constexpr int WV = K == 128 ? 8 : 4;        // waves per instance: one row tile each
    static constexpr int TPB = WV * WAVE;              // threads per instance
    static constexpr int RW = NT / WV;                 // row tiles per wave
    static constexpr int OPS_BYTES = 2 * NT * (KC32 / 4) * WAVE * 4;   // both operand stages
};

// Element-type traits of the GEMM tiers.
template <typename E> struct TpOps;
template <> struct TpOps<float> {
    typedef f32x4 acc_t;
    static constexpr bool f32 = true;
    // exp(x) as the hardware exp2 of x log2(e) (scaled in FP64, then rounded to
    // FP32 like the argument of expf); exponents stay within the tier's range bound
    __device__ static float ex(double x) { return __builtin_amdgcn_exp2f(static_cast<float>(x * 1.4426950408889634)); }
    __device__ static double lg(float d) { return static_cast<double>(logf(d)); }
    __device__ static acc_t mfma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int q, int r) { return 4 * q + r; }
};
template <> struct TpOps<double> {
    typedef f64x4 acc_t;
    static constexpr bool f32 = false;
    __device__ static double ex(double x) { return exp(x); }
    __device__ static double lg(double d) { return log(d); }
    __device__ static acc_t mfma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int q, int r) { return q + 4 * r; }
};

// The per-instance vectors both passes share: c_i (sh), gk range, g_ka,
// gk_ext(ka), h_kb; returns the instance's tier (every thread the same).
template <int K>
__device__ __forceinline__ int tp_setup(const TwoParentArgs& a, long i, double* s_gk, double* s_ut, double* s_hk,
                                        double* s_g, double* s_ext, double* s_h, double* s_scr, double* s_ga1,
                                        double* s_hb, double& sh) {
    constexpr int TPB_ = TpShape<K>::TPB;
    const int tid = threadIdx.x;
    const float* hmat = a.hmat ? static_cast<const float*>(a.hmat) + i * K * K : nullptr;
    for (int k = tid; k < K; k += TPB_) {
        s_gk[k] = a.gk[i * K + k];
        s_ut[k] = a.ut[i * K + k];
        s_hk[k] = a.hk ? a.hk[i * K + k] : 0.0;
        s_ga1[k] = a.ga1[k];
        s_hb[k] = a.hb ? a.hb[k] : 0.0;
    }
    __syncthreads();
    sh = finite_or_zero(block_max(s_ut, K, s_scr));
    double lo = __builtin_inf(), hi = -__builtin_inf(), gam = 0.0;
    for (int k = tid; k < K; k += TPB_) {
        lo = fmin(lo, s_gk[k]);
        hi = fmax(hi, s_gk[k]);
        gam = fmax(gam, fabs(s_ga1[k]));
    }
    lo = -group_max(-lo, WAVE);
    hi = group_max(hi, WAVE);
    gam = group_max(gam, WAVE);
    if ((tid & (WAVE - 1)) == 0) {
        s_scr[tid / WAVE] = lo;
        s_scr[TPB_ / WAVE + tid / WAVE] = hi;
        s_scr[2 * (TPB_ / WAVE) + tid / WAVE] = gam;
    }
    __syncthreads();
    for (int w = 0; w < TPB_ / WAVE; ++w) {
        lo = fmin(lo, s_scr[w]);
        hi = fmax(hi, s_scr[TPB_ / WAVE + w]);
        gam = fmax(gam, s_scr[2 * (TPB_ / WAVE) + w]);
    }
    __syncthreads();
    const double bound = gam * (hi - lo);
    const int tier = bound <= TP_F32_BOUND ? TP_F32 : (bound <= TP_F64_BOUND ? TP_F64 : TP_EXACT);
    if (tier == TP_EXACT) return tier;
    for (int ka = tid; ka < K; ka += TPB_) {
        const double g1 = s_ga1[ka];
        const double ext = g1 >= 0.0 ? hi : lo;
        s_ext[ka] = ext;
        s_g[ka] = (a.ga0 ? a.ga0[ka] : 0.0) + g1 * ext;
    }
    // h_kb: 16-lane row groups
    const int rg = tid / 16, l16 = tid & 15;
    for (int kb = rg; kb < K; kb += TPB_ / 16) {
        double mx = -__builtin_inf();
        for (int k = l16; k < K; k += 16) {
            const double h = hmat ? static_cast<double>(hmat[kb * K + k]) : s_hb[kb] * s_hk[k];
            mx = fmax(mx, h + (s_ut[k] - sh));
        }
        mx = group_max(mx, 16);
        if (l16 == 0) s_h[kb] = mx;
    }
    __syncthreads();
    return tier;
}

// The exponent of B'[kb,k] = exp(H + ut' - h_kb); -inf for a row whose maximum is -inf.
template <int K>
__device__ __forceinline__ double tp_bexp(const double* s_hb, const float* hmat, const double* s_hk,
                                          const double* s_ut, const double* s_h, double sh, int kb, int k) {
    const double hk = s_h[kb];
    if (hk == -__builtin_inf()) return -__builtin_inf();
    const double h = hmat ? static_cast<double>(hmat[kb * K + k]) : s_hb[kb] * s_hk[k];
    return h + (s_ut[k] - sh) - hk;
}

// Forward GEMM of one instance in element type E; writes m.
template <int K, typename E>
__device__ __forceinline__ void tp_fwd_gemm(const TwoParentArgs& a, long i, unsigned char* ops, const double* s_gk,
                                            const double* s_ut, const double* s_hk, const double* s_g,
                                            const double* s_ext, const double* s_h, const double* s_ga1,
                                            const double* s_hb, double sh) {
    typedef TpOps<E> O;
    constexpr int NT = TpShape<K>::NT, RW = TpShape<K>::RW, WV_ = TpShape<K>::WV, TPB_ = TpShape<K>::TPB;
    constexpr int KC = TpShape<K>::KC32 * 4 / static_cast<int>(sizeof(E));
    E (*sA)[KC / 4][WAVE] = reinterpret_cast<E (*)[KC / 4][WAVE]>(ops);
    E (*sB)[KC / 4][WAVE] = reinterpret_cast<E (*)[KC / 4][WAVE]>(ops + NT * (KC / 4) * WAVE * sizeof(E));
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
    const float* hmat = a.hmat ? static_cast<const float*>(a.hmat) + i * K * K : nullptr;
    typename O::acc_t acc[RW][NT];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[r][t] = typename O::acc_t{0, 0, 0, 0};
    for (int kc0 = 0; kc0 < K; kc0 += KC) {
        for (int e = tid; e < K * KC; e += TPB_) {
            const int row = e / KC, kl = e - row * KC, k = kc0 + kl;
            const int slot = (row & 15) + 16 * (kl & 3);
            sA[row >> 4][kl >> 2][slot] = O::ex(s_ga1[row] * (s_gk[k] - s_ext[row]));
            sB[row >> 4][kl >> 2][slot] = O::ex(tp_bexp<K>(s_hb, hmat, s_hk, s_ut, s_h, sh, row, k));
        }
        __syncthreads();
#pragma unroll 2
        for (int kk = 0; kk < KC / 4; ++kk) {
            E av[RW];
#pragma unroll
            for (int r = 0; r < RW; ++r) av[r] = sA[wave + WV_ * r][kk][lane];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const E bv = sB[t][kk][lane];
#pragma unroll
                for (int r = 0; r < RW; ++r) acc[r][t] = O::mfma(av[r], bv, acc[r][t]);
            }
        }
        __syncthreads();
    }
    double* mout = a.m + i * static_cast<long>(K) * K;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int ta = wave + WV_ * r;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int kb = t * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ka = ta * 16 + O::row(lane >> 4, q);
                const E d = acc[r][t][q];
                const double c = a.C ? a.C[ka * K + kb] : 0.0;
                mout[ka * K + kb] = (d > E(0) && s_h[kb] != -__builtin_inf())
                                        ? c + sh + s_g[ka] + s_h[kb] + O::lg(d)
                                        : -__builtin_inf();
            }
        }
    }
}

// Reverse GEMM of one instance in element type E; writes w[i, :].
template <int K, typename E>
__device__ __forceinline__ void tp_bwd_gemm(const TwoParentArgs& a, long i, const double* __restrict__ W,
                                            float* __restrict__ w, unsigned char* ops, double (*s_red)[K],
                                            const double* s_gk, const double* s_ut, const double* s_hk,
                                            const double* s_g, const double* s_ext, const double* s_h,
                                            const double* s_ga1, const double* s_hb, double sh) {
    typedef TpOps<E> O;
    constexpr int NT = TpShape<K>::NT, RW = TpShape<K>::RW, WV_ = TpShape<K>::WV, TPB_ = TpShape<K>::TPB;
    constexpr int KC = TpShape<K>::KC32 * 4 / static_cast<int>(sizeof(E));
    E (*sP)[KC / 4][WAVE] = reinterpret_cast<E (*)[KC / 4][WAVE]>(ops);
    E (*sB)[KC / 4][WAVE] = reinterpret_cast<E (*)[KC / 4][WAVE]>(ops + NT * (KC / 4) * WAVE * sizeof(E));
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
    const float* hmat = a.hmat ? static_cast<const float*>(a.hmat) + i * K * K : nullptr;
    const double* m = a.m + i * static_cast<long>(K) * K;
    typename O::acc_t acc[RW][NT];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[r][t] = typename O::acc_t{0, 0, 0, 0};
    // T[ka,k] = sum_kb P[ka,kb] B'[kb,k], the contraction over kb in chunks
    for (int kc0 = 0; kc0 < K; kc0 += KC) {
        for (int e = tid; e < K * KC; e += TPB_) {
            const int row = e / KC, bl = e - row * KC, kb = kc0 + bl;
            const double Wv = W[row * K + kb], mv = m[row * K + kb];
            const double c = a.C ? a.C[row * K + kb] : 0.0;
            const bool live = Wv > 0.0 && mv != -__builtin_inf();
            sP[row >> 4][bl >> 2][(row & 15) + 16 * (bl & 3)] =
                live ? static_cast<E>(Wv) * O::ex(c + s_g[row] + s_h[kb] + sh - mv) : E(0);
        }
        for (int e = tid; e < KC * K; e += TPB_) {
            const int bl = e / K, k = e - bl * K, kb = kc0 + bl;
            sB[k >> 4][bl >> 2][(k & 15) + 16 * (bl & 3)] = O::ex(tp_bexp<K>(s_hb, hmat, s_hk, s_ut, s_h, sh, kb, k));
        }
        __syncthreads();
#pragma unroll 2
        for (int kk = 0; kk < KC / 4; ++kk) {
            E av[RW];
#pragma unroll
            for (int r = 0; r < RW; ++r) av[r] = sP[wave + WV_ * r][kk][lane];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const E bv = sB[t][kk][lane];
#pragma unroll
                for (int r = 0; r < RW; ++r) acc[r][t] = O::mfma(av[r], bv, acc[r][t]);
            }
        }
        __syncthreads();
    }
    // w[k] = sum_ka A'[ka,k] T[ka,k]: per lane over its rows, then the lane
    // groups, then the waves in order
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int k = t * 16 + (lane & 15);
        double part = 0.0;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int ta = wave + WV_ * r;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ka = ta * 16 + O::row(lane >> 4, q);
                const E ap = O::ex(s_ga1[ka] * (s_gk[k] - s_ext[ka]));
                part += static_cast<double>(ap * acc[r][t][q]);
            }
        }
        part += __shfl_xor(part, 16, WAVE);
        part += __shfl_xor(part, 32, WAVE);
        if (lane < 16) s_red[wave][k] = part;
    }
    __syncthreads();
    for (int k = tid; k < K; k += TPB_) {
        double sum = 0.0;
        for (int v = 0; v < WV_; ++v) sum += s_red[v][k];
        w[i * K + k] = static_cast<float>(sum);
    }
}

// One kernel per tier, so that each has its own register allocation (the
// FP64 accumulators would otherwise halve the FP32 kernel's occupancy).  The
// FP32 forward computes every instance's tier and records it in flags
// (TP_F32 done, TP_F64 / TP_EXACT pending); the FP64 kernels and the exact
// VALU kernels take the instances flagged for them.
template <int K, typename E>
__global__ void __launch_bounds__(TpShape<K>::TPB) k_tp_fwd_mfma(TwoParentArgs a) {
    __shared__ __align__(16) unsigned char s_ops[TpShape<K>::OPS_BYTES];
    __shared__ double s_gk[K], s_ut[K], s_hk[K], s_g[K], s_ext[K], s_h[K], s_ga1[K], s_hb[K];
    __shared__ double s_scr[3 * TpShape<K>::WV];
    constexpr int MINE = sizeof(E) == 4 ? TP_F32 : TP_F64;
    const long i = blockIdx.x;
    if (MINE == TP_F64 && a.flags[i] != TP_F64) return;
    double sh;
    const int tier = tp_setup<K>(a, i, s_gk, s_ut, s_hk, s_g, s_ext, s_h, s_scr, s_ga1, s_hb, sh);
    if (MINE == TP_F32 && threadIdx.x == 0) a.flags[i] = static_cast<uint8_t>(tier);
    if (tier == MINE) tp_fwd_gemm<K, E>(a, i, s_ops, s_gk, s_ut, s_hk, s_g, s_ext, s_h, s_ga1, s_hb, sh);
}

template <int K, typename E>
__global__ void __launch_bounds__(TpShape<K>::TPB) k_tp_bwd_mfma(TwoParentArgs a, const double* __restrict__ W,
                                                       float* __restrict__ w) {
    __shared__ __align__(16) unsigned char s_ops[TpShape<K>::OPS_BYTES];
    __shared__ double s_gk[K], s_ut[K], s_hk[K], s_g[K], s_ext[K], s_h[K], s_ga1[K], s_hb[K];
    __shared__ double s_scr[3 * TpShape<K>::WV];
    __shared__ double s_red[TpShape<K>::WV][K];
    constexpr int MINE = sizeof(E) == 4 ? TP_F32 : TP_F64;
    const long i = blockIdx.x;
    if (a.flags[i] != MINE) return;
    double sh;
    tp_setup<K>(a, i, s_gk, s_ut, s_hk, s_g, s_ext, s_h, s_scr, s_ga1, s_hb, sh);
    tp_bwd_gemm<K, E>(a, i, W, w, s_ops, s_red, s_gk, s_ut, s_hk, s_g, s_ext, s_h, s_ga1, s_hb, sh);
}

}  // namespace

bool twoparent_mfma_supported(bool f64, int Ka, int Kb, int K) {
    return !f64 && Ka == K && Kb == K && (K == 64 || K == 128);
}

hipError_t twoparent_fwd_mfma(hipStream_t s, const TwoParentArgs& a) {
    if (!a.flags) return hipErrorInvalidValue;
#define QEM_TPF(KK)                                                                                    \
    hipLaunchKernelGGL((k_tp_fwd_mfma<KK, float>), dim3(a.n), dim3(TpShape<KK>::TPB), 0, s, a);                 \
    hipLaunchKernelGGL((k_tp_fwd_mfma<KK, double>), dim3(a.n), dim3(TpShape<KK>::TPB), 0, s, a)
    if (a.K == 64) { QEM_TPF(64); }
    else if (a.K == 128) { QEM_TPF(128); }
    else return hipErrorInvalidValue;
#undef QEM_TPF
    return hipGetLastError();
}

hipError_t twoparent_bwd_mfma(hipStream_t s, const TwoParentArgs& a, const double* W, void* w) {
    if (!a.flags) return hipErrorInvalidValue;
#define QEM_TPB(KK)                                                                                    \
    hipLaunchKernelGGL((k_tp_bwd_mfma<KK, float>), dim3(a.n), dim3(TpShape<KK>::TPB), 0, s, a, W, (float*)w);  \
    hipLaunchKernelGGL((k_tp_bwd_mfma<KK, double>), dim3(a.n), dim3(TpShape<KK>::TPB), 0, s, a, W, (float*)w)
    if (a.K == 64) { QEM_TPB(64); }
    else if (a.K == 128) { QEM_TPB(128); }
    else return hipErrorInvalidValue;
#undef QEM_TPB
    return hipGetLastError();
}

}  // namespace qemk
