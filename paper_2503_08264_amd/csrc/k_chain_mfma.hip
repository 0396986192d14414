// Chains in BF16-exp mode: the K x K log-semiring products along a series run
// as max-shifted exponential GEMMs in BF16 on MFMA with FP32 accumulation.
//
// Factors.  For step t of series g:  F_t[kp,k] = log N(z_t^k; a z_{t-1}^kp + b, var),
// stored as  A_t[kp,k] = bf16(exp(F_t[kp,k] - c_t[kp]))  with the FP32 row
// shift c_t[kp] = max_k F_t[kp,k], so every stored entry lies in [0, 1].
//
// Forward (elimination from the last step to the first, as the VALU chain):
// the carried transfer matrix R_t[k, kend] = sum over paths from (t, k) to
// (T-1, kend) of exp(factors) is kept as BF16 entries R~ in [0,1] with FP32
// column log-scales r[kend]:
//   P        = A_t * R~_t                                   (MFMA, FP32 accumulation)
//   m_t[kp]  = c_t[kp] + log sum_kend exp(r[kend]) P[kp,kend]   (message into t-1)
//   R~_{t-1} = bf16( P * f[kp] / colmax[kend] ),  f[kp] = exp(ut_{t-1}[kp] + c_t[kp] - mu)
//   r[kend] += mu + log colmax[kend]
// with R~_{T-1} = I and r = ut_{T-1}.  Each step executes 2 K^3 flops where a
// message-vector recursion needs 2 K^2: the carried matrix resolves every
// end-state of the series (it is the product of all transfer matrices).
// log P_MP of the series is LSE_k(ut_0[k] + m_1[k]).
//
// MFMA layout (v_mfma_f32_16x16x32_bf16): lane l = 16 j + i holds A row i,
// B column i, and k values that are free to permute as long as A and B agree.
// The carried matrix stays in registers: the D fragment of row tiles 2c and
// 2c+1 (rows 4j..4j+3 and 16+4j..16+4j+3 of the 32-row chunk c) becomes the
// B fragment of chunk c, so A fragments are read with the same k order:
// {32c + 4j + 0..3, 32c + 16 + 4j + 0..3}.
//
// Weights (reverse pass) use the stored BF16 factors on VALU:
//   w_t[k] = sum_kp w_{t-1}[kp] exp(c_t[kp] + log A_t[kp,k] + ut~_t[k] - m_t[kp]),
// renormalised to sum to one at every step.
#include <algorithm>

#include "qem_internal.h"
#include "dev_common.h"

namespace qemk {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr double LOG_2PI = 1.8378770664093454835606594728112;
constexpr float LOG2E_F = 1.44269504088896340736f;

// ------------------------------------------------------------------ factors
// One block per (series, step t >= 1); groups of K/8 lanes own a row, each
// lane 8 consecutive columns written as one 16-byte vector.
template <int K>
__global__ void __launch_bounds__(BLOCK) k_chain_bexp_factors(const float* __restrict__ z, __bf16* __restrict__ A,
                                                              float* __restrict__ csh, int T, float a, float b,
                                                              float c0, float half_prec) {
    constexpr int LPR = K / 8;
    constexpr int GROUPS = BLOCK / LPR;
    __shared__ float s_zc[K], s_mean[K];
    const long r = blockIdx.x;
    const long g = r / (T - 1), t = r % (T - 1) + 1;
    for (int k = threadIdx.x; k < K; k += BLOCK) {
        s_zc[k] = z[(g * T + t) * K + k];
        s_mean[k] = a * z[(g * T + t - 1) * K + k] + b;
    }
    __syncthreads();
    const int lane = threadIdx.x % LPR, grp = threadIdx.x / LPR;
    __bf16* out = A + r * static_cast<long>(K) * K;
    for (int kp = grp; kp < K; kp += GROUPS) {
        const float mean = s_mean[kp];
        float f[8];
        float mx = -__builtin_inff();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float e = s_zc[lane * 8 + q] - mean;
            f[q] = c0 - half_prec * e * e;
            mx = fmaxf(mx, f[q]);
        }
        mx = group_max(mx, LPR);
        bf16x8 v;
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = static_cast<__bf16>(__expf(f[q] - mx));
        __builtin_nontemporal_store(v, reinterpret_cast<bf16x8*>(out + static_cast<long>(kp) * K + lane * 8));
        if (lane == 0) csh[r * K + kp] = mx;
    }
}

// ------------------------------------------------------------------ MFMA fold
template <int K>
__global__ void __launch_bounds__(2 * K) k_chain_fold_mfma(const __bf16* __restrict__ A, const float* __restrict__ csh,
                                                           double* __restrict__ ut, double* __restrict__ msg,
                                                           double* __restrict__ L, int T) {
    constexpr int W = K / 32;          // waves; each owns 32 columns (two 16-column tiles)
    constexpr int RT = K / 16;         // row tiles
    constexpr int NC = K / 32;         // 32-wide contraction chunks
    constexpr int NT = 64 * W;
    constexpr int LDA = K + 8;         // padded LDS row (bf16 elements)
    __shared__ __bf16 s_a[2][16 * LDA];
    __shared__ float s_r[K];
    __shared__ float s_f[K];
    __shared__ float s_red[W][K];
    __shared__ float s_scal[2];
    __shared__ double s_dred[NT / 64];
    const int tid = threadIdx.x, wave = tid / 64, l = tid % 64, j = l / 16, li = l % 16;
    const long g = blockIdx.x;
    const int col0 = wave * 32 + li, col1 = wave * 32 + 16 + li;

    bf16x8 bop[NC][2];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = 32 * c + (q < 4 ? 4 * j + q : 16 + 4 * j + (q - 4));
            bop[c][0][q] = static_cast<__bf16>(k == col0 ? 1.0f : 0.0f);
            bop[c][1][q] = static_cast<__bf16>(k == col1 ? 1.0f : 0.0f);
        }
    for (int e = tid; e < K; e += NT) s_r[e] = static_cast<float>(ut[(g * T + T - 1) * K + e]);
    __syncthreads();

    for (int t = T - 1; t >= 1; --t) {
        const __bf16* At = A + (g * (T - 1) + (t - 1)) * static_cast<long>(K) * K;
        const float* ct = csh + (g * (T - 1) + (t - 1)) * K;
        f32x4 acc[RT][2];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            acc[rt][0] = f32x4{0.f, 0.f, 0.f, 0.f};
            acc[rt][1] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        // Rows [16 rt, 16 rt + 16) of A_t are 2 K 16-byte vectors: one per thread
        // (NT = 2 K).  The next tile is loaded into registers while the
        // current tile's MFMAs run, then stored to the other LDS buffer.
        const int srow = tid / (K / 8), sc8 = tid % (K / 8);
        bf16x8 pre = __builtin_nontemporal_load(reinterpret_cast<const bf16x8*>(At + static_cast<long>(srow) * K + sc8 * 8));
        *reinterpret_cast<bf16x8*>(s_a[0] + srow * LDA + sc8 * 8) = pre;
        __syncthreads();
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            if (rt + 1 < RT)
                pre = __builtin_nontemporal_load(
                    reinterpret_cast<const bf16x8*>(At + static_cast<long>(16 * (rt + 1) + srow) * K + sc8 * 8));
            const __bf16* sa = s_a[rt & 1];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const bf16x4 lo = *reinterpret_cast<const bf16x4*>(sa + li * LDA + 32 * c + 4 * j);
                const bf16x4 hi = *reinterpret_cast<const bf16x4*>(sa + li * LDA + 32 * c + 16 + 4 * j);
                const bf16x8 av = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                acc[rt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[c][0], acc[rt][0], 0, 0, 0);
                acc[rt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[c][1], acc[rt][1], 0, 0, 0);
            }
            if (rt + 1 < RT) *reinterpret_cast<bf16x8*>(s_a[(rt + 1) & 1] + srow * LDA + sc8 * 8) = pre;
            __syncthreads();
        }
        // messages m_t[kp] = c_t[kp] + rmax + log sum_kend exp(r - rmax) P[kp, kend]
        if (wave == 0) {
            float mx = -__builtin_inff();
            for (int e = l; e < K; e += 64) mx = fmaxf(mx, s_r[e]);
            mx = group_max(mx, 64);
            if (l == 0) s_scal[0] = mx;
        }
        __syncthreads();
        const float rmax = s_scal[0];
        const float e0 = (rmax == -__builtin_inff()) ? 0.f : __expf(s_r[col0] - rmax);
        const float e1 = (rmax == -__builtin_inff()) ? 0.f : __expf(s_r[col1] - rmax);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float v = acc[rt][0][q] * e0 + acc[rt][1][q] * e1;
                v = group_sum(v, 16);
                if (li == 0) s_red[wave][16 * rt + 4 * j + q] = v;
            }
        __syncthreads();
        for (int kp = tid; kp < K; kp += NT) {
            float s = 0.f;
#pragma unroll
            for (int w = 0; w < W; ++w) s += s_red[w][kp];
            const double m = (s > 0.f) ? static_cast<double>(ct[kp]) + rmax + log(static_cast<double>(s))
                                       : -__builtin_inf();
            msg[(g * T + t) * K + kp] = m;
            const double u_prev = ut[(g * T + t - 1) * K + kp];
            s_f[kp] = static_cast<float>(u_prev + ct[kp]);
            ut[(g * T + t - 1) * K + kp] = u_prev + m;
        }
        __syncthreads();
        if (t == 1) break;
        // carried matrix of step t-1: rows scaled by exp(ut_{t-1} + c_t - mu), columns renormalised
        if (wave == 0) {
            float mx = -__builtin_inff();
            for (int e = l; e < K; e += 64) mx = fmaxf(mx, s_f[e]);
            mx = group_max(mx, 64);
            if (l == 0) s_scal[1] = mx;
        }
        __syncthreads();
        const float mu = s_scal[1];
        float cmax0 = 0.f, cmax1 = 0.f;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float f = __expf(s_f[16 * rt + 4 * j + q] - mu);
                acc[rt][0][q] *= f;
                acc[rt][1][q] *= f;
                cmax0 = fmaxf(cmax0, acc[rt][0][q]);
                cmax1 = fmaxf(cmax1, acc[rt][1][q]);
            }
        cmax0 = fmaxf(cmax0, __shfl_xor(cmax0, 16, 64));
        cmax0 = fmaxf(cmax0, __shfl_xor(cmax0, 32, 64));
        cmax1 = fmaxf(cmax1, __shfl_xor(cmax1, 16, 64));
        cmax1 = fmaxf(cmax1, __shfl_xor(cmax1, 32, 64));
        const float inv0 = cmax0 > 0.f ? 1.f / cmax0 : 0.f;
        const float inv1 = cmax1 > 0.f ? 1.f / cmax1 : 0.f;
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                bop[c][0][q] = static_cast<__bf16>(acc[2 * c][0][q] * inv0);
                bop[c][0][4 + q] = static_cast<__bf16>(acc[2 * c + 1][0][q] * inv0);
                bop[c][1][q] = static_cast<__bf16>(acc[2 * c][1][q] * inv1);
                bop[c][1][4 + q] = static_cast<__bf16>(acc[2 * c + 1][1][q] * inv1);
            }
        if (j == 0) {
            s_r[col0] = cmax0 > 0.f ? s_r[col0] + mu + __logf(cmax0) : -__builtin_inff();
            s_r[col1] = cmax1 > 0.f ? s_r[col1] + mu + __logf(cmax1) : -__builtin_inff();
        }
        __syncthreads();
    }
    // root of the series: ut_0 now holds u_0 + m_1
    const double* u0 = ut + g * T * K;
    double mx = -__builtin_inf();
    for (int k = tid; k < K; k += NT) mx = fmax(mx, u0[k]);
    mx = group_max(mx, 64);
    if (l == 0) s_dred[wave] = mx;
    __syncthreads();
    mx = s_dred[0];
    for (int w = 1; w < W; ++w) mx = fmax(mx, s_dred[w]);
    __syncthreads();
    double s = 0.0;
    if (mx != -__builtin_inf())
        for (int k = tid; k < K; k += NT) s += exp(u0[k] - mx);
    s = group_sum(s, 64);
    if (l == 0) s_dred[wave] = s;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int w = 0; w < W; ++w) tot += s_dred[w];
        L[g] = (mx == -__builtin_inf()) ? mx : mx + log(tot);
    }
}

// ------------------------------------------------------------------ weights
// One block per series; LPR = K/8 lanes share a row (8 columns each), row
// groups split kp, reduction over kp through shuffles and LDS.
template <int K>
__global__ void __launch_bounds__(BLOCK) k_chain_bwd_bexp(const __bf16* __restrict__ A, const float* __restrict__ csh,
                                                          const double* __restrict__ ut, const double* __restrict__ msg,
                                                          const double* __restrict__ L, float* __restrict__ w, int T,
                                                          const double* __restrict__ gsc) {
    constexpr int LPR = K / 8;
    constexpr int GROUPS = BLOCK / LPR;
    __shared__ float s_w[K], s_rowc[K];
    __shared__ float s_red[GROUPS][K];
    __shared__ double s_scr[BLOCK / WAVE];
    __shared__ float s_tot;
    const long g = blockIdx.x;
    const int lane = threadIdx.x % LPR, grp = threadIdx.x / LPR;
    const double sc = gsc ? *gsc : 1.0;
    const double Lg = L[g];
    for (int k = threadIdx.x; k < K; k += BLOCK) {
        const float v = static_cast<float>(Lg == -__builtin_inf() ? 0.0 : exp(ut[g * T * K + k] - Lg));
        s_w[k] = v;
        w[g * T * K + k] = static_cast<float>(sc * v);
    }
    __syncthreads();
    for (int t = 1; t < T; ++t) {
        const double* utt = ut + (g * T + t) * K;
        const double sh = finite_or_zero(block_max(utt, K, s_scr));
        const __bf16* At = A + (g * (T - 1) + (t - 1)) * static_cast<long>(K) * K;
        const float* ct = csh + (g * (T - 1) + (t - 1)) * K;
        for (int kp = threadIdx.x; kp < K; kp += BLOCK)
            s_rowc[kp] = static_cast<float>((static_cast<double>(ct[kp]) - msg[(g * T + t) * K + kp] + sh) * LOG2E_F);
        float uc[8], acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            uc[q] = static_cast<float>((utt[lane * 8 + q] - sh) * LOG2E_F);
            acc[q] = 0.f;
        }
        __syncthreads();
        for (int kp = grp; kp < K; kp += GROUPS) {
            const float wk = s_w[kp];
            if (wk > 0.f) {
                const bf16x8 av = __builtin_nontemporal_load(reinterpret_cast<const bf16x8*>(At + static_cast<long>(kp) * K + lane * 8));
                const float rc = s_rowc[kp];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float x = static_cast<float>(av[q]);
                    acc[q] += x > 0.f ? wk * exp2f(__log2f(x) + rc + uc[q]) : 0.f;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) s_red[grp][lane * 8 + q] = acc[q];
        __syncthreads();
        if (threadIdx.x < WAVE) {
            float part = 0.f;
            for (int k = threadIdx.x; k < K; k += WAVE) {
                float s = 0.f;
                for (int gi = 0; gi < GROUPS; ++gi) s += s_red[gi][k];
                s_w[k] = s;
                part += s;
            }
            part = group_sum(part, WAVE);
            if (threadIdx.x == 0) s_tot = part;
        }
        __syncthreads();
        const float inv = s_tot > 0.f ? 1.f / s_tot : 0.f;
        for (int k = threadIdx.x; k < K; k += BLOCK) {
            const float v = s_w[k] * inv;
            s_w[k] = v;
            w[(g * T + t) * K + k] = static_cast<float>(sc * v);
        }
        __syncthreads();
    }
}

template <int K>
hipError_t launch_all(hipStream_t s, int which, const void* z, void* A, float* csh, double* ut, double* msg,
                      double* L, float* w, long G, int T, double a, double b, double var, const double* g) {
    if (which == 0) {
        const double c0 = -0.5 * (LOG_2PI + std::log(var));
        hipLaunchKernelGGL(k_chain_bexp_factors<K>, dim3(G * (T - 1)), dim3(BLOCK), 0, s, (const float*)z, (__bf16*)A,
                           csh, T, (float)a, (float)b, (float)c0, (float)(0.5 / var));
    } else if (which == 1) {
        hipLaunchKernelGGL(k_chain_fold_mfma<K>, dim3(G), dim3(2 * K), 0, s, (const __bf16*)A, (const float*)csh, ut,
                           msg, L, T);
    } else {
        hipLaunchKernelGGL(k_chain_bwd_bexp<K>, dim3(G), dim3(BLOCK), 0, s, (const __bf16*)A, (const float*)csh,
                           (const double*)ut, (const double*)msg, (const double*)L, w, T, g);
    }
    return hipGetLastError();
}

hipError_t dispatch(hipStream_t s, int which, int K, const void* z, void* A, float* csh, double* ut, double* msg,
                    double* L, float* w, long G, int T, double a, double b, double var, const double* g) {
    switch (K) {
        case 64: return launch_all<64>(s, which, z, A, csh, ut, msg, L, w, G, T, a, b, var, g);
        case 128: return launch_all<128>(s, which, z, A, csh, ut, msg, L, w, G, T, a, b, var, g);
        case 256: return launch_all<256>(s, which, z, A, csh, ut, msg, L, w, G, T, a, b, var, g);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool chain_bexp_supported(int K) { return K == 64 || K == 128 || K == 256; }

hipError_t chain_bexp_factors(hipStream_t s, const void* z, void* A, float* csh, long G, int T, int K, double a,
                              double b, double var) {
    return dispatch(s, 0, K, z, A, csh, nullptr, nullptr, nullptr, nullptr, G, T, a, b, var, nullptr);
}

hipError_t chain_bexp_fwd(hipStream_t s, const void* A, const float* csh, double* ut, double* msg, double* L, long G,
                          int T, int K) {
    return dispatch(s, 1, K, nullptr, const_cast<void*>(A), const_cast<float*>(csh), ut, msg, L, nullptr, G, T, 0, 0,
                    1, nullptr);
}

hipError_t chain_bexp_bwd(hipStream_t s, const void* A, const float* csh, const double* ut, const double* msg,
                          const double* L, void* w, long G, int T, int K, const double* g) {
    return dispatch(s, 2, K, nullptr, const_cast<void*>(A), const_cast<float*>(csh), const_cast<double*>(ut),
                    const_cast<double*>(msg), const_cast<double*>(L), static_cast<float*>(w), G, T, 0, 0, 1, g);
}

}  // namespace qemk
