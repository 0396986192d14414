// Chains in BF16-exp mode: the K x K log-semiring products along a series run
// as max-shifted exponential GEMMs in BF16 on MFMA with FP32 accumulation.
//
// Factors.  For step t of series g:  F_t[kp,k] = log N(z_t^k; a z_{t-1}^kp + b, var),
// used as  A_t[kp,k] = bf16(exp(F_t[kp,k] - c_t[kp]))  with the FP32 row
// shift c_t[kp] = max_k F_t[kp,k], so every entry lies in [0, 1].  The fold
// forms each 16-row tile of A_t from the step's samples where it multiplies
// it: no factor tensor is stored.
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
// The reverse pass (marginal weights) is the FP32 chain kernel with the
// factors in FP32 and these messages, its weights renormalised to sum to one
// at every step (chain_bwd_pn with renorm).
#include <algorithm>

#include "qem_internal.h"
#include "dev_common.h"

namespace qemk {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr double LOG_2PI = 1.8378770664093454835606594728112;

// ------------------------------------------------------------------ MFMA fold
// One workgroup of 2K threads per series.  Per step the means a z_{t-1}^kp + b
// and the row shifts c_t[kp] = max_k F_t[kp,k] = c0 - hp min_k (z_k - mean)^2
// (two threads per row) go to LDS, then the workgroup forms the whole tile
// A_t = bf16(exp(F_t - c_t)) in LDS in two halves of K/2 rows (each thread 8
// columns of a row per pass, its 8 samples z_t held in registers for the
// step, F_t = c0 - hp (z - mean)^2 in base 2): the second half is formed
// while the first half's MFMAs run, with one barrier between them.

template <int K>
__global__ void __launch_bounds__(2 * K) k_chain_fold_gen(const float* __restrict__ z, double* __restrict__ ut,
                                                          double* __restrict__ msg, double* __restrict__ L, int T,
                                                          float a, float b, float c0, float hp) {
    constexpr int W = K / 32;
    constexpr int RT = K / 16;
    constexpr int NC = K / 32;
    constexpr int NT = 64 * W;
    constexpr int LDA = K + 8;
    constexpr int CPR = K / 8;         // threads per row of a formed tile (8 entries each)
    constexpr int RPP = NT / CPR;      // rows formed per pass (16)
    __shared__ __bf16 s_a[K * LDA];
    __shared__ float s_r[K];
    __shared__ float s_f[K];
    __shared__ float s_red[W][K];
    __shared__ float s_scal[2];
    __shared__ __align__(16) float s_z[K];
    __shared__ float s_mu[K], s_c[K];
    __shared__ double s_dred[NT / 64];
    const int tid = threadIdx.x, wave = tid / 64, l = tid % 64, j = l / 16, li = l % 16;
    const long g = blockIdx.x;
    const int col0 = wave * 32 + li, col1 = wave * 32 + 16 + li;
    const int grow = tid / CPR, gc8 = tid % CPR;   // the row within a pass and the 8-column slice of this thread
    const float hp2 = hp * 1.44269504088896341f;

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

    // rows [r0, r0 + K/2) of A_t into LDS: RPP rows per pass
    auto form_half = [&](int r0, const float (&zr)[8]) {
#pragma unroll 2
        for (int p = 0; p < K / 2 / RPP; ++p) {
            const int kp = r0 + p * RPP + grow;
            // exp(F - c) = 2^((c0 - c) log2 e - hp log2 e (z - mean)^2): one
            // multiply, one fused multiply-add and the hardware exp2 per entry
            const float mean = s_mu[kp], crow = (c0 - s_c[kp]) * 1.44269504088896341f;
            bf16x8 v;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float e = zr[q] - mean;
                v[q] = static_cast<__bf16>(__builtin_amdgcn_exp2f(fmaf(-(hp2 * e), e, crow)));
            }
            *reinterpret_cast<bf16x8*>(s_a + kp * LDA + gc8 * 8) = v;
        }
    };
    f32x4 acc[RT][2];
    // the MFMAs of row tiles [rt0, rt0 + RT/2)
    auto mma_half = [&](int rt0) {
#pragma unroll
        for (int rr = 0; rr < RT / 2; ++rr) {
            const int rt = rt0 + rr;
            const __bf16* sa = s_a + 16 * rt * LDA;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const bf16x4 lo = *reinterpret_cast<const bf16x4*>(sa + li * LDA + 32 * c + 4 * j);
                const bf16x4 hi = *reinterpret_cast<const bf16x4*>(sa + li * LDA + 32 * c + 16 + 4 * j);
                const bf16x8 av = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                acc[rt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[c][0], acc[rt][0], 0, 0, 0);
                acc[rt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bop[c][1], acc[rt][1], 0, 0, 0);
            }
        }
    };

    for (int t = T - 1; t >= 1; --t) {
        for (int e = tid; e < K; e += NT) {
            s_z[e] = z[(g * T + t) * K + e];
            s_mu[e] = a * z[(g * T + t - 1) * K + e] + b;
        }
        __syncthreads();
        {   // row shifts: two threads per row (NT = 2 K), each over half of the columns
            const int kp = tid >> 1, h = tid & 1;
            // the row's largest factor is at its nearest sample: c0 - hp min_k (z_k - mean)^2
            const float mean = s_mu[kp];
            const float4* zz = reinterpret_cast<const float4*>(s_z + h * (K / 2));
            float mn = __builtin_inff();
#pragma unroll 8
            for (int k4 = 0; k4 < K / 8; ++k4) {
                const float4 v = zz[k4];
                const float d0 = v.x - mean, d1 = v.y - mean, d2 = v.z - mean, d3 = v.w - mean;
                mn = fminf(mn, d0 * d0);
                mn = fminf(mn, d1 * d1);
                mn = fminf(mn, d2 * d2);
                mn = fminf(mn, d3 * d3);
            }
            mn = fminf(mn, __shfl_xor(mn, 1, 64));
            if (h == 0) s_c[kp] = c0 - hp * mn;
        }
        float zr[8];
        {
            const float4 z0 = *reinterpret_cast<const float4*>(s_z + gc8 * 8);
            const float4 z1 = *reinterpret_cast<const float4*>(s_z + gc8 * 8 + 4);
            zr[0] = z0.x; zr[1] = z0.y; zr[2] = z0.z; zr[3] = z0.w;
            zr[4] = z1.x; zr[5] = z1.y; zr[6] = z1.z; zr[7] = z1.w;
        }
        __syncthreads();
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            acc[rt][0] = f32x4{0.f, 0.f, 0.f, 0.f};
            acc[rt][1] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        form_half(0, zr);
        __syncthreads();
        mma_half(0);
        form_half(K / 2, zr);   // issued while the first half's products run
        __syncthreads();
        mma_half(RT / 2);
        __syncthreads();
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
            float sm = 0.f;
#pragma unroll
            for (int w = 0; w < W; ++w) sm += s_red[w][kp];
            const double m = (sm > 0.f) ? static_cast<double>(s_c[kp]) + rmax + log(static_cast<double>(sm))
                                        : -__builtin_inf();
            msg[(g * T + t) * K + kp] = m;
            const double u_prev = ut[(g * T + t - 1) * K + kp];
            s_f[kp] = static_cast<float>(u_prev + s_c[kp]);
            ut[(g * T + t - 1) * K + kp] = u_prev + m;
        }
        __syncthreads();
        if (t == 1) break;
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
    const double* u0 = ut + g * T * K;
    double mx = -__builtin_inf();
    for (int k = tid; k < K; k += NT) mx = fmax(mx, u0[k]);
    mx = group_max(mx, 64);
    if (l == 0) s_dred[wave] = mx;
    __syncthreads();
    mx = s_dred[0];
    for (int w = 1; w < W; ++w) mx = fmax(mx, s_dred[w]);
    __syncthreads();
    double sacc = 0.0;
    if (mx != -__builtin_inf())
        for (int k = tid; k < K; k += NT) sacc += exp(u0[k] - mx);
    sacc = group_sum(sacc, 64);
    if (l == 0) s_dred[wave] = sacc;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int w = 0; w < W; ++w) tot += s_dred[w];
        L[g] = (mx == -__builtin_inf()) ? mx : mx + log(tot);
    }
}

template <int K>
hipError_t launch_fold(hipStream_t s, const float* z, double* ut, double* msg, double* L, long G, int T, double a,
                       double b, double var) {
    const double c0 = -0.5 * (LOG_2PI + std::log(var));
    hipLaunchKernelGGL(k_chain_fold_gen<K>, dim3(G), dim3(2 * K), 0, s, z, ut, msg, L, T, (float)a, (float)b,
                       (float)c0, (float)(0.5 / var));
    return hipGetLastError();
}

}  // namespace

bool chain_bexp_supported(int K) { return K == 64 || K == 128 || K == 256; }

hipError_t chain_bexp_fwd(hipStream_t s, const void* z, double* ut, double* msg, double* L, long G, int T, int K,
                          double a, double b, double var) {
    const float* zf = static_cast<const float*>(z);
    switch (K) {
        case 64: return launch_fold<64>(s, zf, ut, msg, L, G, T, a, b, var);
        case 128: return launch_fold<128>(s, zf, ut, msg, L, G, T, a, b, var);
        case 256: return launch_fold<256>(s, zf, ut, msg, L, G, T, a, b, var);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qemk
