// Chains under a K-sampled scalar parent as exponential GEMMs in FP64 on MFMA.
//
// Series g hangs under the parent instance p(g) with samples beta^kb.  Step t
// of the elimination (t = T-1 .. 1) computes, for every parent sample kb and
// previous-step sample kp,
//   m_t[kb,kp] = LSE_k ( F[kb,kp,k] + ub_t[kb,k] ),
//   F[kb,kp,k] = c0 - hp (x_t^k - a x_{t-1}^kp - c_kb)^2,  c_kb = (1 - a) beta^kb + b,
// with ub_{T-1} = u_{T-1} and ub_{t-1} = u_{t-1} + m_t (the start term joins
// ub_0).  With the samples of each step centered on their midrange
// (xt = x_t - xbar, yt = x_{t-1} - ybar, d_kb = c_kb + a ybar - xbar) the
// exponent splits into three parts:
//   F + ub = C[kb,kp] + A[kb,k] + S[kp,k],
//   C = c0 - hp (a yt_kp + d_kb)^2,  A = ub - hp xt_k (xt_k - 2 d_kb),
//   S = 2 hp a yt_kp xt_k,
// so the sum over k is a GEMM of A' = exp(A - alpha_kb) (alpha the row maximum)
// with S' = exp(S - sigma_kp) (sigma the row maximum, in closed form since S
// is linear in xt):
//   m_t = C + alpha + sigma + log( A' S'^T ).
// Every entry of A' and S' lies in (0, 1], and A' S'^T >= exp(-B) with
// B = |2 hp a| max|yt| range(xt): the k where A' = 1 keeps at least that
// much of S'.  For B <= CHAINP_EXACT_BOUND nothing relevant leaves the FP64
// range; a step with a larger B takes the log-sum-exp over k per entry
// instead (same result, K times the exponentials).  With FP32 samples and
// B <= CHAINP_F32_BOUND the step runs in FP32 (hardware exp2, v_mfma_f32_16x16x4f32):
// the entries that carry the sum stay far above FP32's smallest normal, and
// the messages keep the accuracy of the FP32 path.
//
// The reverse pass, t = 1 .. T-1, is the transposed product:
//   w_t[kb,k] = sum_kp w_{t-1}[kb,kp] exp(F + ub_t - m_t)
//             = A'[kb,k] * ( P S' )[kb,k],   P[kb,kp] = w_{t-1} exp(C + alpha + sigma - m_t),
// with w_0[kb,k] = w_parent[kb] exp(ub_0[kb,k] - L[kb]); it rebuilds ub_t from
// the unary terms and the saved messages, and writes, per block, the sum of
// its rows' weights (the parent samples it covers) for the final sum over kb.
//
// Blocks.  One block per (series, R = 16 RT consecutive parent samples); four
// waves, each owning 16-column tiles of the output.  MFMA 16x16x4 in FP64 and
// FP32: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its four
// results are D[l / 16 + 4 r][l % 16] (FP64) and D[4 (l / 16) + r][l % 16]
// (FP32), r = 0..3.  A' (forward) and P (reverse) are staged in
// LDS in that operand order; S' is evaluated in registers, each entry once
// per block and reused by the RT row tiles.
#include <algorithm>
#include <cmath>

#include "qem_internal.h"
#include "dev_common.h"

namespace qemk {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr double CHAINP_EXACT_BOUND = 600.0;
constexpr double CHAINP_F32_BOUND = 60.0;

// The arithmetic of a step: FP32 GEMM, FP64 GEMM, or the per-entry log-sum-exp.
enum StepTier { TIER_F32 = 0, TIER_F64 = 1, TIER_EXACT = 2 };

// exp(x) in the FP32 tier: the hardware exp2 of x log2(e), scaled in FP64 and
// rounded to FP32 as expf rounds its argument.  The tier's range bound keeps
// the exponents below overflow; an entry that underflows is below 2^-126 of
// its row's maximum.
__device__ __forceinline__ float ex32(double x) {
    return __builtin_amdgcn_exp2f(static_cast<float>(x * 1.4426950408889634));
}

// The row of the output tile that result r of a lane in column group q holds.
__device__ __forceinline__ int tile_row(bool f32, int q, int r) { return f32 ? 4 * q + r : q + 4 * r; }
constexpr double LOG_2PI = 1.8378770664093454835606594728112;

// Row tiles per block: one.  Two (each S' entry reused twice) halve the
// blocks, and with a few hundred series the chip is short of blocks, not of
// arithmetic (92 series, K = 64: 0.41 ms forward with one, 0.51 ms with two).
template <int K> struct ChainpShape {
    static constexpr int RT = 1;
    static constexpr int R = 16 * RT;
    static constexpr int NB = K / R;
};

// A barrier that orders LDS accesses only: global stores still in flight do
// not hold it up (no other wave of the block reads them).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The samples of one step, read by wave 0 ahead of their use.
template <int K> constexpr int row_per_lane() { return (K + WAVE - 1) / WAVE; }

template <typename T, int K>
__device__ __forceinline__ void load_row(const T* __restrict__ zrow, double (&v)[row_per_lane<K>()]) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int q = 0; q < row_per_lane<K>(); ++q) {
        const int k = lane + q * WAVE;
        v[q] = k < K ? static_cast<double>(zrow[k]) : 0.0;
    }
}

// Wave 0 centers the K samples of one step on their midrange: c[k] = x_k - mid,
// st = {mid, min c, max c}.
template <int K>
__device__ __forceinline__ void center_row(const double (&v)[row_per_lane<K>()], double* __restrict__ c,
                                           double* __restrict__ st) {
    constexpr int PER = row_per_lane<K>();
    const int lane = threadIdx.x & (WAVE - 1);
    double mn = __builtin_inf(), mx = -__builtin_inf();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int k = lane + q * WAVE;
        if (k < K) { mn = fmin(mn, v[q]); mx = fmax(mx, v[q]); }
    }
    mn = -group_max(-mn, WAVE);
    mx = group_max(mx, WAVE);
    const double mid = 0.5 * (mn + mx);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int k = lane + q * WAVE;
        if (k < K) c[k] = v[q] - mid;
    }
    if (lane == 0) { st[0] = mid; st[1] = mn - mid; st[2] = mx - mid; }
}

// The tier of a step from the bound B of its centered sample ranges (a NaN
// bound selects the per-entry path).
__device__ __forceinline__ int step_tier(bool f32_ok, double s2, const double* sx, const double* sy) {
    const double bound = fabs(s2) * fmax(-sy[1], sy[2]) * (sx[2] - sx[1]);
    if (f32_ok && bound <= CHAINP_F32_BOUND) return TIER_F32;
    return bound <= CHAINP_EXACT_BOUND ? TIER_F64 : TIER_EXACT;
}

__device__ __forceinline__ double sigma_of(double sy, const double* sx) { return sy >= 0.0 ? sy * sx[2] : sy * sx[1]; }

template <typename T, int K>
__global__ void __launch_bounds__(BLOCK) k_chainp_fwd_mfma(const T* __restrict__ z, const double* __restrict__ usrc,
                                                           const T* __restrict__ zb, const int32_t* __restrict__ sp,
                                                           double* __restrict__ m, double* __restrict__ L, int T_,
                                                           double a, double b, double c0, double hp, double ib,
                                                           double ic0, double ihp) {
    constexpr int RT = ChainpShape<K>::RT, R = ChainpShape<K>::R, NB = ChainpShape<K>::NB;
    constexpr int KP = K + 1;
    constexpr int CPL = K / 16;
    __shared__ double s_ub[2][R][KP];
    constexpr bool F32 = sizeof(T) == 4;
    __shared__ double s_A[RT][K / 4][WAVE];
    __shared__ float s_Af[F32 ? RT : 1][F32 ? K / 4 : 1][WAVE];
    __shared__ double s_c[3][K];
    __shared__ double s_st[3][3];
    __shared__ double s_alpha[R], s_d[R], s_cb[R], s_beta[R];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
    const int rg = tid / 16, l16 = tid & 15;
    const long g = blockIdx.x / NB;
    const int kb0 = static_cast<int>(blockIdx.x % NB) * R;
    const double s2 = 2.0 * hp * a;
    const T* zg = z + g * T_ * K;
    const double* ug = usrc + g * T_ * K;
    if (tid < R) {
        const double beta = static_cast<double>(zb[static_cast<long>(sp[g]) * K + kb0 + tid]);
        s_beta[tid] = beta;
        s_cb[tid] = b + (1.0 - a) * beta;
    }
    for (int e = tid; e < R * K; e += BLOCK) s_ub[(T_ - 1) & 1][e / K][e % K] = ug[(T_ - 1) * K + e % K];
    if (wave == 0) {
        double v[row_per_lane<K>()];
        load_row<T, K>(zg + (T_ - 1) * K, v);
        center_row<K>(v, s_c[(T_ - 1) % 3], s_st[(T_ - 1) % 3]);
        load_row<T, K>(zg + (T_ - 2) * K, v);
        center_row<K>(v, s_c[(T_ - 2) % 3], s_st[(T_ - 2) % 3]);
    }
    __syncthreads();
    constexpr int JW = (K / 16 + BLOCK / WAVE - 1) / (BLOCK / WAVE);   // column tiles per wave
    for (int t = T_ - 1; t >= 1; --t) {
        const int cb = t & 1, nb = cb ^ 1;
        // global rows this step consumes late, requested first: the samples of
        // step t-2 (wave 0) and the unary terms of step t-1 at this lane's columns
        double zpre[row_per_lane<K>()];
        if (wave == 0 && t >= 2) load_row<T, K>(zg + (t - 2) * K, zpre);
        double upre[JW];
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
            const int jt = wave + jj * (BLOCK / WAVE);
            upre[jj] = jt < K / 16 ? ug[(t - 1) * K + jt * 16 + (lane & 15)] : 0.0;
        }
        const double* xc = s_c[t % 3];
        const double* yc = s_c[(t - 1) % 3];
        const double* sx = s_st[t % 3];
        const double* sy = s_st[(t - 1) % 3];
        const int tier = step_tier(F32, s2, sx, sy);
        const bool exact = tier == TIER_EXACT, t32 = tier == TIER_F32;
        // A = ub - hp xt (xt - 2 d), its row maximum, and A' = exp(A - alpha)
#pragma unroll
        for (int p = 0; p < RT; ++p) {
            const int i = p * 16 + rg;
            const double d = s_cb[i] + a * sy[0] - sx[0];
            double av[CPL];
            double mx = -__builtin_inf();
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                const int k = l16 + 16 * q;
                const double x = xc[k];
                av[q] = s_ub[cb][i][k] - hp * x * (x - 2.0 * d);
                mx = fmax(mx, av[q]);
            }
            mx = group_max(mx, 16);
            if (l16 == 0) { s_alpha[i] = mx; s_d[i] = d; }
            const double sh = finite_or_zero(mx);
            if (t32) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const int k = l16 + 16 * q;
                    s_Af[F32 ? p : 0][F32 ? k >> 2 : 0][(i & 15) + 16 * (k & 3)] =
                        ex32(av[q] - sh);
                }
            } else if (!exact) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const int k = l16 + 16 * q;
                    s_A[p][k >> 2][(i & 15) + 16 * (k & 3)] = exp(av[q] - sh);
                }
            }
        }
        lds_barrier();
        // m_t = C + alpha + sigma + log(A' S'^T), 16 columns kp per tile
        const int kq = lane >> 4;
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
            const int jt = wave + jj * (BLOCK / WAVE);
            if (jt >= K / 16) continue;
            const int kp = jt * 16 + (lane & 15);
            const double yk = yc[kp];
            const double sy2 = s2 * yk;
            const double sig = sigma_of(sy2, sx);
            f64x4 acc[RT];
            f32x4 accf[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                acc[rt] = f64x4{0.0, 0.0, 0.0, 0.0};
                accf[rt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            }
            if (F32 && t32) {
#pragma unroll 4
                for (int kk = 0; kk < K / 4; ++kk) {
                    const float bv = ex32(sy2 * xc[4 * kk + kq] - sig);
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        accf[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(s_Af[F32 ? rt : 0][F32 ? kk : 0][lane], bv,
                                                                        accf[rt], 0, 0, 0);
                }
            } else if (!exact) {
#pragma unroll 4
                for (int kk = 0; kk < K / 4; ++kk) {
                    const double bv = exp(sy2 * xc[4 * kk + kq] - sig);
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(s_A[rt][kk][lane], bv, acc[rt], 0, 0, 0);
                }
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = rt * 16 + tile_row(t32, kq, r);
                    const double d = s_d[i];
                    double mv;
                    if (!exact) {
                        const double gs = t32 ? static_cast<double>(accf[rt][r]) : acc[rt][r];
                        const double e = a * yk + d;
                        const double lg = t32 ? static_cast<double>(logf(static_cast<float>(gs))) : log(gs);
                        mv = gs > 0.0 ? (c0 - hp * e * e) + finite_or_zero(s_alpha[i]) + sig + lg
                                      : -__builtin_inf();
                    } else {
                        const double mu = a * yk + d;
                        double mx = -__builtin_inf();
                        for (int k = 0; k < K; ++k) {
                            const double dx = xc[k] - mu;
                            mx = fmax(mx, c0 - hp * dx * dx + s_ub[cb][i][k]);
                        }
                        double s = 0.0;
                        if (mx != -__builtin_inf())
                            for (int k = 0; k < K; ++k) {
                                const double dx = xc[k] - mu;
                                s += exp(c0 - hp * dx * dx + s_ub[cb][i][k] - mx);
                            }
                        mv = mx == -__builtin_inf() ? mx : mx + log(s);
                    }
                    m[((g * K + kb0 + i) * T_ + t) * K + kp] = mv;
                    s_ub[nb][i][kp] = upre[jj] + mv;
                }
            }
        }
        // the samples of step t-2, centered for the step after next
        if (wave == 0 && t >= 2) center_row<K>(zpre, s_c[(t - 2) % 3], s_st[(t - 2) % 3]);
        lds_barrier();
    }
    // ub_0 = (u_0 + m_1) + log N(x_0; beta + ib, var0); L = LSE_k ub_0
#pragma unroll
    for (int p = 0; p < RT; ++p) {
        const int i = p * 16 + rg;
        const double beta = s_beta[i];
        double v[CPL];
        double mx = -__builtin_inf();
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int k = l16 + 16 * q;
            const double dx = static_cast<double>(zg[k]) - beta - ib;
            v[q] = s_ub[0][i][k] + (ic0 - ihp * dx * dx);
            mx = fmax(mx, v[q]);
        }
        mx = group_max(mx, 16);
        double s = 0.0;
        if (mx != -__builtin_inf())
#pragma unroll
            for (int q = 0; q < CPL; ++q) s += exp(v[q] - mx);
        s = group_sum(s, 16);
        if (l16 == 0) L[g * K + kb0 + i] = mx == -__builtin_inf() ? mx : mx + log(s);
    }
}

template <typename T, int K>
__global__ void __launch_bounds__(BLOCK) k_chainp_bwd_mfma(const T* __restrict__ z, const double* __restrict__ usrc,
                                                           const T* __restrict__ zb, const T* __restrict__ wb,
                                                           const int32_t* __restrict__ sp, const double* __restrict__ m,
                                                           const double* __restrict__ L, double* __restrict__ part,
                                                           int T_, double a, double b, double c0, double hp, double ib,
                                                           double ic0, double ihp) {
    constexpr int RT = ChainpShape<K>::RT, R = ChainpShape<K>::R, NB = ChainpShape<K>::NB;
    constexpr int KP = K + 1;
    constexpr int CPL = K / 16;
    constexpr int JT = (K / 16 + BLOCK / WAVE - 1) / (BLOCK / WAVE);   // column tiles per wave
    __shared__ double s_ub[R][KP];
    __shared__ double s_w[R][KP];
    constexpr bool F32 = sizeof(T) == 4;
    __shared__ double s_P[RT][K / 4][WAVE];
    __shared__ float s_Pf[F32 ? RT : 1][F32 ? K / 4 : 1][WAVE];
    __shared__ double s_c[3][K];
    __shared__ double s_st[3][3];
    __shared__ double s_alpha[R], s_d[R], s_cb[R], s_beta[R], s_wp[R];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
    const int rg = tid / 16, l16 = tid & 15;
    const long g = blockIdx.x / NB;
    const int bt = static_cast<int>(blockIdx.x % NB);
    const int kb0 = bt * R;
    const double s2 = 2.0 * hp * a;
    const T* zg = z + g * T_ * K;
    const double* ug = usrc + g * T_ * K;
    const double* mg = m + (g * K + kb0) * T_ * K;   // rows of this block: [R, T, K]
    double* pg = part + (g * NB + bt) * T_ * K;
    if (tid < R) {
        const long pb = static_cast<long>(sp[g]) * K + kb0 + tid;
        const double beta = static_cast<double>(zb[pb]);
        s_beta[tid] = beta;
        s_cb[tid] = b + (1.0 - a) * beta;
        s_wp[tid] = static_cast<double>(wb[pb]);
    }
    if (wave == 0) {
        double v[row_per_lane<K>()];
        load_row<T, K>(zg, v);
        center_row<K>(v, s_c[0], s_st[0]);
        load_row<T, K>(zg + K, v);
        center_row<K>(v, s_c[1], s_st[1]);
    }
    // the message rows each step reads, held in registers at the rows and
    // columns this thread covers: mP = m_t (step t's P), mA = m_{t+1} (step
    // t's u-tilde), uA = u_t; the next step's rows are requested a step ahead
    double mP[RT][CPL], mA[RT][CPL], uA[CPL];
#pragma unroll
    for (int p = 0; p < RT; ++p)
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const long row = static_cast<long>(p * 16 + rg) * T_;
            mP[p][q] = mg[(row + 1) * K + l16 + 16 * q];
            mA[p][q] = T_ > 2 ? mg[(row + 2) * K + l16 + 16 * q] : 0.0;
        }
#pragma unroll
    for (int q = 0; q < CPL; ++q) uA[q] = ug[K + l16 + 16 * q];
    __syncthreads();
    // w_0 = w_parent exp(ub_0 - L), ub_0 = (u_0 + m_1) + start term
#pragma unroll
    for (int p = 0; p < RT; ++p) {
        const int i = p * 16 + rg;
        const double Li = L[g * K + kb0 + i];
        const double beta = s_beta[i];
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int k = l16 + 16 * q;
            const double dx = static_cast<double>(zg[k]) - beta - ib;
            const double u0 = (ug[k] + mP[p][q]) + (ic0 - ihp * dx * dx);
            s_w[i][k] = Li == -__builtin_inf() ? 0.0 : s_wp[i] * exp(u0 - Li);
        }
    }
    __syncthreads();
    if (tid < K) {
        double acc = 0.0;
        for (int i = 0; i < R; ++i) acc += s_w[i][tid];
        pg[tid] = acc;
    }
    const int cq = lane >> 4;
    for (int t = 1; t < T_; ++t) {
        double mN[RT][CPL], uN[CPL], zpre[row_per_lane<K>()];
#pragma unroll
        for (int p = 0; p < RT; ++p)
#pragma unroll
            for (int q = 0; q < CPL; ++q)
                mN[p][q] = t + 2 < T_ ? mg[(static_cast<long>(p * 16 + rg) * T_ + t + 2) * K + l16 + 16 * q] : 0.0;
#pragma unroll
        for (int q = 0; q < CPL; ++q) uN[q] = t + 1 < T_ ? ug[(t + 1) * K + l16 + 16 * q] : 0.0;
        if (wave == 0 && t + 1 < T_) load_row<T, K>(zg + (t + 1) * K, zpre);
        const double* xc = s_c[t % 3];
        const double* yc = s_c[(t - 1) % 3];
        const double* sx = s_st[t % 3];
        const double* sy = s_st[(t - 1) % 3];
        const int tier = step_tier(F32, s2, sx, sy);
        const bool exact = tier == TIER_EXACT, t32 = tier == TIER_F32;
        // ub_t = u_t + m_{t+1}, A and its row maximum
#pragma unroll
        for (int p = 0; p < RT; ++p) {
            const int i = p * 16 + rg;
            const double d = s_cb[i] + a * sy[0] - sx[0];
            double mx = -__builtin_inf();
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                const int k = l16 + 16 * q;
                const double ub = uA[q] + (t < T_ - 1 ? mA[p][q] : 0.0);
                s_ub[i][k] = ub;
                const double x = xc[k];
                mx = fmax(mx, ub - hp * x * (x - 2.0 * d));
            }
            mx = group_max(mx, 16);
            if (l16 == 0) { s_alpha[i] = mx; s_d[i] = d; }
        }
        lds_barrier();
        // P = w_{t-1} exp(C + alpha + sigma - m_t)
        if (!exact) {
#pragma unroll
            for (int p = 0; p < RT; ++p) {
                const int i = p * 16 + rg;
                const double al = finite_or_zero(s_alpha[i]);
                const double d = s_d[i];
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const int kp = l16 + 16 * q;
                    const double yk = yc[kp];
                    const double e = a * yk + d;
                    const double mt = mP[p][q];
                    const double wv = s_w[i][kp];
                    const bool live = wv > 0.0 && mt != -__builtin_inf();
                    const double arg = (c0 - hp * e * e) + al + sigma_of(s2 * yk, sx) - mt;
                    if (t32)
                        s_Pf[F32 ? p : 0][F32 ? kp >> 2 : 0][(i & 15) + 16 * (kp & 3)] =
                            live ? static_cast<float>(wv) * ex32(arg) : 0.0f;
                    else
                        s_P[p][kp >> 2][(i & 15) + 16 * (kp & 3)] = live ? wv * exp(arg) : 0.0;
                }
            }
        }
        lds_barrier();
        // w_t = A' (P S'), and the sum of this block's rows per column
        double wout[JT][RT][4];
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) {
            const int jt = wave + jj * (BLOCK / WAVE);
            if (jt >= K / 16) continue;
            const int k = jt * 16 + (lane & 15);
            const double x = xc[k];
            f64x4 acc[RT];
            f32x4 accf[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                acc[rt] = f64x4{0.0, 0.0, 0.0, 0.0};
                accf[rt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            }
            if (F32 && t32) {
#pragma unroll 4
                for (int kk = 0; kk < K / 4; ++kk) {
                    const double sy2 = s2 * yc[4 * kk + cq];
                    const float bv = ex32(sy2 * x - sigma_of(sy2, sx));
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        accf[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(s_Pf[F32 ? rt : 0][F32 ? kk : 0][lane], bv,
                                                                        accf[rt], 0, 0, 0);
                }
            } else if (!exact) {
#pragma unroll 4
                for (int kk = 0; kk < K / 4; ++kk) {
                    const double sy2 = s2 * yc[4 * kk + cq];
                    const double bv = exp(sy2 * x - sigma_of(sy2, sx));
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(s_P[rt][kk][lane], bv, acc[rt], 0, 0, 0);
                }
            }
            double colsum = 0.0;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                double ts = 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = rt * 16 + tile_row(t32, cq, r);
                    const double d = s_d[i];
                    const double ub = s_ub[i][k];
                    const double arg = ub - hp * x * (x - 2.0 * d) - finite_or_zero(s_alpha[i]);
                    double wv;
                    if (t32) {
                        wv = static_cast<double>(accf[rt][r] * ex32(arg));
                    } else if (!exact) {
                        wv = acc[rt][r] * exp(arg);
                    } else {
                        wv = 0.0;
                        for (int kp = 0; kp < K; ++kp) {
                            const double wp = s_w[i][kp];
                            const double mt = mg[(static_cast<long>(i) * T_ + t) * K + kp];
                            if (wp > 0.0 && mt != -__builtin_inf()) {
                                const double dx = x - (a * yc[kp] + d);
                                wv = fma(wp, exp(c0 - hp * dx * dx + ub - mt), wv);
                            }
                        }
                    }
                    wout[jj][rt][r] = wv;
                    ts += wv;
                }
                ts += __shfl_xor(ts, 16, WAVE);
                ts += __shfl_xor(ts, 32, WAVE);
                colsum += ts;
            }
            if (cq == 0) pg[t * K + k] = colsum;
        }
        // the samples of step t+1, centered for the next step
        if (wave == 0 && t + 1 < T_) center_row<K>(zpre, s_c[(t + 1) % 3], s_st[(t + 1) % 3]);
        lds_barrier();
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) {
            const int jt = wave + jj * (BLOCK / WAVE);
            if (jt >= K / 16) continue;
            const int k = jt * 16 + (lane & 15);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) s_w[rt * 16 + tile_row(t32, cq, r)][k] = wout[jj][rt][r];
        }
#pragma unroll
        for (int p = 0; p < RT; ++p)
#pragma unroll
            for (int q = 0; q < CPL; ++q) { mP[p][q] = mA[p][q]; mA[p][q] = mN[p][q]; }
#pragma unroll
        for (int q = 0; q < CPL; ++q) uA[q] = uN[q];
    }
}

template <int K>
hipError_t launch_fwd(hipStream_t s, bool f64, const void* z, const double* usrc, const void* zb, const int32_t* sp,
                      double* m, double* L, long G, int T, double a, double b, double c0, double hp, double ib,
                      double ic0, double ihp) {
    const dim3 grid(static_cast<unsigned>(G * ChainpShape<K>::NB));
    if (f64)
        hipLaunchKernelGGL((k_chainp_fwd_mfma<double, K>), grid, dim3(BLOCK), 0, s, (const double*)z, usrc,
                           (const double*)zb, sp, m, L, T, a, b, c0, hp, ib, ic0, ihp);
    else
        hipLaunchKernelGGL((k_chainp_fwd_mfma<float, K>), grid, dim3(BLOCK), 0, s, (const float*)z, usrc,
                           (const float*)zb, sp, m, L, T, a, b, c0, hp, ib, ic0, ihp);
    return hipGetLastError();
}

template <int K>
hipError_t launch_bwd(hipStream_t s, bool f64, const void* z, const double* usrc, const void* zb, const void* wb,
                      const int32_t* sp, const double* m, const double* L, double* part, long G, int T, double a,
                      double b, double c0, double hp, double ib, double ic0, double ihp) {
    const dim3 grid(static_cast<unsigned>(G * ChainpShape<K>::NB));
    if (f64)
        hipLaunchKernelGGL((k_chainp_bwd_mfma<double, K>), grid, dim3(BLOCK), 0, s, (const double*)z, usrc,
                           (const double*)zb, (const double*)wb, sp, m, L, part, T, a, b, c0, hp, ib, ic0, ihp);
    else
        hipLaunchKernelGGL((k_chainp_bwd_mfma<float, K>), grid, dim3(BLOCK), 0, s, (const float*)z, usrc,
                           (const float*)zb, (const float*)wb, sp, m, L, part, T, a, b, c0, hp, ib, ic0, ihp);
    return hipGetLastError();
}

}  // namespace

bool chainp_mfma_supported(int K) { return K == 16 || K == 32 || K == 64 || K == 128; }

int chainp_mfma_blocks(int K) {
    switch (K) {
        case 16: return ChainpShape<16>::NB;
        case 32: return ChainpShape<32>::NB;
        case 64: return ChainpShape<64>::NB;
        case 128: return ChainpShape<128>::NB;
        default: return 0;
    }
}

hipError_t chainp_fwd_mfma(hipStream_t s, bool f64, const void* z, const double* usrc, const void* zb,
                           const int32_t* sp, double* m, double* L, long G, int T, int K, double a, double b,
                           double var, double ib, double var0) {
    const double c0 = -0.5 * (LOG_2PI + std::log(var)), hp = 0.5 / var;
    const double ic0 = -0.5 * (LOG_2PI + std::log(var0)), ihp = 0.5 / var0;
    switch (K) {
        case 16: return launch_fwd<16>(s, f64, z, usrc, zb, sp, m, L, G, T, a, b, c0, hp, ib, ic0, ihp);
        case 32: return launch_fwd<32>(s, f64, z, usrc, zb, sp, m, L, G, T, a, b, c0, hp, ib, ic0, ihp);
        case 64: return launch_fwd<64>(s, f64, z, usrc, zb, sp, m, L, G, T, a, b, c0, hp, ib, ic0, ihp);
        case 128: return launch_fwd<128>(s, f64, z, usrc, zb, sp, m, L, G, T, a, b, c0, hp, ib, ic0, ihp);
        default: return hipErrorInvalidValue;
    }
}

hipError_t chainp_bwd_mfma(hipStream_t s, bool f64, const void* z, const double* usrc, const void* zb, const void* wb,
                           const int32_t* sp, const double* m, const double* L, double* part, long G, int T, int K,
                           double a, double b, double var, double ib, double var0) {
    const double c0 = -0.5 * (LOG_2PI + std::log(var)), hp = 0.5 / var;
    const double ic0 = -0.5 * (LOG_2PI + std::log(var0)), ihp = 0.5 / var0;
    switch (K) {
        case 16: return launch_bwd<16>(s, f64, z, usrc, zb, wb, sp, m, L, part, G, T, a, b, c0, hp, ib, ic0, ihp);
        case 32: return launch_bwd<32>(s, f64, z, usrc, zb, wb, sp, m, L, part, G, T, a, b, c0, hp, ib, ic0, ihp);
        case 64: return launch_bwd<64>(s, f64, z, usrc, zb, wb, sp, m, L, part, G, T, a, b, c0, hp, ib, ic0, ihp);
        case 128: return launch_bwd<128>(s, f64, z, usrc, zb, wb, sp, m, L, part, G, T, a, b, c0, hp, ib, ic0, ihp);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qemk
