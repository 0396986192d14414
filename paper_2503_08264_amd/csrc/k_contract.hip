// Log-space contraction of the MPIW sum over all K^n index tuples (Eq. Prmp)
// by elimination along plates and chains, children first, and the reverse
// pass that gives the marginal weights (the moments of Eq. mmp with an
// indicator; equal to d log P_MP / d u by the source-term identity).
//
//   ut_v[i,k] = u_v[i,k] + sum_{child instances c of i} m_c[c,k]      (FP64)
//   m_v[i,kp] = LSE_k (F_v[i,kp,k] + ut_v[i,k])                       (plate forward)
//   w_v[i,k]  = sum_kp w_par[p(i),kp] exp(F_v[i,kp,k] + ut_v[i,k] - m_v[i,kp])
//
// ut and the messages m are FP64 in every mode.  Before the FP32 arithmetic
// each instance's ut is shifted by c_i = max_k ut[i,k]; LSE is
// shift-invariant, so only offsets from the dominant sample (not the large
// accumulated log densities of whole sub-trees) are rounded to FP32, the
// entries that carry the weight sit near 0, and m = c_i + LSE is formed in
// FP64.
//
// Plate forward streams F row by row: each row of K entries is read as
// 16-byte vectors by a group of LPR lanes (consecutive groups read
// consecutive rows, so a wave covers one contiguous span), reduced with a
// max then a sum of exponentials by DPP lane moves inside the group.
// Plate backward keeps one instance's Kp x K tile in one workgroup, lanes
// along k and row groups along kp, and reduces over kp through shuffles and
// LDS in a fixed order.  No floating-point atomics anywhere.
#include <algorithm>

#include "qem_internal.h"
#include "dev_common.h"
#include "dev_finish.h"
#include "dev_sample.h"
#include "dev_pair.h"

namespace qemk {

namespace {

// ---------------------------------------------------------------- helpers

struct RowPlan { int vec, lpr, nch; };

int next_pow2(int x) { int p = 1; while (p < x) p <<= 1; return p; }

// Lanes per row and 16-byte vectors per lane for a row of K entries.
RowPlan plan_rows(int K, int elem_bytes) {
    const int full = 16 / elem_bytes;
    const int vec = (K % full == 0) ? full : 1;
    const int nv = (K + vec - 1) / vec;
    int lpr = std::max(std::min(16, next_pow2(nv)), next_pow2((nv + 3) / 4));
    lpr = std::min(lpr, 64);
    int nch = (nv + lpr - 1) / lpr;
    nch = next_pow2(nch);
    return {vec, lpr, nch};
}

// A row of the factor table plus the thread's shifted u-tilde columns utv
// (formed once per step), in the row's lane layout.
template <typename T, int VEC, int NCH>
__device__ __forceinline__ void load_row_plus(const T* __restrict__ row, const T (&utv)[NCH * VEC], int K, int lane,
                                              int lpr, T (&v)[NCH * VEC], bool nt) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int e0 = (c * lpr + lane) * VEC;
        if (e0 < K) {
            T f[VEC];
            load_vec_hint<T, VEC>(row + e0, f, nt);
#pragma unroll
            for (int q = 0; q < VEC; ++q) v[c * VEC + q] = f[q] + utv[c * VEC + q];
        } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) v[c * VEC + q] = neg_inf<T>();
        }
    }
}

// exp(x - m) with the row's shift m formed once (rs = row_shift(m)): in FP32
// the hardware exp2 of one fused multiply-add, x log2 e - m log2 e (one
// operation per entry fewer than subtracting, then scaling inside expf); in
// FP64 exp(x - m).
__device__ __forceinline__ float row_shift(float m) { return -(m * 1.44269504088896341f); }
__device__ __forceinline__ double row_shift(double m) { return m; }
__device__ __forceinline__ float exp_minus(float x, float rs) {
    return __builtin_amdgcn_exp2f(fmaf(x, 1.44269504088896341f, rs));
}
__device__ __forceinline__ double exp_minus(double x, double rs) { return exp(x - rs); }

template <typename T, int N>
__device__ __forceinline__ T lse_group(const T (&v)[N], int lpr) {
    T mx = v[0];
#pragma unroll
    for (int q = 1; q < N; ++q) mx = fmax(mx, v[q]);
    mx = group_max(mx, lpr);
    if (mx == neg_inf<T>()) return mx;   // uniform across the group
    const T rs = row_shift(mx);
    T s = 0;
#pragma unroll
    for (int q = 0; q < N; ++q) s += exp_minus(v[q], rs);
    s = group_sum(s, lpr);
    return mx + flog(s);
}

// Log-sum-exp of a row whose entries do not exceed U: a linear-Gaussian
// chain step, F = c0 - hp (z - mean)^2 <= c0 and u-tilde minus its maximum
// <= 0, so U = c0 bounds every entry.  The exponentials are taken against U
// and no row maximum is formed.  A row whose sum falls below lse_small (all
// of its entries so far below U that the small ones would leave the format's
// normal range) is redone against its maximum; the sum is the same in every
// lane of the row group, so each group takes one branch.
__device__ __forceinline__ constexpr float lse_small(float) { return 0x1p-80f; }
__device__ __forceinline__ constexpr double lse_small(double) { return 0x1p-900; }

template <typename T, int N>
__device__ __forceinline__ T lse_group_bounded(const T (&v)[N], int lpr, T U) {
    const T rs = row_shift(U);
    T s = 0;
#pragma unroll
    for (int q = 0; q < N; ++q) s += exp_minus(v[q], rs);
    s = group_sum(s, lpr);
    if (s >= lse_small(T(0))) return U + flog(s);
    return lse_group<T, N>(v, lpr);
}

// ---------------------------------------------------------------- kernels

// A node without children: ut = u in FP64.
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_ut_from_u(double* __restrict__ ut, const T* __restrict__ u, long total) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < total) ut[t] = static_cast<double>(u[t]);
}

// Parents with children: one workgroup of CS_BLOCK threads per parent
// instance; ut[q,:] = base[q,:] + the messages of up to MAX_CHILD_LISTS child
// lists, in the order block_gather fixes.
constexpr int CS_BLOCK = 1024;

template <typename T>
__global__ void __launch_bounds__(CS_BLOCK) k_gather(double* __restrict__ ut, const T* __restrict__ u, ChildLists cl,
                                                     int K) {
    __shared__ double s_ut[512];
    __shared__ double red[1024];
    __shared__ int32_t s_idx[1024];
    const long q = blockIdx.x;
    if (u) block_gather(s_ut, u, cl, q, K, red, s_idx);
    else block_gather(s_ut, static_cast<const double*>(ut), cl, q, K, red, s_idx);
    for (int k = threadIdx.x; k < K; k += CS_BLOCK) ut[q * K + k] = s_ut[k];
}

// A workgroup covers ipb consecutive instances (ipb*Kp rows of F).  It first
// stages each instance's shift c_i = max_k ut[i,k] and ut[i,:] - c_i (in T)
// in LDS; then groups of lpr lanes take RPI rows at a time, loading all of
// them before reducing any.
template <typename T, int VEC, int NCH, int RPI, int LPR>
__global__ void __launch_bounds__(BLOCK) k_plate_fwd(const T* __restrict__ F, const double* __restrict__ ut,
                                                     double* __restrict__ m, long n, int K, int Kp,
                                                     int ipb, int kp_shift, bool nt, uint32_t* __restrict__ status) {
    constexpr int lpr = LPR;
    extern __shared__ unsigned char smem_raw[];
    double* s_sh = reinterpret_cast<double*>(smem_raw);      // [ipb]
    T* s_u = reinterpret_cast<T*>(s_sh + ipb);               // [ipb, K]
    const int lane = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int gpb = BLOCK / lpr;
    const int wl = threadIdx.x & (WAVE - 1);
    const long i0 = static_cast<long>(blockIdx.x) * ipb;
    const int ni = static_cast<int>(std::min(static_cast<long>(ipb), n - i0));
    const int nr = ni * Kp;
    const T* Fb = F + i0 * Kp * K;
    double* mb = m + i0 * Kp;
    T v[RPI][NCH * VEC];
    auto load_pass = [&](int rb0) {
#pragma unroll
        for (int r = 0; r < RPI; ++r) {
            const int row = rb0 + r * gpb + grp;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
                if (row < nr && e0 < K) {
                    T f[VEC];
                    load_vec_hint<T, VEC>(Fb + static_cast<long>(row) * K + e0, f, nt);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) v[r][c * VEC + q] = f[q];
                } else {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) v[r][c * VEC + q] = neg_inf<T>();
                }
            }
        }
    };
    // the first rows are requested before the shifts are staged, so the two
    // memory latencies overlap
    load_pass(0);
    for (int li = threadIdx.x / WAVE; li < ni; li += BLOCK / WAVE) {
        const double* row = ut + (i0 + li) * K;
        double mx = -__builtin_inf();
        for (int k = wl; k < K; k += WAVE) mx = fmax(mx, row[k]);
        mx = group_max(mx, WAVE);
        if (wl == 0) s_sh[li] = finite_or_zero(mx);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ni * K; e += BLOCK) s_u[e] = static_cast<T>(ut[i0 * K + e] - s_sh[e / K]);
    __syncthreads();
    for (int rb0 = 0; rb0 < nr; rb0 += gpb * RPI) {
        if (rb0 > 0) load_pass(rb0);
#pragma unroll
        for (int r = 0; r < RPI; ++r) {
            const int row = rb0 + r * gpb + grp;
            const int rr = row < nr ? row : nr - 1;
            const int li = kp_shift >= 0 ? (rr >> kp_shift) : rr / Kp;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
                if (e0 < K) {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) v[r][c * VEC + q] += s_u[li * K + e0 + q];
                }
            }
            const T res = lse_group<T, NCH * VEC>(v[r], lpr);
            if (lane == 0 && row < nr) {
                mb[row] = (res == neg_inf<T>()) ? -__builtin_inf() : s_sh[li] + static_cast<double>(res);
                if (res == neg_inf<T>()) flag_neg_inf_row(status);
            }
        }
    }
}

// Plate forward with the linear-Gaussian pair table evaluated in place, one
// instance per workgroup: the rows of F are computed from the samples (the
// thread's child-sample columns and its u-tilde columns stay in registers,
// the parent means sit in LDS), written out for the backward pass, and
// reduced exactly as k_plate_fwd reduces the rows it loads (same lanes, same
// order, same shift), so F and m are the same bits as the pair-table kernel
// followed by k_plate_fwd.  One HBM pass over F (the write) replaces two.
// Every global load of the prologue is issued before the first wait; each
// lane group spans a whole row, so the shift max_k ut[i,k] is reduced inside
// the group without a barrier.
// GATHER: the instance's u-tilde is first formed here, u plus its child
// messages in block_gather's order (the bits of k_gather), and written to
// ut for the backward pass; otherwise ut holds it on entry.
template <typename T, int VEC, int NCH, int RPI, int D, int LPR, bool GATHER>
__global__ void __launch_bounds__(BLOCK) k_plate_fwd_pn(T* __restrict__ F, const T* __restrict__ zc,
                                                        const T* __restrict__ zp, const int32_t* __restrict__ pidx,
                                                        double* __restrict__ ut, double* __restrict__ m,
                                                        int K, int Kp, T a, T b, T c0, T hp, bool nt,
                                                        const T* __restrict__ u, ChildLists cl,
                                                        uint32_t* __restrict__ status) {
    constexpr int lpr = LPR;
    constexpr int NV = NCH * VEC;
    constexpr int MP = 4;   // parent-mean entries staged per thread from registers
    extern __shared__ unsigned char smem_raw[];
    T* s_mean = reinterpret_cast<T*>(smem_raw);   // [Kp, D]
    __shared__ double s_g[GATHER ? 512 + 1024 : 1];   // u-tilde row [K], gather partials [1024]
    __shared__ int32_t s_gi[GATHER ? 1024 : 1];        // staged child indices
    const int lane = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int gpb = BLOCK / lpr;
    const long i = blockIdx.x;
    const long pi = pidx ? pidx[i] : 0;
    const double* urow = ut + i * K;
    if constexpr (GATHER) {
        block_gather(s_g, u, cl, i, K, s_g + 512, s_gi);
        for (int k = threadIdx.x; k < K; k += BLOCK) ut[i * K + k] = s_g[k];
        urow = s_g;
    }
    T zr[NV][D];
    double ud[NV];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int e0 = (c * lpr + lane) * VEC;
        const int ec = e0 < K ? e0 : K - VEC;   // in-bounds address for lanes past the row end
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
#pragma unroll
            for (int j = 0; j < D; ++j) zr[c * VEC + q][j] = zc[(i * K + ec + q) * D + j];
            ud[c * VEC + q] = urow[ec + q];
        }
    }
    const int nmean = Kp * D;
    T zpv[MP];
#pragma unroll
    for (int r = 0; r < MP; ++r) {
        const int e = threadIdx.x + r * BLOCK;
        zpv[r] = zp[pi * nmean + (e < nmean ? e : 0)];
    }
    double mx = -__builtin_inf();
#pragma unroll
    for (int c = 0; c < NCH; ++c)
        if ((c * lpr + lane) * VEC < K)
#pragma unroll
            for (int q = 0; q < VEC; ++q) mx = fmax(mx, ud[c * VEC + q]);
    const double sh = finite_or_zero(group_max(mx, lpr));
    T su[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) su[q] = static_cast<T>(ud[q] - sh);
#pragma unroll
    for (int r = 0; r < MP; ++r) {
        const int e = threadIdx.x + r * BLOCK;
        if (e < nmean) s_mean[e] = pair_mean(a, zpv[r], b);
    }
    for (int e = threadIdx.x + MP * BLOCK; e < nmean; e += BLOCK) s_mean[e] = pair_mean(a, zp[pi * nmean + e], b);
    __syncthreads();
    T* Fi = F ? F + i * static_cast<long>(Kp) * K : nullptr;
    for (int rb0 = 0; rb0 < Kp; rb0 += gpb * RPI) {
#pragma unroll
        for (int r = 0; r < RPI; ++r) {
            const int row = rb0 + r * gpb + grp;
            const int rr = row < Kp ? row : Kp - 1;
            T mean[D];
#pragma unroll
            for (int j = 0; j < D; ++j) mean[j] = s_mean[rr * D + j];
            T v[NV];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
                if (e0 < K) {
                    T f[VEC];
#pragma unroll
                    for (int q = 0; q < VEC; ++q) f[q] = normal_pair_value<T, D>(zr[c * VEC + q], mean, D, c0, hp);
                    if (F && row < Kp) store_vec_hint<T, VEC>(Fi + static_cast<long>(row) * K + e0, f, nt);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) v[c * VEC + q] = f[q] + su[c * VEC + q];
                } else {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) v[c * VEC + q] = neg_inf<T>();
                }
            }
            const T res = lse_group<T, NV>(v, lpr);
            if (lane == 0 && row < Kp) {
                m[i * Kp + row] = (res == neg_inf<T>()) ? -__builtin_inf() : sh + static_cast<double>(res);
                if (res == neg_inf<T>()) flag_neg_inf_row(status);
            }
        }
    }
}

// ---------------------------------------------------------------- FP32, K = 64
//
// FP32 plate forward for K = Kp = 64 with one wave per instance: groups of 4
// lanes take whole rows (16 groups, each 4 rows kp = g, g + 16, g + 32,
// g + 48), and a lane holds 16 entries of a row, the float4s at
// k = 16 c + 4 t (c = 0..3, t its place in the group), so each of its four
// 16-byte accesses covers, with the other lanes of its group, 64 contiguous
// bytes of a row.  With 16 entries per lane a row's log-sum-exp needs only
// two cross-lane stages (the lanes-along-k layout of the general kernels
// spends most of its instructions on the DPP max and sum of every row), and
// the child samples a lane needs are loaded once for its four rows.  A row's
// LSE, in this fixed order: the lane's max over its entries, the quad max,
// four interleaved partial sums of exp2((v - max) log2 e) added as
// (s0 + s1) + (s2 + s3), the quad sum, then max + ln 2 log2(sum) (the sum is
// at least 1; hardware exp2 and log2).
constexpr float L2E_F = 1.4426950408889634f;
constexpr float LN2_F = 0.69314718055994531f;
constexpr int Q4_K = 64;     // samples per instance and per parent instance
constexpr int Q4_E = 16;     // entries per lane

__host__ __device__ constexpr bool q4_layout(int K, int Kp) { return K == Q4_K && Kp == Q4_K; }

__device__ __forceinline__ int q4_col(int e, int t) { return (e >> 2) * 16 + t * 4 + (e & 3); }

__device__ __forceinline__ float q4_row_lse(const float (&v)[Q4_E]) {
    float mx = v[0];
#pragma unroll
    for (int q = 1; q < Q4_E; ++q) mx = fmaxf(mx, v[q]);
    mx = group_max(mx, 4);
    if (mx == neg_inf<float>()) return mx;   // uniform across the group
    const float nm = -mx * L2E_F;
    float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < Q4_E; ++q) s[q & 3] += __builtin_amdgcn_exp2f(fmaf(v[q], L2E_F, nm));
    const float t = group_sum((s[0] + s[1]) + (s[2] + s[3]), 4);
    return fmaf(__builtin_amdgcn_logf(t), LN2_F, mx);
}

// The instance's shift max_k ut[i,k] (FP64, reduced inside the group, which
// spans all K) and the lane's shifted u-tilde entries su[e] = ut - shift.
__device__ __forceinline__ double q4_shift(const double* __restrict__ urow, int t, float (&su)[Q4_E]) {
    double ud[Q4_E];
#pragma unroll
    for (int e = 0; e < Q4_E; ++e) ud[e] = urow[q4_col(e, t)];
    double mx = ud[0];
#pragma unroll
    for (int e = 1; e < Q4_E; ++e) mx = fmax(mx, ud[e]);
    const double sh = finite_or_zero(group_max(mx, 4));
#pragma unroll
    for (int e = 0; e < Q4_E; ++e) su[e] = static_cast<float>(ud[e] - sh);
    return sh;
}

// With the linear-Gaussian pair factor evaluated in place (normal_pair_value,
// the function of the pair-table kernels) and, when F is not null, written.
// Without GATHER: four instances per workgroup, one per wave.  With GATHER:
// one instance per workgroup, whose u-tilde the whole workgroup first forms
// from u and its child messages (block_gather's order, the bits of
// k_gather); wave w then takes the rows g + 16 w (a row's sums do not depend
// on which wave forms them).  With SAMPLE (no GATHER), lane k of the wave
// first draws sample k of its instance with its unary factor (the sampling
// kernel's gauss_sample_in_wave, split so that every load is issued before
// the draws), writes z, u and ut = u, and passes the samples and ut to the
// row layout through LDS.
template <int D, bool GATHER, bool SAMPLE>
__global__ void __launch_bounds__(BLOCK) k_plate_fwd_q4_pn(float* __restrict__ F, const float* __restrict__ zc,
                                                           const float* __restrict__ zp,
                                                           const int32_t* __restrict__ pidx,
                                                           double* __restrict__ ut, double* __restrict__ m, long n,
                                                           float a, float b, float c0, float hp, bool nt,
                                                           const float* __restrict__ u, ChildLists cl,
                                                           uint32_t* __restrict__ status, FwdSample fs) {
    constexpr int K = Q4_K;
    static_assert(!(GATHER && SAMPLE), "a gathering forward does not draw samples");
    __shared__ double s_g[GATHER ? 512 + 1024 : 1];
    __shared__ int32_t s_gi[GATHER ? 1024 : 1];
    __shared__ float s_zs[SAMPLE ? BLOCK / WAVE : 1][SAMPLE ? Q4_K * D : 1];
    __shared__ double s_us[SAMPLE ? BLOCK / WAVE : 1][SAMPLE ? Q4_K : 1];
    const int wave = threadIdx.x / WAVE;
    const int wl = threadIdx.x & (WAVE - 1);
    const int g = wl >> 2, t = wl & 3;
    const long i = GATHER ? static_cast<long>(blockIdx.x) : static_cast<long>(blockIdx.x) * (BLOCK / WAVE) + wave;
    const double* urow = ut + i * K;
    if constexpr (!GATHER)
        if (i >= n) return;
    // the rows' parent samples and (unless drawn here) the columns' samples
    // are loaded first, so that their latency overlaps the gather's
    const long pi = pidx ? pidx[i] : 0;
    float zpr[4][D];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (!GATHER || r == wave)
#pragma unroll
            for (int j = 0; j < D; ++j) zpr[r][j] = zp[(pi * K + g + 16 * r) * D + j];
    float zr[Q4_E][D];
    if constexpr (!SAMPLE) {
#pragma unroll
        for (int c = 0; c < Q4_E / 4; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int j = 0; j < D; ++j) zr[c * 4 + q][j] = zc[(i * K + c * 16 + t * 4 + q) * D + j];
    }
    if constexpr (GATHER) {
        block_gather(s_g, u, cl, i, K, s_g + 512, s_gi);
        for (int k = threadIdx.x; k < K; k += BLOCK) ut[i * K + k] = s_g[k];
        urow = s_g;
    }
    if constexpr (SAMPLE) {
        // every load the draws and the rows need issued first: the iteration
        // word, the instance's proposal and observation statistics, the rows'
        // parent samples (below); the draws then overlap their latency
        Stream st = fs.st;
        const uint32_t itd = fs.it_dev ? static_cast<uint32_t>(*fs.it_dev) : st.it;
        const GaussInst<D> gi = gauss_inst_load<D>(fs.a, static_cast<uint32_t>(i));
        st.it = itd ^ fs.it_xor;
        const uint32_t te = static_cast<uint32_t>(i * K + wl);
        float zs[D];
        const float uT = gauss_sample_from<float, D>(fs.a, st, te, gi, zs);
        float* zo = static_cast<float*>(const_cast<void*>(fs.a.z)) + static_cast<size_t>(te) * D;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            zo[j] = zs[j];
            s_zs[wave][wl * D + j] = zs[j];
        }
        static_cast<float*>(fs.a.u)[te] = uT;
        ut[te] = static_cast<double>(uT);
        s_us[wave][wl] = static_cast<double>(uT);
        // only this wave's lanes read what it wrote: LDS accesses of a wave
        // complete in order, the fences keep the compiler from moving them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int c = 0; c < Q4_E / 4; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int j = 0; j < D; ++j) zr[c * 4 + q][j] = s_zs[wave][(c * 16 + t * 4 + q) * D + j];
        urow = s_us[wave];
    }
    float su[Q4_E];
    const double sh = q4_shift(urow, t, su);
    float* Fi = F ? F + i * static_cast<long>(K) * K : nullptr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (GATHER && r != wave) continue;
        const int kp = g + 16 * r;
        float mean[D];
#pragma unroll
        for (int j = 0; j < D; ++j) mean[j] = pair_mean(a, zpr[r][j], b);
        float v[Q4_E];
#pragma unroll
        for (int c = 0; c < Q4_E / 4; ++c) {
            float f[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) f[q] = normal_pair_value<float, D>(zr[c * 4 + q], mean, D, c0, hp);
            if (Fi) store_vec_hint<float, 4>(Fi + kp * K + c * 16 + t * 4, f, nt);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[c * 4 + q] = f[q] + su[c * 4 + q];
        }
        const float res = q4_row_lse(v);
        if (t == 0) {
            m[i * K + kp] = (res == neg_inf<float>()) ? -__builtin_inf() : sh + static_cast<double>(res);
            if (res == neg_inf<float>()) flag_neg_inf_row(status);
        }
    }
}

// Reading a pair table in the same layout and with the same sums as
// k_plate_fwd_q4_pn (same bits).  Four instances per workgroup, one per wave;
// all 16 loads of a lane are issued before the shift is formed.
__global__ void __launch_bounds__(BLOCK) k_plate_fwd_q4(const float* __restrict__ F, const double* __restrict__ ut,
                                                        double* __restrict__ m, long n, bool nt,
                                                        uint32_t* __restrict__ status) {
    constexpr int K = Q4_K;
    const int wave = threadIdx.x / WAVE;
    const int wl = threadIdx.x & (WAVE - 1);
    const int g = wl >> 2, t = wl & 3;
    const long i = static_cast<long>(blockIdx.x) * (BLOCK / WAVE) + wave;
    if (i >= n) return;
    const float* Fi = F + i * static_cast<long>(K) * K;
    float f[4][Q4_E];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < Q4_E / 4; ++c) {
            float fv[4];
            load_vec_hint<float, 4>(Fi + (g + 16 * r) * K + c * 16 + t * 4, fv, nt);
#pragma unroll
            for (int q = 0; q < 4; ++q) f[r][c * 4 + q] = fv[q];
        }
    float su[Q4_E];
    const double sh = q4_shift(ut + i * K, t, su);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float v[Q4_E];
#pragma unroll
        for (int e = 0; e < Q4_E; ++e) v[e] = f[r][e] + su[e];
        const float res = q4_row_lse(v);
        if (t == 0) {
            m[i * K + g + 16 * r] = (res == neg_inf<float>()) ? -__builtin_inf() : sh + static_cast<double>(res);
            if (res == neg_inf<float>()) flag_neg_inf_row(status);
        }
    }
}

// One workgroup per instance; lanes along k, row groups along kp.  All
// global loads of the prologue (the first rows of F, the thread's u-tilde
// columns, the messages and parent weights, the first samples of the fused
// moments) are issued before the first wait; the shift max_k ut[i,k] is
// reduced inside each lane group, which spans a whole row.
template <typename T, int VEC, int NCH, int LPR>
__global__ void __launch_bounds__(BLOCK) k_plate_bwd(const T* __restrict__ F, const double* __restrict__ ut,
                                                     const double* __restrict__ m, const T* __restrict__ wp,
                                                     const int32_t* __restrict__ pidx, T* __restrict__ w,
                                                     int K, int Kp, bool nt, const T* __restrict__ z,
                                                     double* __restrict__ mone, int d) {
    constexpr int lpr = LPR;
    constexpr int NV = NCH * VEC;
    __shared__ T red[BLOCK / WAVE][512];
    __shared__ T s_m[512], s_wp[512], s_w[512];
    const int lane = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int ngrp = BLOCK / lpr;
    const int wave = threadIdx.x / WAVE;
    const int wl = threadIdx.x & (WAVE - 1);
    const long i = blockIdx.x;
    const T* tile = F + i * static_cast<long>(Kp) * K;
    constexpr int PF = NCH >= 4 ? 1 : 4 / NCH;
    T pf[PF][NV];
#pragma unroll
    for (int r = 0; r < PF; ++r) {
        const int kp = grp + r * ngrp;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e0 = (c * lpr + lane) * VEC;
            if (kp < Kp && e0 < K) {
                T f[VEC];
                load_vec_hint<T, VEC>(tile + static_cast<long>(kp) * K + e0, f, nt);
#pragma unroll
                for (int q = 0; q < VEC; ++q) pf[r][c * VEC + q] = f[q];
            } else {
#pragma unroll
                for (int q = 0; q < VEC; ++q) pf[r][c * VEC + q] = T(0);
            }
        }
    }
    double ud[NV];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int e0 = (c * lpr + lane) * VEC;
        const int ec = e0 < K ? e0 : K - VEC;
#pragma unroll
        for (int q = 0; q < VEC; ++q) ud[c * VEC + q] = ut[i * K + ec + q];
    }
    const long p = pidx ? pidx[i] : 0;
    double mr[2];
    T wr[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int kp = threadIdx.x + r * BLOCK;
        const int kc = kp < Kp ? kp : 0;
        mr[r] = m[i * Kp + kc];
        wr[r] = wp[p * Kp + kc];
    }
    const T z0 = (mone && wave < d && wl < K) ? z[(i * K + wl) * d + wave] : T(0);
    double mx = -__builtin_inf();
#pragma unroll
    for (int c = 0; c < NCH; ++c)
        if ((c * lpr + lane) * VEC < K)
#pragma unroll
            for (int q = 0; q < VEC; ++q) mx = fmax(mx, ud[c * VEC + q]);
    const double sh = finite_or_zero(group_max(mx, lpr));
    // rows whose parent weight is not positive contribute nothing: their
    // weight becomes 0 and their message +inf, so exp(...) = 0 and the
    // accumulation is a plain fused multiply-add
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int kp = threadIdx.x + r * BLOCK;
        if (kp < Kp) {
            const bool live = wr[r] > T(0);
            s_m[kp] = live ? static_cast<T>(mr[r] - sh) : pos_inf<T>();
            s_wp[kp] = live ? wr[r] : T(0);
        }
    }
    T utv[NV], acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        utv[q] = static_cast<T>(ud[q] - sh);
        acc[q] = 0;
    }
    __syncthreads();
    auto add_row = [&](int kp, const T (&f)[NV]) {
        const T wk = s_wp[kp];
        const T rs = row_shift(s_m[kp]);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e0 = (c * lpr + lane) * VEC;
            if (e0 < K) {
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    const T e = exp_minus(f[c * VEC + q] + utv[c * VEC + q], rs);
                    acc[c * VEC + q] = fma(wk, e, acc[c * VEC + q]);
                }
            }
        }
    };
#pragma unroll
    for (int r = 0; r < PF; ++r)
        if (grp + r * ngrp < Kp) add_row(grp + r * ngrp, pf[r]);
#pragma unroll 4
    for (int kp = grp + PF * ngrp; kp < Kp; kp += ngrp) {
        T f[NV];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e0 = (c * lpr + lane) * VEC;
            if (e0 < K) {
                T fv[VEC];
                load_vec_hint<T, VEC>(tile + static_cast<long>(kp) * K + e0, fv, nt);
#pragma unroll
                for (int q = 0; q < VEC; ++q) f[c * VEC + q] = fv[q];
            } else {
#pragma unroll
                for (int q = 0; q < VEC; ++q) f[c * VEC + q] = T(0);
            }
        }
        add_row(kp, f);
    }
    // reduce over the row groups of a wave, then over waves in a fixed order
#pragma unroll
    for (int q = 0; q < NV; ++q)
        for (int off = lpr; off < WAVE; off <<= 1) acc[q] += __shfl_xor(acc[q], off, WAVE);
    if (wl < lpr) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e0 = (c * lpr + lane) * VEC;
#pragma unroll
            for (int q = 0; q < VEC; ++q)
                if (e0 + q < K) red[wave][e0 + q] = acc[c * VEC + q];
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += BLOCK) {
        T sum = red[0][k];
        for (int wv = 1; wv < BLOCK / WAVE; ++wv) sum += red[wv][k];
        w[i * K + k] = sum;
        s_w[k] = sum;
    }
    if (!mone) return;
    // fused moments: mone[i,j,:] = sum_k w (z, z^2), FP64, one wave per dimension
    __syncthreads();
    for (int j = wave; j < d; j += BLOCK / WAVE) {
        double s1 = 0.0, s2 = 0.0;
        for (int k = wl; k < K; k += WAVE) {
            const double wk = static_cast<double>(s_w[k]);
            const double zk = static_cast<double>((j == wave && k == wl) ? z0 : z[(i * K + k) * d + j]);
            s1 += wk * zk;
            s2 += wk * zk * zk;
        }
        s1 = group_sum(s1, WAVE);
        s2 = group_sum(s2, WAVE);
        if (wl == 0) {
            mone[(i * d + j) * 2 + 0] = s1;
            mone[(i * d + j) * 2 + 1] = s2;
        }
    }
}

// Plate backward with the linear-Gaussian factor recomputed instead of read
// (the table is not kept): the thread's child-sample columns in registers,
// the parent means in LDS, the rest as k_plate_bwd, so the weights and
// moments are the same bits as k_plate_bwd over the table k_plate_fwd_pn
// writes.  WPI waves per instance: 4 is k_plate_bwd's layout (one workgroup
// per instance); 1 puts four instances in a workgroup, one wave each, which
// spreads the per-instance work (prologue, shift, reductions, moments) over
// four times as many pairs per thread.  A one-wave instance keeps the rows
// of each of the four waves of the other layout in a sum of its own and
// adds the four in wave order at the end: the same additions in the same
// order, so both layouts give the same bits.
template <typename T, int VEC, int NCH, int LPR, int D, int WPI>
__global__ void __launch_bounds__(BLOCK) k_plate_bwd_pn(const T* __restrict__ zc, const T* __restrict__ zp,
                                                        const int32_t* __restrict__ pidx,
                                                        const double* __restrict__ ut,
                                                        const double* __restrict__ m, const T* __restrict__ wp,
                                                        T* __restrict__ w, long n, int K, int Kp, T a, T b, T c0,
                                                        T hp, double* __restrict__ mone) {
    constexpr int lpr = LPR;
    constexpr int NV = NCH * VEC;
    constexpr int NT = WPI * WAVE;      // threads per instance
    constexpr int IPB = BLOCK / NT;     // instances per workgroup
    constexpr int VW = 4 / WPI;         // waves of the four-wave layout kept by each wave
    constexpr int SM = WPI == 1 ? 128 : 512;
    constexpr int G1 = WAVE / lpr;      // row groups per wave
    constexpr int G4 = BLOCK / lpr;     // row groups of a four-wave instance
    __shared__ T red[WPI > 1 ? BLOCK / WAVE : 1][WPI > 1 ? 512 : 1];
    __shared__ T s_m[IPB][SM], s_wp[IPB][SM], s_w[IPB][SM];
    extern __shared__ unsigned char smem_raw[];
    const int slot = threadIdx.x / NT;
    const int ti = threadIdx.x % NT;
    T* s_mean = reinterpret_cast<T*>(smem_raw) + slot * Kp * D;   // [Kp, D] of this instance
    const int lane = ti & (lpr - 1);
    const int gg = (ti & (WAVE - 1)) / lpr;   // row group within the wave
    const int wave = threadIdx.x / WAVE;
    const int wv = ti / WAVE;                  // wave within the instance
    const int wl = threadIdx.x & (WAVE - 1);
    const long i0 = static_cast<long>(blockIdx.x) * IPB + slot;
    const bool valid = i0 < n;
    const long i = valid ? i0 : n - 1;   // a slot past the end loads in bounds and stores nothing
    const long pi = pidx ? pidx[i] : 0;
    T zr[NV][D];
    double ud[NV];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int e0 = (c * lpr + lane) * VEC;
        const int ec = e0 < K ? e0 : K - VEC;
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
#pragma unroll
            for (int j = 0; j < D; ++j) zr[c * VEC + q][j] = zc[(i * K + ec + q) * D + j];
            ud[c * VEC + q] = ut[i * K + ec + q];
        }
    }
    double mr[2];
    T wr[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int kp = ti + r * NT;
        const int kc = kp < Kp ? kp : 0;
        mr[r] = m[i * Kp + kc];
        wr[r] = wp[pi * Kp + kc];
    }
    for (int e = ti; e < Kp * D; e += NT) s_mean[e] = pair_mean(a, zp[pi * Kp * D + e], b);
    double mx = -__builtin_inf();
#pragma unroll
    for (int c = 0; c < NCH; ++c)
        if ((c * lpr + lane) * VEC < K)
#pragma unroll
            for (int q = 0; q < VEC; ++q) mx = fmax(mx, ud[c * VEC + q]);
    const double sh = finite_or_zero(group_max(mx, lpr));
    // rows whose parent weight is not positive contribute nothing: their
    // weight becomes 0 and their message +inf, so exp(...) = 0
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int kp = ti + r * NT;
        if (kp < Kp) {
            const bool live = wr[r] > T(0);
            s_m[slot][kp] = live ? static_cast<T>(mr[r] - sh) : pos_inf<T>();
            s_wp[slot][kp] = live ? wr[r] : T(0);
        }
    }
    T utv[NV], acc[VW][NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        utv[q] = static_cast<T>(ud[q] - sh);
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[v][q] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < VW; ++v) {
        // the rows of row group (wave wv * VW + v, group gg) of the four-wave layout
#pragma unroll 2
        for (int kp = (wv * VW + v) * G1 + gg; kp < Kp; kp += G4) {
            const T wk = s_wp[slot][kp];
            const T rs = row_shift(s_m[slot][kp]);
            T mean[D];
#pragma unroll
            for (int j = 0; j < D; ++j) mean[j] = s_mean[kp * D + j];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
                if (e0 < K) {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) {
                        const T f = normal_pair_value<T, D>(zr[c * VEC + q], mean, D, c0, hp);
                        const T e = exp_minus(f + utv[c * VEC + q], rs);
                        acc[v][c * VEC + q] = fma(wk, e, acc[v][c * VEC + q]);
                    }
                }
            }
        }
    }
    // the row groups of each wave by lane swaps, then the waves in order
#pragma unroll
    for (int v = 0; v < VW; ++v)
#pragma unroll
        for (int q = 0; q < NV; ++q)
            for (int off = lpr; off < WAVE; off <<= 1) acc[v][q] += __shfl_xor(acc[v][q], off, WAVE);
    if constexpr (WPI == 1) {
        if (wl < lpr) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
#pragma unroll
                for (int q = 0; q < VEC; ++q)
                    if (e0 + q < K) {
                        T sum = acc[0][c * VEC + q];
#pragma unroll
                        for (int v = 1; v < VW; ++v) sum += acc[v][c * VEC + q];
                        s_w[slot][e0 + q] = sum;
                        if (valid) w[i * K + e0 + q] = sum;
                    }
            }
        }
    } else {
        if (wl < lpr) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
#pragma unroll
                for (int q = 0; q < VEC; ++q)
                    if (e0 + q < K) red[wave][e0 + q] = acc[0][c * VEC + q];
            }
        }
        __syncthreads();
        for (int k = ti; k < K; k += NT) {
            T sum = red[0][k];
            for (int v = 1; v < BLOCK / WAVE; ++v) sum += red[v][k];
            w[i * K + k] = sum;
            s_w[slot][k] = sum;
        }
    }
    if (!mone) return;
    __syncthreads();
    // fused moments: mone[i,j,:] = sum_k w (z, z^2), FP64, one wave per dimension
    for (int j = wv; j < D; j += WPI) {
        double s1 = 0.0, s2 = 0.0;
        for (int k = wl; k < K; k += WAVE) {
            const double wk = static_cast<double>(s_w[slot][k]);
            const double zk = static_cast<double>(zc[(i * K + k) * D + j]);
            s1 += wk * zk;
            s2 += wk * zk * zk;
        }
        s1 = group_sum(s1, WAVE);
        s2 = group_sum(s2, WAVE);
        if (wl == 0 && valid) {
            mone[(i * D + j) * 2 + 0] = s1;
            mone[(i * D + j) * 2 + 1] = s2;
        }
    }
}

// One wave per instance.
__global__ void __launch_bounds__(BLOCK) k_root_lse(const double* __restrict__ ut, double* __restrict__ L, long n, int K) {
    const long i = static_cast<long>(blockIdx.x) * (BLOCK / WAVE) + threadIdx.x / WAVE;
    if (i >= n) return;
    const double Li = wave_lse(ut + i * K, K);
    if ((threadIdx.x & (WAVE - 1)) == 0) L[i] = Li;
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_root_w(const double* __restrict__ ut, const double* __restrict__ L,
                                                  T* __restrict__ w, long n, int K, const double* __restrict__ g) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * K) return;
    const long i = t / K;
    const double s = g ? *g : 1.0;
    const double Li = L[i];
    w[t] = static_cast<T>(Li == -__builtin_inf() ? 0.0 : s * exp(ut[t] - Li));
}

// Single workgroup: log P_MP = sum of the components' L.
__global__ void __launch_bounds__(BLOCK) k_sum_L(const double* __restrict__ L, long nL, double* __restrict__ out,
                                                 uint32_t* __restrict__ status) {
    __shared__ double red[BLOCK];
    const double v = block_sum(L, nL, red);
    if (threadIdx.x == 0) {
        *out = v;
        if (!isfinite(v)) atomicOr(status, 0x1u);
    }
}

// Subset sums of one parent instance's child messages, one workgroup per
// (child list, subset): the strided subsets and the in-subset order of
// block_gather, so adding them in subset order gives its bits, with the
// reads spread over many compute units (one workgroup's outstanding misses
// bound a large single-workgroup gather).
constexpr int SUBSET_CHUNK = 4096;   // child indices of one subset staged in LDS at a time

__global__ void __launch_bounds__(BLOCK) k_gather_subsets(ChildLists cl, long q, int K, double* __restrict__ part) {
    __shared__ int32_t s_idx[SUBSET_CHUNK];
    const int S = 1024 / K;
    const int c = blockIdx.x / S, p = blockIdx.x % S;
    const int per = cl.per[c];
    const int j0 = per ? static_cast<int>(q) * per : cl.off[c][q];
    const int j1 = per ? j0 + per : cl.off[c][q + 1];
    const int n = j1 - j0 > p ? (j1 - j0 - p + S - 1) / S : 0;   // positions j0 + p + t S, t < n
    const double* __restrict__ mc = cl.mc[c];
    const int32_t* __restrict__ idx = cl.idx[c];
    double acc[(512 + BLOCK - 1) / BLOCK] = {};
    for (int t0 = 0; t0 < n; t0 += SUBSET_CHUNK) {
        const int tn = n - t0 < SUBSET_CHUNK ? n - t0 : SUBSET_CHUNK;
        if (!per) {
            __syncthreads();
            for (int t = threadIdx.x; t < tn; t += BLOCK) s_idx[t] = idx[j0 + p + static_cast<long>(t0 + t) * S];
            __syncthreads();
        }
        for (int r = 0; r * BLOCK < K; ++r) {
            const int k = r * BLOCK + threadIdx.x;
            if (k < K)
                acc[r] = per ? sum_rows_in_order(acc[r], mc, nullptr, j0 + p + static_cast<long>(t0) * S, tn, S, K, k)
                             : sum_rows_in_order(acc[r], mc, s_idx, 0, tn, 1, K, k);
        }
    }
    for (int r = 0; r * BLOCK < K; ++r) {
        const int k = r * BLOCK + threadIdx.x;
        if (k < K) part[(c * S + p) * K + k] = acc[r];
    }
}

// ut = u + the subset sums of k_gather_subsets, list by list, subsets in
// order: block_gather's additions for a single-instance parent, so its bits.
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_gather_finish(double* __restrict__ ut, const T* __restrict__ u, int nl,
                                                         int K, const double* __restrict__ part) {
    const int k = blockIdx.x * BLOCK + threadIdx.x;
    if (k >= K) return;
    const int S = 1024 / K;
    double sum = static_cast<double>(u[k]);
    for (int c = 0; c < nl; ++c)
        for (int p = 0; p < S; ++p) sum += part[(c * S + p) * K + k];
    ut[k] = sum;
}

// The whole root level of a single-instance root node in one workgroup:
// ut = u + child messages (block_gather), L = LSE_k ut (wave_lse), log P_MP =
// sum of all components' L (block_sum; nL = 0 leaves it to k_sum_L), the
// root weights w = g exp(ut - L), their moments (moment_sums) and the
// M-step of the node (mstep_entry), and the device iteration counter.  Same
// arithmetic, in the same order, as k_gather, k_root_lse, k_sum_L, k_root_w,
// k_moments and k_mstep.
constexpr int ROOT_FIN_Z = 2048;   // samples of the root staged in LDS when K*d fits

template <typename T>
__global__ void __launch_bounds__(CS_BLOCK) k_root_fin(RootFinArgs a) {
    __shared__ double s_ut[512];
    __shared__ double red[1024];
    __shared__ int32_t s_idx[1024];
    __shared__ T s_z[ROOT_FIN_Z];
    __shared__ T s_w[512];
    __shared__ double s_L;
    __shared__ int s_nonfinite;
    const int K = a.K;
    const bool z_lds = K * a.d <= ROOT_FIN_Z;
    if (z_lds)
        for (int e = threadIdx.x; e < K * a.d; e += CS_BLOCK) s_z[e] = static_cast<const T*>(a.z)[e];
    // every load that does not wait on this kernel's own results goes out
    // first: the M-step's previous mean parameters and EMA weight, the parent
    // weight scale, the status word and the iteration counter
    const bool ms_here = a.ms.mema && static_cast<int>(threadIdx.x) < a.d;
    const double pm1 = ms_here ? a.ms.mema[threadIdx.x * 2] : 0.0;
    const double pm2 = ms_here ? a.ms.mema[threadIdx.x * 2 + 1] : 0.0;
    const double lam = ms_here ? (a.ms.lam_dev ? *a.ms.lam_dev : a.ms.lam) : 0.0;
    const double gs = a.g ? *a.g : 1.0;
    const uint32_t st0 = (a.nL <= 0 && threadIdx.x == 0) ? a.status[0] : 0u;
    const uint64_t it0 = (a.iter_dev && threadIdx.x == 0) ? *a.iter_dev : 0u;
    if (a.part) {
        // u plus the subset sums, list by list, subsets in order (as block_gather adds them)
        const int S = 1024 / K;
        for (int k = threadIdx.x; k < K; k += CS_BLOCK) {
            double sum = static_cast<double>(static_cast<const T*>(a.u)[k]);
            for (int c = 0; c < a.cl.n; ++c)
                for (int p = 0; p < S; ++p) sum += a.part[(c * S + p) * K + k];
            s_ut[k] = sum;
        }
        __syncthreads();
    } else {
        block_gather(s_ut, static_cast<const T*>(a.u), a.cl, 0, K, red, s_idx);
    }
    for (int k = threadIdx.x; k < K; k += CS_BLOCK) a.ut[k] = s_ut[k];
    if (threadIdx.x < WAVE) {
        const double L = wave_lse(s_ut, K);
        if (threadIdx.x == 0) {
            *a.L = L;
            s_L = L;
        }
    }
    __syncthreads();   // the L slot is read back by the sum below
    if (a.nL == 1 && a.L == a.Lall) {
        // the only component: block_sum would return 0 + L
        if (threadIdx.x == 0) {
            const double v = 0.0 + s_L;
            *a.logphat = v;
            s_nonfinite = !isfinite(v);
            if (!isfinite(v)) atomicOr(a.status, 0x1u);
        }
    } else if (a.nL > 0) {
        const double v = block_sum(a.Lall, a.nL, red);
        if (threadIdx.x == 0) {
            *a.logphat = v;
            s_nonfinite = !isfinite(v);
            if (!isfinite(v)) atomicOr(a.status, 0x1u);
        }
    } else if (threadIdx.x == 0) {
        s_nonfinite = (st0 & 0x1u) != 0u;
    }
    __syncthreads();
    const double L = s_L;
    T* w = static_cast<T*>(a.w);
    for (int k = threadIdx.x; k < K; k += CS_BLOCK) {
        const T wk = static_cast<T>(L == -__builtin_inf() ? 0.0 : gs * exp(s_ut[k] - L));
        w[k] = wk;
        s_w[k] = wk;
    }
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < a.d) {
        const int j = threadIdx.x;
        double s1, s2;
        moment_sums(z_lds ? s_z : static_cast<const T*>(a.z), s_w, j, K, a.d, s1, s2, a.logz);
        a.mone[j * 2 + 0] = s1;
        a.mone[j * 2 + 1] = s2;
        if (ms_here)
            mstep_update(a.ms.mema, a.ms.qp, j, pm1, pm2, s1, s2, a.ms.qfamily, lam, s_nonfinite != 0,
                         a.ms.status);
    }
    if (a.iter_dev && threadIdx.x == 0) *a.iter_dev = it0 + 1;
}

// ---------------------------------------------------------------- chains
// One workgroup per series g; steps t = T-1 .. 1 are eliminated in order.
// ut[g*T + t, :] holds u plus child messages on entry; on exit it holds the
// full u-tilde of every step (needed by the reverse pass).

template <typename T, int VEC, int NCH, int LPR>
__global__ void __launch_bounds__(BLOCK) k_chain_fwd(const T* __restrict__ F, double* __restrict__ ut,
                                                     double* __restrict__ m, double* __restrict__ L,
                                                     int T_, int K, bool nt, T U) {
    constexpr int lpr = LPR;
    __shared__ double s_ut[512];
    __shared__ double s_msg[512];
    __shared__ double s_scr[BLOCK / WAVE];
    const int lane = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int ngrp = BLOCK / lpr;
    const long g = blockIdx.x;
    const long tileKK = static_cast<long>(K) * K;
    for (int t = T_ - 1; t >= 1; --t) {
        double* utt = ut + (g * T_ + t) * K;
        for (int k = threadIdx.x; k < K; k += BLOCK) {
            const double v = utt[k] + ((t < T_ - 1) ? s_msg[k] : 0.0);
            s_ut[k] = v;
            utt[k] = v;
        }
        __syncthreads();
        const double sh = finite_or_zero(block_max(s_ut, K, s_scr));
        // the thread's columns of ut - sh, once per step
        T utv[NCH * VEC];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e0 = (c * lpr + lane) * VEC;
#pragma unroll
            for (int q = 0; q < VEC; ++q) utv[c * VEC + q] = (e0 < K) ? static_cast<T>(s_ut[e0 + q] - sh) : T(0);
        }
        const T* Ft = F + (g * (T_ - 1) + (t - 1)) * tileKK;
        for (int kp0 = 0; kp0 < K; kp0 += ngrp * 2) {
            T v[2][NCH * VEC];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int kp = kp0 + r * ngrp + grp;
                if (kp < K) load_row_plus<T, VEC, NCH>(Ft + static_cast<long>(kp) * K, utv, K, lane, lpr, v[r], nt);
                else {
#pragma unroll
                    for (int q = 0; q < NCH * VEC; ++q) v[r][q] = neg_inf<T>();
                }
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int kp = kp0 + r * ngrp + grp;
                const T res = lse_group_bounded<T, NCH * VEC>(v[r], lpr, U);
                if (lane == 0 && kp < K) {
                    const double mv = (res == neg_inf<T>()) ? -__builtin_inf() : sh + static_cast<double>(res);
                    m[(g * T_ + t) * K + kp] = mv;
                    s_msg[kp] = mv;
                }
            }
        }
        __syncthreads();
    }
    // step 0: u-tilde and the series' root log-sum-exp
    double* ut0 = ut + g * T_ * K;
    for (int k = threadIdx.x; k < K; k += BLOCK) {
        const double v = ut0[k] + ((T_ > 1) ? s_msg[k] : 0.0);
        s_ut[k] = v;
        ut0[k] = v;
    }
    __syncthreads();
    if (threadIdx.x < WAVE) {
        double mx = -__builtin_inf();
        for (int k = threadIdx.x; k < K; k += WAVE) mx = fmax(mx, s_ut[k]);
        mx = group_max(mx, WAVE);
        double s = 0.0;
        if (mx != -__builtin_inf())
            for (int k = threadIdx.x; k < K; k += WAVE) s += exp(s_ut[k] - mx);
        s = group_sum(s, WAVE);
        if (threadIdx.x == 0) L[g] = (mx == -__builtin_inf()) ? mx : mx + log(s);
    }
}

// The chain forward with the linear-Gaussian step factor evaluated in place:
// F_t[kp,k] = c0 - hp (z_t[k] - (a z_{t-1}[kp] + b))^2 is computed from the
// series' samples (the thread's columns of z_t in registers), written out for
// the reverse pass and reduced exactly as k_chain_fwd reduces the rows it
// loads, so F, the messages and L are the same bits as the pair-table kernel
// followed by k_chain_fwd.  With vs.Kb > 0 block g is the virtual series
// (g / Kb, parent sample g % Kb) of a chain under a sampled parent: the
// samples are series g / Kb's, the mean offset b + (1 - a) beta, ut is
// written from vs.usrc with the start term added at step 0.
template <typename T, int VEC, int NCH, int LPR>
__global__ void __launch_bounds__(BLOCK) k_chain_fwd_pn(T* __restrict__ F, const T* __restrict__ z,
                                                        double* __restrict__ ut, double* __restrict__ m,
                                                        double* __restrict__ L, int T_, int K, T a, T b, T c0,
                                                        T hp, bool nt, VSeries vs) {
    constexpr int lpr = LPR;
    constexpr int NV = NCH * VEC;
    __shared__ double s_ut[512];
    __shared__ double s_msg[512];
    __shared__ double s_scr[BLOCK / WAVE];
    __shared__ T s_zp[512];
    const int lane = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int ngrp = BLOCK / lpr;
    const long g = blockIdx.x;
    // a virtual series (vs.Kb > 0) reads the samples of series gz and its
    // parent sample beta
    const long gz = vs.Kb ? g / vs.Kb : g;
    const double beta = vs.Kb ? static_cast<double>(static_cast<const T*>(vs.zb)[
                                    static_cast<long>(vs.sp[gz]) * vs.Kb + g % vs.Kb]) : 0.0;
    const T bg = vs.Kb ? static_cast<T>(vs.b + (1.0 - vs.a) * beta) : b;
    const double* usrc = vs.Kb ? vs.usrc + gz * T_ * K : ut + g * T_ * K;
    const long tileKK = static_cast<long>(K) * K;
    for (int t = T_ - 1; t >= 1; --t) {
        const T* zt = z + (gz * T_ + t) * K;
        const T* zp = zt - K;
        T zr[NV];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e0 = (c * lpr + lane) * VEC;
            const int ec = e0 < K ? e0 : K - VEC;
#pragma unroll
            for (int q = 0; q < VEC; ++q) zr[c * VEC + q] = zt[ec + q];
        }
        double* utt = ut + (g * T_ + t) * K;
        const double* srct = usrc + static_cast<long>(t) * K;
        // the step's u-tilde and the previous step's samples (the rows'
        // means) into LDS, so the row loop issues no global load
        for (int k = threadIdx.x; k < K; k += BLOCK) {
            const double v = srct[k] + ((t < T_ - 1) ? s_msg[k] : 0.0);
            s_ut[k] = v;
            utt[k] = v;
            s_zp[k] = zp[k];
        }
        __syncthreads();
        const double sh = finite_or_zero(block_max(s_ut, K, s_scr));
        // the thread's columns of ut - sh, once per step
        T utv[NV];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e0 = (c * lpr + lane) * VEC;
#pragma unroll
            for (int q = 0; q < VEC; ++q) utv[c * VEC + q] = (e0 < K) ? static_cast<T>(s_ut[e0 + q] - sh) : T(0);
        }
        T* Ft = F ? F + (g * (T_ - 1) + (t - 1)) * tileKK : nullptr;
        for (int kp0 = 0; kp0 < K; kp0 += ngrp * 2) {
            T v[2][NV];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int kp = kp0 + r * ngrp + grp;
                const T mean = pair_mean(a, s_zp[kp < K ? kp : K - 1], bg);
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const int e0 = (c * lpr + lane) * VEC;
                    if (kp < K && e0 < K) {
                        T f[VEC];
#pragma unroll
                        for (int q = 0; q < VEC; ++q) f[q] = normal_pair_value<T, 1>(&zr[c * VEC + q], &mean, 1, c0, hp);
                        if (F) store_vec_hint<T, VEC>(Ft + static_cast<long>(kp) * K + e0, f, nt);
#pragma unroll
                        for (int q = 0; q < VEC; ++q) v[r][c * VEC + q] = f[q] + utv[c * VEC + q];
                    } else {
#pragma unroll
                        for (int q = 0; q < VEC; ++q) v[r][c * VEC + q] = neg_inf<T>();
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int kp = kp0 + r * ngrp + grp;
                const T res = lse_group_bounded<T, NV>(v[r], lpr, c0);
                if (lane == 0 && kp < K) {
                    const double mv = (res == neg_inf<T>()) ? -__builtin_inf() : sh + static_cast<double>(res);
                    m[(g * T_ + t) * K + kp] = mv;
                    s_msg[kp] = mv;
                }
            }
        }
        __syncthreads();
    }
    double* ut0 = ut + g * T_ * K;
    for (int k = threadIdx.x; k < K; k += BLOCK) {
        double v = usrc[k];
        if (vs.Kb) {
            const double dx = static_cast<double>(z[gz * T_ * K + k]) - beta - vs.ib;
            v += vs.ic0 - vs.ihp * dx * dx;
        }
        v += (T_ > 1) ? s_msg[k] : 0.0;
        s_ut[k] = v;
        ut0[k] = v;
    }
    __syncthreads();
    if (threadIdx.x < WAVE) {
        double mx = -__builtin_inf();
        for (int k = threadIdx.x; k < K; k += WAVE) mx = fmax(mx, s_ut[k]);
        mx = group_max(mx, WAVE);
        double s = 0.0;
        if (mx != -__builtin_inf())
            for (int k = threadIdx.x; k < K; k += WAVE) s += exp(s_ut[k] - mx);
        s = group_sum(s, WAVE);
        if (threadIdx.x == 0) L[g] = (mx == -__builtin_inf()) ? mx : mx + log(s);
    }
}

template <typename T, int VEC, int NCH, int LPR>
__global__ void __launch_bounds__(BLOCK) k_chain_bwd(const T* __restrict__ F, const double* __restrict__ ut,
                                                     const double* __restrict__ m, const double* __restrict__ L,
                                                     T* __restrict__ w, int T_, int K,
                                                     const double* __restrict__ gsc, bool nt) {
    constexpr int lpr = LPR;
    constexpr int RPT = (512 + BLOCK - 1) / BLOCK;   // rows staged per thread
    __shared__ T s_w[512];
    __shared__ T red[BLOCK / WAVE][512];
    __shared__ double s_scr[BLOCK / WAVE];
    __shared__ T s_mk[512];
    const int lane = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int ngrp = BLOCK / lpr;
    const long g = blockIdx.x;
    const long tileKK = static_cast<long>(K) * K;
    const double sc = gsc ? *gsc : 1.0;
    const double Lg = L[g];
    for (int k = threadIdx.x; k < K; k += BLOCK) {
        const T v = static_cast<T>(Lg == -__builtin_inf() ? 0.0 : sc * exp(ut[g * T_ * K + k] - Lg));
        s_w[k] = v;
        w[g * T_ * K + k] = v;
    }
    __syncthreads();
    for (int t = 1; t < T_; ++t) {
        const double* utt = ut + (g * T_ + t) * K;
        const double* mt = m + (g * T_ + t) * K;
        // the rows' messages, fetched with the shift's loads, then shifted
        // into LDS (+inf where the previous weight is not positive)
        double mrow[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int k = r * BLOCK + threadIdx.x;
            mrow[r] = k < K ? mt[k] : 0.0;
        }
        const double sh = finite_or_zero(block_max(utt, K, s_scr));
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int k = r * BLOCK + threadIdx.x;
            if (k < K) s_mk[k] = s_w[k] > T(0) ? static_cast<T>(mrow[r] - sh) : pos_inf<T>();
        }
        __syncthreads();
        T utv[NCH * VEC], acc[NCH * VEC];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e0 = (c * lpr + lane) * VEC;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                utv[c * VEC + q] = (e0 < K) ? static_cast<T>(utt[e0 + q] - sh) : T(0);
                acc[c * VEC + q] = 0;
            }
        }
        const T* Ft = F + (g * (T_ - 1) + (t - 1)) * tileKK;
#pragma unroll 2
        for (int kp = grp; kp < K; kp += ngrp) {
            // a row whose weight is not positive contributes nothing (weight 0, message +inf)
            const T wr = s_w[kp];
            const T wk = wr > T(0) ? wr : T(0);
            const T rs = row_shift(s_mk[kp]);
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
                if (e0 < K) {
                    T f[VEC];
                    load_vec_hint<T, VEC>(Ft + static_cast<long>(kp) * K + e0, f, nt);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) {
                        const T e = exp_minus(f[q] + utv[c * VEC + q], rs);
                        acc[c * VEC + q] = fma(wk, e, acc[c * VEC + q]);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NCH * VEC; ++q)
            for (int off = lpr; off < WAVE; off <<= 1) acc[q] += __shfl_xor(acc[q], off, WAVE);
        const int wave = threadIdx.x / WAVE;
        if ((threadIdx.x & (WAVE - 1)) < lpr) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
#pragma unroll
                for (int q = 0; q < VEC; ++q)
                    if (e0 + q < K) red[wave][e0 + q] = acc[c * VEC + q];
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += BLOCK) {
            T s = red[0][k];
            for (int wv = 1; wv < BLOCK / WAVE; ++wv) s += red[wv][k];
            s_w[k] = s;
            w[(g * T_ + t) * K + k] = s;
        }
        __syncthreads();
    }
}

// Chain reverse pass with the step factor recomputed instead of read (the
// table is not kept); otherwise as k_chain_bwd (same lanes, same order).
// With vs.Kb > 0 (a chain under a sampled parent) the weights of virtual
// series g start from the parent weight of its sample, vs.wb[sp * Kb + kb].
template <typename T, int VEC, int NCH, int LPR, bool RENORM>
__global__ void __launch_bounds__(BLOCK) k_chain_bwd_pn(const T* __restrict__ z, const double* __restrict__ ut,
                                                        const double* __restrict__ m, const double* __restrict__ L,
                                                        T* __restrict__ w, int T_, int K, T a, T b, T c0, T hp,
                                                        const double* __restrict__ gsc, VSeries vs) {
    constexpr int lpr = LPR;
    constexpr int NV = NCH * VEC;
    constexpr int RPT = (512 + BLOCK - 1) / BLOCK;   // rows staged per thread
    __shared__ T s_w[512];
    __shared__ T red[BLOCK / WAVE][512];
    __shared__ double s_scr[BLOCK / WAVE];
    __shared__ T s_tot;
    __shared__ T s_mk[512], s_mean[512];
    const int lane = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int ngrp = BLOCK / lpr;
    const long g = blockIdx.x;
    const long gz = vs.Kb ? g / vs.Kb : g;
    const long pb = vs.Kb ? static_cast<long>(vs.sp[gz]) * vs.Kb + g % vs.Kb : 0;
    const T bg = vs.Kb ? static_cast<T>(vs.b + (1.0 - vs.a) * static_cast<double>(static_cast<const T*>(vs.zb)[pb])) : b;
    const double sc = vs.Kb ? static_cast<double>(static_cast<const T*>(vs.wb)[pb]) : (gsc ? *gsc : 1.0);
    const double Lg = L[g];
    for (int k = threadIdx.x; k < K; k += BLOCK) {
        const T v = static_cast<T>(Lg == -__builtin_inf() ? 0.0 : sc * exp(ut[g * T_ * K + k] - Lg));
        s_w[k] = v;
        w[g * T_ * K + k] = v;
    }
    __syncthreads();
    for (int t = 1; t < T_; ++t) {
        const double* utt = ut + (g * T_ + t) * K;
        const double* mt = m + (g * T_ + t) * K;
        const T* zt = z + (gz * T_ + t) * K;
        const T* zp = zt - K;
        // the rows' messages and previous samples, fetched with the shift's loads
        double mrow[RPT];
        T zrow[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int k = r * BLOCK + threadIdx.x;
            mrow[r] = k < K ? mt[k] : 0.0;
            zrow[r] = k < K ? zp[k] : T(0);
        }
        const double sh = finite_or_zero(block_max(utt, K, s_scr));
        // per row: the shifted message (+inf where the previous weight is not
        // positive, so its exponential is 0) and the mean, in LDS
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int k = r * BLOCK + threadIdx.x;
            if (k < K) {
                s_mk[k] = s_w[k] > T(0) ? static_cast<T>(mrow[r] - sh) : pos_inf<T>();
                s_mean[k] = pair_mean(a, zrow[r], bg);
            }
        }
        __syncthreads();
        T utv[NV], acc[NV], zr[NV];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e0 = (c * lpr + lane) * VEC;
            const int ec = e0 < K ? e0 : K - VEC;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                utv[c * VEC + q] = (e0 < K) ? static_cast<T>(utt[e0 + q] - sh) : T(0);
                acc[c * VEC + q] = 0;
                zr[c * VEC + q] = zt[ec + q];
            }
        }
#pragma unroll 2
        for (int kp = grp; kp < K; kp += ngrp) {
            const T wr = s_w[kp];
            const T wk = wr > T(0) ? wr : T(0);
            const T rs = row_shift(s_mk[kp]);
            const T mean = s_mean[kp];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
                if (e0 < K) {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) {
                        const T f = normal_pair_value<T, 1>(&zr[c * VEC + q], &mean, 1, c0, hp);
                        const T e = exp_minus(f + utv[c * VEC + q], rs);
                        acc[c * VEC + q] = fma(wk, e, acc[c * VEC + q]);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NV; ++q)
            for (int off = lpr; off < WAVE; off <<= 1) acc[q] += __shfl_xor(acc[q], off, WAVE);
        const int wave = threadIdx.x / WAVE;
        if ((threadIdx.x & (WAVE - 1)) < lpr) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
#pragma unroll
                for (int q = 0; q < VEC; ++q)
                    if (e0 + q < K) red[wave][e0 + q] = acc[c * VEC + q];
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += BLOCK) {
            T sum = red[0][k];
            for (int wv = 1; wv < BLOCK / WAVE; ++wv) sum += red[wv][k];
            s_w[k] = sum;
            if (!RENORM) w[(g * T_ + t) * K + k] = sum;
        }
        __syncthreads();
        if constexpr (RENORM) {
            // rescale the step's weights to sum to the series' scale (k-strided
            // partial sums of wave 0, then its shuffle tree)
            if (threadIdx.x < WAVE) {
                T part = 0;
                for (int k = threadIdx.x; k < K; k += WAVE) part += s_w[k];
                for (int off = WAVE / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, WAVE);
                if (threadIdx.x == 0) s_tot = part;
            }
            __syncthreads();
            const T f = s_tot > T(0) ? static_cast<T>(sc) / s_tot : T(0);
            for (int k = threadIdx.x; k < K; k += BLOCK) {
                const T v = s_w[k] * f;
                s_w[k] = v;
                w[(g * T_ + t) * K + k] = v;
            }
            __syncthreads();
        }
    }
}

// The weights of a chain under a sampled parent: the sum over np parts per
// series (the parent samples kb, or blocks of them) of their weights
// [G, np, T, K], added in part order in FP64.  Consecutive threads take
// consecutive (t, k), so every part is read coalesced.
template <typename S, typename T>
__global__ void __launch_bounds__(BLOCK) k_chainp_wsum(const S* __restrict__ vw, T* __restrict__ w, long G, int np,
                                                       int T_, int K) {
    const long row = static_cast<long>(T_) * K;
    const long total = G * row;
    for (long e = blockIdx.x * static_cast<long>(BLOCK) + threadIdx.x; e < total;
         e += static_cast<long>(gridDim.x) * BLOCK) {
        const long g = e / row, r = e - g * row;
        const S* src = vw + g * np * row + r;
        double acc = 0.0;
        for (int q = 0; q < np; ++q) acc += static_cast<double>(src[q * row]);
        w[e] = static_cast<T>(acc);
    }
}

// ---------------------------------------------------------------- dispatch
// The (lanes per row, chunks per lane) pairs plan_rows produces for K <= 512;
// both are template parameters of the kernels, so the group reductions
// compile to straight-line lane moves.
#define QEM_ROW_PLANS(X) X(1, 1) X(2, 1) X(4, 1) X(8, 1) X(16, 1) X(16, 2) X(16, 4) X(32, 4) X(64, 4) X(64, 8)

template <typename T, int VEC, int NCH, int LPR>
hipError_t launch_fwd(hipStream_t s, const void* F, const double* ut, void* m, long n, int K, int Kp,
                      uint32_t* status) {
    constexpr int RPI = (NCH <= 2) ? 4 : 2;
    const int rows_per_pass = (BLOCK / LPR) * RPI;
    const int ipb = std::max(1, rows_per_pass / Kp);
    const int kp_shift = (Kp & (Kp - 1)) == 0 ? __builtin_ctz(static_cast<unsigned>(Kp)) : -1;
    const dim3 grid((n + ipb - 1) / ipb);
    const size_t sm = static_cast<size_t>(ipb) * (8 + static_cast<size_t>(K) * sizeof(T));
    const bool nt = static_cast<size_t>(n) * Kp * K * sizeof(T) > STREAM_BYTES;
    hipLaunchKernelGGL((k_plate_fwd<T, VEC, NCH, RPI, LPR>), grid, dim3(BLOCK), sm, s, (const T*)F, ut, (double*)m, n,
                       K, Kp, ipb, kp_shift, nt, status);
    return hipGetLastError();
}

template <typename T, int VEC>
hipError_t fwd_plan(hipStream_t s, const RowPlan& p, const void* F, const double* ut, void* m, long R, int K, int Kp,
                    uint32_t* status) {
#define QEM_CASE(L, N) \
    if (p.lpr == L && p.nch == N) return launch_fwd<T, VEC, N, L>(s, F, ut, m, R, K, Kp, status);
    QEM_ROW_PLANS(QEM_CASE)
#undef QEM_CASE
    return hipErrorInvalidValue;
}

template <typename T, int VEC, int NCH, int LPR, int D>
hipError_t launch_fwd_pn(hipStream_t s, void* F, const void* zc, const void* zp, const int32_t* pidx,
                         double* ut, void* m, long n, int K, int Kp, double a, double b, double c0, double hp,
                         const void* u, const ChildLists* cl, uint32_t* status) {
    if constexpr (NCH * VEC * D > 64 || LPR < 8) {
        return hipErrorInvalidValue;
    } else {
        constexpr int RPI = (NCH <= 2) ? 4 : 2;
        const size_t sm = static_cast<size_t>(Kp) * D * sizeof(T);
        const bool nt = static_cast<size_t>(n) * Kp * K * sizeof(T) > STREAM_BYTES;
        if (cl)
            hipLaunchKernelGGL((k_plate_fwd_pn<T, VEC, NCH, RPI, D, LPR, true>), dim3(n), dim3(BLOCK), sm, s, (T*)F,
                               (const T*)zc, (const T*)zp, pidx, ut, (double*)m, K, Kp, (T)a, (T)b, (T)c0, (T)hp, nt,
                               (const T*)u, *cl, status);
        else
            hipLaunchKernelGGL((k_plate_fwd_pn<T, VEC, NCH, RPI, D, LPR, false>), dim3(n), dim3(BLOCK), sm, s, (T*)F,
                               (const T*)zc, (const T*)zp, pidx, ut, (double*)m, K, Kp, (T)a, (T)b, (T)c0, (T)hp, nt,
                               (const T*)nullptr, ChildLists{}, status);
        return hipGetLastError();
    }
}

template <typename T, int VEC, int NCH, int LPR>
hipError_t fwd_pn_d(hipStream_t s, int d, void* F, const void* zc, const void* zp, const int32_t* pidx,
                    double* ut, void* m, long n, int K, int Kp, double a, double b, double c0, double hp,
                    const void* u, const ChildLists* cl, uint32_t* status) {
    switch (d) {
        case 1: return launch_fwd_pn<T, VEC, NCH, LPR, 1>(s, F, zc, zp, pidx, ut, m, n, K, Kp, a, b, c0, hp, u, cl, status);
        case 2: return launch_fwd_pn<T, VEC, NCH, LPR, 2>(s, F, zc, zp, pidx, ut, m, n, K, Kp, a, b, c0, hp, u, cl, status);
        case 3: return launch_fwd_pn<T, VEC, NCH, LPR, 3>(s, F, zc, zp, pidx, ut, m, n, K, Kp, a, b, c0, hp, u, cl, status);
        case 4: return launch_fwd_pn<T, VEC, NCH, LPR, 4>(s, F, zc, zp, pidx, ut, m, n, K, Kp, a, b, c0, hp, u, cl, status);
        case 8: return launch_fwd_pn<T, VEC, NCH, LPR, 8>(s, F, zc, zp, pidx, ut, m, n, K, Kp, a, b, c0, hp, u, cl, status);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int VEC>
hipError_t fwd_pn_plan(hipStream_t s, const RowPlan& p, int d, void* F, const void* zc, const void* zp,
                       const int32_t* pidx, double* ut, void* m, long n, int K, int Kp, double a, double b,
                       double c0, double hp, const void* u, const ChildLists* cl, uint32_t* status) {
#define QEM_CASE(L, N)                                                                                      \
    if (p.lpr == L && p.nch == N)                                                                           \
        return fwd_pn_d<T, VEC, N, L>(s, d, F, zc, zp, pidx, ut, m, n, K, Kp, a, b, c0, hp, u, cl, status);
    QEM_ROW_PLANS(QEM_CASE)
#undef QEM_CASE
    return hipErrorInvalidValue;
}

template <typename T, int VEC, int NCH, int LPR>
hipError_t launch_bwd(hipStream_t s, const void* F, const double* ut, const void* m, const void* wp,
                      const int32_t* pidx, void* w, long n, int K, int Kp, const void* z, double* mone, int d) {
    // The pair table is the last use of F in the iteration: nontemporal loads
    // whatever its size.  Measured at the 134 MB class level: the same time
    // when the forward pass has just written F (it is then partly in the
    // Infinity Cache), and about twice the rate of plain loads when the cache
    // holds other data (plain loads of a 128 MB stream behind a 512 MB
    // scrub: 2.5 TB/s; nontemporal: 5.8 TB/s).
    const bool nt = true;
    hipLaunchKernelGGL((k_plate_bwd<T, VEC, NCH, LPR>), dim3(n), dim3(BLOCK), 0, s, (const T*)F, ut, (const double*)m,
                       (const T*)wp, pidx, (T*)w, K, Kp, nt, (const T*)z, mone, d);
    return hipGetLastError();
}

template <typename T, int VEC>
hipError_t bwd_plan(hipStream_t s, const RowPlan& p, const void* F, const double* ut, const void* m, const void* wp,
                    const int32_t* pidx, void* w, long n, int K, int Kp, const void* z, double* mone, int d) {
#define QEM_CASE(L, N)                                                                                      \
    if (p.lpr == L && p.nch == N)                                                                           \
        return launch_bwd<T, VEC, N, L>(s, F, ut, m, wp, pidx, w, n, K, Kp, z, mone, d);
    QEM_ROW_PLANS(QEM_CASE)
#undef QEM_CASE
    return hipErrorInvalidValue;
}

template <typename T, int VEC, int NCH, int LPR>
hipError_t launch_chain(hipStream_t s, bool fwd, const void* F, double* ut, const void* m_in, void* m_out,
                        double* L, void* w, long G, int T_, int K, const double* g, double U) {
    const bool nt = static_cast<size_t>(G) * (T_ - 1) * K * K * sizeof(T) > STREAM_BYTES;
    if (fwd)
        hipLaunchKernelGGL((k_chain_fwd<T, VEC, NCH, LPR>), dim3(G), dim3(BLOCK), 0, s, (const T*)F, ut,
                           (double*)m_out, L, T_, K, nt, static_cast<T>(U));
    else
        hipLaunchKernelGGL((k_chain_bwd<T, VEC, NCH, LPR>), dim3(G), dim3(BLOCK), 0, s, (const T*)F,
                           (const double*)ut, (const double*)m_in, (const double*)L, (T*)w, T_, K, g, nt);
    return hipGetLastError();
}

template <typename T, int VEC>
hipError_t chain_plan(hipStream_t s, const RowPlan& p, bool fwd, const void* F, double* ut, const void* m_in,
                      void* m_out, double* L, void* w, long G, int T_, int K, const double* g, double U) {
#define QEM_CASE(L, N) \
    if (p.lpr == L && p.nch == N) return launch_chain<T, VEC, N, L>(s, fwd, F, ut, m_in, m_out, L_, w, G, T_, K, g, U);
    double* L_ = L;
    QEM_ROW_PLANS(QEM_CASE)
#undef QEM_CASE
    return hipErrorInvalidValue;
}

template <typename T, int VEC, int NCH, int LPR>
hipError_t launch_chain_pn(hipStream_t s, void* F, const void* z, double* ut, void* m, double* L, long G, int T_,
                           int K, double a, double b, double c0, double hp, const VSeries& vs) {
    const bool nt = static_cast<size_t>(G) * (T_ - 1) * K * K * sizeof(T) > STREAM_BYTES;
    hipLaunchKernelGGL((k_chain_fwd_pn<T, VEC, NCH, LPR>), dim3(G), dim3(BLOCK), 0, s, (T*)F, (const T*)z, ut,
                       (double*)m, L, T_, K, (T)a, (T)b, (T)c0, (T)hp, nt, vs);
    return hipGetLastError();
}

template <typename T, int VEC>
hipError_t chain_pn_plan(hipStream_t s, const RowPlan& p, void* F, const void* z, double* ut, void* m, double* L,
                         long G, int T_, int K, double a, double b, double c0, double hp, const VSeries& vs) {
#define QEM_CASE(LL, N) \
    if (p.lpr == LL && p.nch == N) return launch_chain_pn<T, VEC, N, LL>(s, F, z, ut, m, L, G, T_, K, a, b, c0, hp, vs);
    QEM_ROW_PLANS(QEM_CASE)
#undef QEM_CASE
    return hipErrorInvalidValue;
}

template <typename T, int VEC, int NCH, int LPR>
hipError_t launch_chain_bwd_pn(hipStream_t s, const void* z, const double* ut, const double* m, const double* L,
                               void* w, long G, int T_, int K, double a, double b, double c0, double hp,
                               const double* g, const VSeries& vs, bool renorm) {
    if (renorm)
        hipLaunchKernelGGL((k_chain_bwd_pn<T, VEC, NCH, LPR, true>), dim3(G), dim3(BLOCK), 0, s, (const T*)z, ut, m, L,
                           (T*)w, T_, K, (T)a, (T)b, (T)c0, (T)hp, g, vs);
    else
        hipLaunchKernelGGL((k_chain_bwd_pn<T, VEC, NCH, LPR, false>), dim3(G), dim3(BLOCK), 0, s, (const T*)z, ut, m, L,
                           (T*)w, T_, K, (T)a, (T)b, (T)c0, (T)hp, g, vs);
    return hipGetLastError();
}

template <typename T, int VEC>
hipError_t chain_bwd_pn_plan(hipStream_t s, const RowPlan& p, const void* z, const double* ut, const double* m,
                             const double* L, void* w, long G, int T_, int K, double a, double b, double c0,
                             double hp, const double* g, const VSeries& vs, bool renorm) {
#define QEM_CASE(LL, N)                                                                                         \
    if (p.lpr == LL && p.nch == N)                                                                              \
        return launch_chain_bwd_pn<T, VEC, N, LL>(s, z, ut, m, L, w, G, T_, K, a, b, c0, hp, g, vs, renorm);
    QEM_ROW_PLANS(QEM_CASE)
#undef QEM_CASE
    return hipErrorInvalidValue;
}

// One-wave instances of the recomputing plate backward pay off once there
// are enough instances to give every SIMD several waves.
constexpr long BWD_PN_ONE_WAVE_MIN = 4096;

template <typename T, int VEC, int NCH, int LPR, int D>
hipError_t launch_bwd_pn(hipStream_t s, const void* zc, const void* zp, const int32_t* pidx, const double* ut,
                         const double* m, const void* wp, void* w, long n, int K, int Kp, double a, double b,
                         double c0, double hp, double* mone) {
    if constexpr (NCH * VEC * D > 64) {
        return hipErrorInvalidValue;
    } else {
        if (K <= 128 && Kp <= 128 && n >= BWD_PN_ONE_WAVE_MIN) {
            // four instances per workgroup, one wave each
            const size_t sm = 4 * static_cast<size_t>(Kp) * D * sizeof(T);
            hipLaunchKernelGGL((k_plate_bwd_pn<T, VEC, NCH, LPR, D, 1>), dim3((n + 3) / 4), dim3(BLOCK), sm, s,
                               (const T*)zc, (const T*)zp, pidx, ut, m, (const T*)wp, (T*)w, n, K, Kp, (T)a, (T)b,
                               (T)c0, (T)hp, mone);
            return hipGetLastError();
        }
        const size_t sm = static_cast<size_t>(Kp) * D * sizeof(T);
        hipLaunchKernelGGL((k_plate_bwd_pn<T, VEC, NCH, LPR, D, 4>), dim3(n), dim3(BLOCK), sm, s, (const T*)zc,
                           (const T*)zp, pidx, ut, m, (const T*)wp, (T*)w, n, K, Kp, (T)a, (T)b, (T)c0, (T)hp, mone);
        return hipGetLastError();
    }
}

template <typename T, int VEC, int NCH, int LPR>
hipError_t bwd_pn_d(hipStream_t s, int d, const void* zc, const void* zp, const int32_t* pidx, const double* ut,
                    const double* m, const void* wp, void* w, long n, int K, int Kp, double a, double b, double c0,
                    double hp, double* mone) {
    switch (d) {
        case 1: return launch_bwd_pn<T, VEC, NCH, LPR, 1>(s, zc, zp, pidx, ut, m, wp, w, n, K, Kp, a, b, c0, hp, mone);
        case 2: return launch_bwd_pn<T, VEC, NCH, LPR, 2>(s, zc, zp, pidx, ut, m, wp, w, n, K, Kp, a, b, c0, hp, mone);
        case 3: return launch_bwd_pn<T, VEC, NCH, LPR, 3>(s, zc, zp, pidx, ut, m, wp, w, n, K, Kp, a, b, c0, hp, mone);
        case 4: return launch_bwd_pn<T, VEC, NCH, LPR, 4>(s, zc, zp, pidx, ut, m, wp, w, n, K, Kp, a, b, c0, hp, mone);
        case 8: return launch_bwd_pn<T, VEC, NCH, LPR, 8>(s, zc, zp, pidx, ut, m, wp, w, n, K, Kp, a, b, c0, hp, mone);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int VEC>
hipError_t bwd_pn_plan(hipStream_t s, const RowPlan& p, int d, const void* zc, const void* zp, const int32_t* pidx,
                       const double* ut, const double* m, const void* wp, void* w, long n, int K, int Kp, double a,
                       double b, double c0, double hp, double* mone) {
#define QEM_CASE(LL, N)                                                                                         \
    if (p.lpr == LL && p.nch == N)                                                                              \
        return bwd_pn_d<T, VEC, N, LL>(s, d, zc, zp, pidx, ut, m, wp, w, n, K, Kp, a, b, c0, hp, mone);
    QEM_ROW_PLANS(QEM_CASE)
#undef QEM_CASE
    return hipErrorInvalidValue;
}

hipError_t chain_any(hipStream_t s, bool f64, bool fwd, const void* F, double* ut, const void* m_in, void* m_out,
                     double* L, void* w, long G, int T_, int K, const double* g, double U) {
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    if (f64) {
        if (p.vec == 2) return chain_plan<double, 2>(s, p, fwd, F, ut, m_in, m_out, L, w, G, T_, K, g, U);
        return chain_plan<double, 1>(s, p, fwd, F, ut, m_in, m_out, L, w, G, T_, K, g, U);
    }
    if (p.vec == 4) return chain_plan<float, 4>(s, p, fwd, F, ut, m_in, m_out, L, w, G, T_, K, g, U);
    return chain_plan<float, 1>(s, p, fwd, F, ut, m_in, m_out, L, w, G, T_, K, g, U);
}

}  // namespace

hipError_t gather(hipStream_t s, bool f64, double* ut, const void* u, const ChildLists& cl, int n_par, int K) {
    if (cl.n > 0) {
        if (f64) hipLaunchKernelGGL(k_gather<double>, dim3(n_par), dim3(CS_BLOCK), 0, s, ut, (const double*)u, cl, K);
        else hipLaunchKernelGGL(k_gather<float>, dim3(n_par), dim3(CS_BLOCK), 0, s, ut, (const float*)u, cl, K);
        return hipGetLastError();
    }
    const long total = static_cast<long>(n_par) * K;
    const dim3 grid((total + BLOCK - 1) / BLOCK);
    if (f64) hipLaunchKernelGGL(k_ut_from_u<double>, grid, dim3(BLOCK), 0, s, ut, (const double*)u, total);
    else hipLaunchKernelGGL(k_ut_from_u<float>, grid, dim3(BLOCK), 0, s, ut, (const float*)u, total);
    return hipGetLastError();
}

hipError_t gather_finish(hipStream_t s, bool f64, double* ut, const void* u, int nl, int K, const double* part) {
    if (K > 1024 || nl < 1 || nl > MAX_CHILD_LISTS) return hipErrorInvalidValue;
    const dim3 grid((K + BLOCK - 1) / BLOCK);
    if (f64) hipLaunchKernelGGL(k_gather_finish<double>, grid, dim3(BLOCK), 0, s, ut, (const double*)u, nl, K, part);
    else hipLaunchKernelGGL(k_gather_finish<float>, grid, dim3(BLOCK), 0, s, ut, (const float*)u, nl, K, part);
    return hipGetLastError();
}

hipError_t gather_subsets(hipStream_t s, const ChildLists& cl, long q, int K, double* part) {
    if (cl.n < 1 || K < 1 || K > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather_subsets, dim3(cl.n * (1024 / K)), dim3(BLOCK), 0, s, cl, q, K, part);
    return hipGetLastError();
}

hipError_t root_fin(hipStream_t s, bool f64, const RootFinArgs& a) {
    if (f64) hipLaunchKernelGGL(k_root_fin<double>, dim3(1), dim3(CS_BLOCK), 0, s, a);
    else hipLaunchKernelGGL(k_root_fin<float>, dim3(1), dim3(CS_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fwd_q4(hipStream_t s, const void* F, const double* ut, void* m, long n, uint32_t* status) {
    const bool nt = static_cast<size_t>(n) * Q4_K * Q4_K * sizeof(float) > STREAM_BYTES;
    hipLaunchKernelGGL(k_plate_fwd_q4, dim3((n + BLOCK / WAVE - 1) / (BLOCK / WAVE)), dim3(BLOCK), 0, s,
                       (const float*)F, ut, (double*)m, n, nt, status);
    return hipGetLastError();
}

template <int D>
hipError_t launch_fwd_q4_pn(hipStream_t s, void* F, const void* zc, const void* zp, const int32_t* pidx,
                            double* ut, void* m, long n, double a, double b, double c0, double hp, const void* u,
                            const ChildLists* cl, uint32_t* status, const FwdSample* fs) {
    const bool nt = static_cast<size_t>(n) * Q4_K * Q4_K * sizeof(float) > STREAM_BYTES;
    const dim3 g4((n + BLOCK / WAVE - 1) / (BLOCK / WAVE));
    if (cl)
        hipLaunchKernelGGL((k_plate_fwd_q4_pn<D, true, false>), dim3(n), dim3(BLOCK), 0, s, (float*)F,
                           (const float*)zc, (const float*)zp, pidx, ut, (double*)m, n, (float)a, (float)b, (float)c0,
                           (float)hp, nt, (const float*)u, *cl, status, FwdSample{});
    else if (fs)
        hipLaunchKernelGGL((k_plate_fwd_q4_pn<D, false, true>), g4, dim3(BLOCK), 0, s, (float*)F, (const float*)zc,
                           (const float*)zp, pidx, ut, (double*)m, n, (float)a, (float)b, (float)c0, (float)hp, nt,
                           (const float*)nullptr, ChildLists{}, status, *fs);
    else
        hipLaunchKernelGGL((k_plate_fwd_q4_pn<D, false, false>), g4, dim3(BLOCK), 0, s, (float*)F, (const float*)zc,
                           (const float*)zp, pidx, ut, (double*)m, n, (float)a, (float)b, (float)c0, (float)hp, nt,
                           (const float*)nullptr, ChildLists{}, status, FwdSample{});
    return hipGetLastError();
}

hipError_t plate_fwd(hipStream_t s, bool f64, const void* F, const double* ut, void* m, long n, int Kp, int K,
                     uint32_t* status) {
    if (!f64 && q4_layout(K, Kp)) return launch_fwd_q4(s, F, ut, m, n, status);
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    if (f64)
        return p.vec == 2 ? fwd_plan<double, 2>(s, p, F, ut, m, n, K, Kp, status)
                          : fwd_plan<double, 1>(s, p, F, ut, m, n, K, Kp, status);
    return p.vec == 4 ? fwd_plan<float, 4>(s, p, F, ut, m, n, K, Kp, status)
                      : fwd_plan<float, 1>(s, p, F, ut, m, n, K, Kp, status);
}

bool plate_fwd_pn_supported(bool f64, int K, int Kp, int d) {
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    const int full = f64 ? 2 : 4;
    const bool dim_ok = d == 1 || d == 2 || d == 3 || d == 4 || d == 8;
    // the K = 64 FP32 layout keeps 16 child samples per lane: up to 4 dimensions
    if (!f64 && q4_layout(K, Kp) && d > 4) return false;
    return p.vec == full && dim_ok && p.nch * p.vec * d <= 64 && BLOCK / p.lpr <= Kp;
}

bool plate_fwd_samples_supported(bool f64, int K, int Kp, int d) {
    return !f64 && q4_layout(K, Kp) && d >= 1 && d <= 4;
}

hipError_t plate_fwd_pn(hipStream_t s, bool f64, void* F, const void* zc, const void* zp, const int32_t* pidx,
                        double* ut, void* m, long n, int Kp, int K, int d, double a, double b, double var,
                        const void* u, const ChildLists* cl, uint32_t* status, const FwdSample* fs) {
    if (!plate_fwd_pn_supported(f64, K, Kp, d)) return hipErrorInvalidValue;
    if (fs && (cl || !plate_fwd_samples_supported(f64, K, Kp, d) || fs->a.d != d || fs->a.K != K ||
               fs->a.n != n || fs->a.qfamily != QF_GAUSS))
        return hipErrorInvalidValue;
    if (cl) {
        if (!u || K > 512 || cl->n < 1 || cl->n > MAX_CHILD_LISTS) return hipErrorInvalidValue;
        // block_gather at BLOCK threads: at most 8 strided subsets per thread
        const int splits = 1024 / K, tpc = BLOCK / std::min(K, BLOCK);
        if ((splits + tpc - 1) / tpc > 8) return hipErrorInvalidValue;
    }
    double c0, hp;
    normal_pair_consts(d, var, &c0, &hp);
    if (!f64 && q4_layout(K, Kp)) {
        switch (d) {   // d <= 4 (plate_fwd_pn_supported)
            case 1: return launch_fwd_q4_pn<1>(s, F, zc, zp, pidx, ut, m, n, a, b, c0, hp, u, cl, status, fs);
            case 2: return launch_fwd_q4_pn<2>(s, F, zc, zp, pidx, ut, m, n, a, b, c0, hp, u, cl, status, fs);
            case 3: return launch_fwd_q4_pn<3>(s, F, zc, zp, pidx, ut, m, n, a, b, c0, hp, u, cl, status, fs);
            case 4: return launch_fwd_q4_pn<4>(s, F, zc, zp, pidx, ut, m, n, a, b, c0, hp, u, cl, status, fs);
            default: return hipErrorInvalidValue;
        }
    }
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    if (f64) return fwd_pn_plan<double, 2>(s, p, d, F, zc, zp, pidx, ut, m, n, K, Kp, a, b, c0, hp, u, cl, status);
    return fwd_pn_plan<float, 4>(s, p, d, F, zc, zp, pidx, ut, m, n, K, Kp, a, b, c0, hp, u, cl, status);
}

hipError_t plate_bwd(hipStream_t s, bool f64, const void* F, const double* ut, const void* m,
                     const void* wp, const int32_t* pidx, void* w, long n, int Kp, int K, const void* z,
                     double* mone, int d) {
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    if (f64) return p.vec == 2 ? bwd_plan<double, 2>(s, p, F, ut, m, wp, pidx, w, n, K, Kp, z, mone, d)
                               : bwd_plan<double, 1>(s, p, F, ut, m, wp, pidx, w, n, K, Kp, z, mone, d);
    return p.vec == 4 ? bwd_plan<float, 4>(s, p, F, ut, m, wp, pidx, w, n, K, Kp, z, mone, d)
                      : bwd_plan<float, 1>(s, p, F, ut, m, wp, pidx, w, n, K, Kp, z, mone, d);
}

hipError_t root_lse(hipStream_t s, const double* ut, double* L, long n, int K) {
    const long per = BLOCK / WAVE;
    hipLaunchKernelGGL(k_root_lse, dim3((n + per - 1) / per), dim3(BLOCK), 0, s, ut, L, n, K);
    return hipGetLastError();
}

hipError_t root_w(hipStream_t s, bool f64, const double* ut, const double* L, void* w, long n, int K,
                  const double* g) {
    const long total = n * K;
    const dim3 grid((total + BLOCK - 1) / BLOCK);
    if (f64) hipLaunchKernelGGL(k_root_w<double>, grid, dim3(BLOCK), 0, s, ut, L, (double*)w, n, K, g);
    else hipLaunchKernelGGL(k_root_w<float>, grid, dim3(BLOCK), 0, s, ut, L, (float*)w, n, K, g);
    return hipGetLastError();
}

hipError_t sum_L(hipStream_t s, const double* L, long nL, double* logphat, uint32_t* status) {
    hipLaunchKernelGGL(k_sum_L, dim3(1), dim3(BLOCK), 0, s, L, nL, logphat, status);
    return hipGetLastError();
}

hipError_t chain_fwd_pn(hipStream_t s, bool f64, void* F, const void* z, double* ut, void* m, double* L, long G,
                        int T, int K, double a, double b, double var, const VSeries& vs) {
    double c0, hp;
    normal_pair_consts(1, var, &c0, &hp);
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    const long nb = vs.Kb ? G * vs.Kb : G;
    if (f64) {
        if (p.vec == 2) return chain_pn_plan<double, 2>(s, p, F, z, ut, m, L, nb, T, K, a, b, c0, hp, vs);
        return chain_pn_plan<double, 1>(s, p, F, z, ut, m, L, nb, T, K, a, b, c0, hp, vs);
    }
    if (p.vec == 4) return chain_pn_plan<float, 4>(s, p, F, z, ut, m, L, nb, T, K, a, b, c0, hp, vs);
    return chain_pn_plan<float, 1>(s, p, F, z, ut, m, L, nb, T, K, a, b, c0, hp, vs);
}

hipError_t chain_bwd_pn(hipStream_t s, bool f64, const void* z, const double* ut, const double* m, const double* L,
                        void* w, long G, int T, int K, double a, double b, double var, const double* g,
                        const VSeries& vs, bool renorm) {
    double c0, hp;
    normal_pair_consts(1, var, &c0, &hp);
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    const long nb = vs.Kb ? G * vs.Kb : G;
    if (f64) {
        if (p.vec == 2) return chain_bwd_pn_plan<double, 2>(s, p, z, ut, m, L, w, nb, T, K, a, b, c0, hp, g, vs, renorm);
        return chain_bwd_pn_plan<double, 1>(s, p, z, ut, m, L, w, nb, T, K, a, b, c0, hp, g, vs, renorm);
    }
    if (p.vec == 4) return chain_bwd_pn_plan<float, 4>(s, p, z, ut, m, L, w, nb, T, K, a, b, c0, hp, g, vs, renorm);
    return chain_bwd_pn_plan<float, 1>(s, p, z, ut, m, L, w, nb, T, K, a, b, c0, hp, g, vs, renorm);
}

hipError_t chainp_wsum(hipStream_t s, bool f64, bool parts_f64, const void* vw, void* w, long G, int np, int T,
                       int K) {
    const long total = G * T * K;
    const long blocks = std::min((total + BLOCK - 1) / BLOCK, 65536L);
    if (f64)
        hipLaunchKernelGGL((k_chainp_wsum<double, double>), dim3(blocks), dim3(BLOCK), 0, s, (const double*)vw,
                           (double*)w, G, np, T, K);
    else if (parts_f64)
        hipLaunchKernelGGL((k_chainp_wsum<double, float>), dim3(blocks), dim3(BLOCK), 0, s, (const double*)vw,
                           (float*)w, G, np, T, K);
    else
        hipLaunchKernelGGL((k_chainp_wsum<float, float>), dim3(blocks), dim3(BLOCK), 0, s, (const float*)vw,
                           (float*)w, G, np, T, K);
    return hipGetLastError();
}

hipError_t plate_bwd_pn(hipStream_t s, bool f64, const void* zc, const void* zp, const int32_t* pidx,
                        const double* ut, const double* m, const void* wp, void* w, long n, int Kp, int K, int d,
                        double a, double b, double var, double* mone) {
    if (!plate_fwd_pn_supported(f64, K, Kp, d)) return hipErrorInvalidValue;
    double c0, hp;
    normal_pair_consts(d, var, &c0, &hp);
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    if (f64) return bwd_pn_plan<double, 2>(s, p, d, zc, zp, pidx, ut, m, wp, w, n, K, Kp, a, b, c0, hp, mone);
    return bwd_pn_plan<float, 4>(s, p, d, zc, zp, pidx, ut, m, wp, w, n, K, Kp, a, b, c0, hp, mone);
}

hipError_t chain_fwd(hipStream_t s, bool f64, const void* F, double* ut, void* m, double* L,
                     long G, int T, int K, double var) {
    // the entries' bound: c0 of the step factor, in the precision the
    // recomputing kernel receives it
    double c0, hp;
    normal_pair_consts(1, var, &c0, &hp);
    return chain_any(s, f64, true, F, ut, nullptr, m, L, nullptr, G, T, K, nullptr, c0);
}

hipError_t chain_bwd(hipStream_t s, bool f64, const void* F, const double* ut, const void* m,
                     const double* L, void* w, long G, int T, int K, const double* g) {
    return chain_any(s, f64, false, F, const_cast<double*>(ut), m, nullptr, const_cast<double*>(L), w, G, T, K, g, 0.0);
}

}  // namespace qemk
