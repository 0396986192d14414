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

template <typename T, int VEC, int NCH>
__device__ __forceinline__ void load_row_plus(const T* __restrict__ row, const double* __restrict__ ut, double shift,
                                              int K, int lane, int lpr, T (&v)[NCH * VEC], bool nt) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int e0 = (c * lpr + lane) * VEC;
        if (e0 < K) {
            T f[VEC];
            load_vec_hint<T, VEC>(row + e0, f, nt);
#pragma unroll
            for (int q = 0; q < VEC; ++q) v[c * VEC + q] = f[q] + static_cast<T>(ut[e0 + q] - shift);
        } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) v[c * VEC + q] = neg_inf<T>();
        }
    }
}

template <typename T, int N>
__device__ __forceinline__ T lse_group(const T (&v)[N], int lpr) {
    T mx = v[0];
#pragma unroll
    for (int q = 1; q < N; ++q) mx = fmax(mx, v[q]);
    mx = group_max(mx, lpr);
    if (mx == neg_inf<T>()) return mx;   // uniform across the group
    T s = 0;
#pragma unroll
    for (int q = 0; q < N; ++q) s += fexp(v[q] - mx);
    s = group_sum(s, lpr);
    return mx + flog(s);
}

// ---------------------------------------------------------------- kernels

__global__ void __launch_bounds__(BLOCK) k_child_sum_f64(double* __restrict__ ut, const double* __restrict__ u,
                                                         const double* __restrict__ mc, const int32_t* __restrict__ off,
                                                         const int32_t* __restrict__ idx, int n_par, int K) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<long>(n_par) * K) return;
    const long q = t / K, k = t % K;
    double acc = u ? u[t] : ut[t];
    if (mc) for (int j = off[q]; j < off[q + 1]; ++j) acc += mc[static_cast<long>(idx[j]) * K + k];
    ut[t] = acc;
}

__global__ void __launch_bounds__(BLOCK) k_child_sum_f32(double* __restrict__ ut, const float* __restrict__ u,
                                                         const double* __restrict__ mc, const int32_t* __restrict__ off,
                                                         const int32_t* __restrict__ idx, int n_par, int K) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<long>(n_par) * K) return;
    const long q = t / K, k = t % K;
    double acc = u ? static_cast<double>(u[t]) : ut[t];
    if (mc) for (int j = off[q]; j < off[q + 1]; ++j) acc += mc[static_cast<long>(idx[j]) * K + k];
    ut[t] = acc;
}

// Parents with children: one workgroup per parent instance; the children of
// the instance are split over CS_BLOCK / K thread groups, each summing a
// strided subset in index order, then the groups are added in a fixed order.
constexpr int CS_BLOCK = 1024;

template <typename T>
__global__ void __launch_bounds__(CS_BLOCK) k_child_sum_par(double* __restrict__ ut, const T* __restrict__ u,
                                                            const double* __restrict__ mc, const int32_t* __restrict__ off,
                                                            const int32_t* __restrict__ idx, int K) {
    __shared__ double red[CS_BLOCK];
    const long q = blockIdx.x;
    const int cols = K < CS_BLOCK ? K : CS_BLOCK;
    const int splits = CS_BLOCK / cols;
    const int tk = threadIdx.x % cols, sp = threadIdx.x / cols;
    const int j0 = off[q], j1 = off[q + 1];
    for (int k0 = 0; k0 < K; k0 += cols) {
        const int k = k0 + tk;
        double acc = 0.0;
        if (sp < splits && k < K) {
#pragma unroll 8
            for (int j = j0 + sp; j < j1; j += splits) acc += mc[static_cast<long>(idx[j]) * K + k];
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        if (sp == 0 && k < K) {
            double sum = u ? static_cast<double>(u[q * K + k]) : ut[q * K + k];
            for (int p = 0; p < splits; ++p) sum += red[p * cols + tk];
            ut[q * K + k] = sum;
        }
        __syncthreads();
    }
}

// A workgroup covers ipb consecutive instances (ipb*Kp rows of F).  It first
// stages each instance's shift c_i = max_k ut[i,k] and ut[i,:] - c_i (in T)
// in LDS; then groups of lpr lanes take RPI rows at a time, loading all of
// them before reducing any.
template <typename T, int VEC, int NCH, int RPI>
__global__ void __launch_bounds__(BLOCK) k_plate_fwd(const T* __restrict__ F, const double* __restrict__ ut,
                                                     double* __restrict__ m, long n, int K, int Kp, int lpr,
                                                     int ipb, int kp_shift, bool nt) {
    extern __shared__ unsigned char smem_raw[];
    double* s_sh = reinterpret_cast<double*>(smem_raw);      // [ipb]
    T* s_u = reinterpret_cast<T*>(s_sh + ipb);               // [ipb, K]
    const int lane = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int gpb = BLOCK / lpr;
    const int wl = threadIdx.x & (WAVE - 1);
    const long i0 = static_cast<long>(blockIdx.x) * ipb;
    const int ni = static_cast<int>(std::min(static_cast<long>(ipb), n - i0));
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
    const int nr = ni * Kp;
    const T* Fb = F + i0 * Kp * K;
    double* mb = m + i0 * Kp;
    for (int rb0 = 0; rb0 < nr; rb0 += gpb * RPI) {
        T v[RPI][NCH * VEC];
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
            if (lane == 0 && row < nr)
                mb[row] = (res == neg_inf<T>()) ? -__builtin_inf() : s_sh[li] + static_cast<double>(res);
        }
    }
}

// One workgroup per instance; lanes along k, row groups along kp.
template <typename T, int VEC, int NCH>
__global__ void __launch_bounds__(BLOCK) k_plate_bwd(const T* __restrict__ F, const double* __restrict__ ut,
                                                     const double* __restrict__ m, const T* __restrict__ wp,
                                                     const int32_t* __restrict__ pidx, T* __restrict__ w,
                                                     int K, int Kp, int lpr, bool nt, const T* __restrict__ z,
                                                     double* __restrict__ mone, int d) {
    __shared__ T red[BLOCK / WAVE][512];
    __shared__ T s_m[512], s_wp[512];
    __shared__ double s_scr[BLOCK / WAVE];
    const int lane = threadIdx.x & (lpr - 1);
    const int grp = threadIdx.x / lpr;
    const int ngrp = BLOCK / lpr;
    const long i = blockIdx.x;
    const long p = pidx ? pidx[i] : 0;
    const double sh = finite_or_zero(block_max(ut + i * K, K, s_scr));
    for (int kp = threadIdx.x; kp < Kp; kp += BLOCK) {
        s_m[kp] = static_cast<T>(m[i * Kp + kp] - sh);
        s_wp[kp] = wp[p * Kp + kp];
    }
    __syncthreads();
    T utv[NCH * VEC], acc[NCH * VEC];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int e0 = (c * lpr + lane) * VEC;
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            utv[c * VEC + q] = (e0 < K) ? static_cast<T>(ut[i * K + e0 + q] - sh) : T(0);
            acc[c * VEC + q] = 0;
        }
    }
    const T* tile = F + i * static_cast<long>(Kp) * K;
#pragma unroll 4
    for (int kp = grp; kp < Kp; kp += ngrp) {
        const T wk = s_wp[kp];
        const T mk = s_m[kp];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e0 = (c * lpr + lane) * VEC;
            if (e0 < K) {
                T f[VEC];
                load_vec_hint<T, VEC>(tile + static_cast<long>(kp) * K + e0, f, nt);
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    const T e = fexp(f[q] + utv[c * VEC + q] - mk);
                    acc[c * VEC + q] += (wk > T(0)) ? wk * e : T(0);
                }
            }
        }
    }
    // reduce over the row groups of a wave, then over waves in a fixed order
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
        w[i * K + k] = s;
        s_m[k] = s;   // the messages are no longer needed: keep the weights
    }
    if (!mone) return;
    __syncthreads();
    const int wl = threadIdx.x & (WAVE - 1);
    for (int j = threadIdx.x / WAVE; j < d; j += BLOCK / WAVE) {
        double s1 = 0.0, s2 = 0.0;
        for (int k = wl; k < K; k += WAVE) {
            const double wk = static_cast<double>(s_m[k]);
            const double zk = static_cast<double>(z[(i * K + k) * d + j]);
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

// One wave per instance.
__global__ void __launch_bounds__(BLOCK) k_root_lse(const double* __restrict__ ut, double* __restrict__ L, long n, int K) {
    const long i = static_cast<long>(blockIdx.x) * (BLOCK / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (i >= n) return;
    double mx = -__builtin_inf();
    for (int k = lane; k < K; k += WAVE) mx = fmax(mx, ut[i * K + k]);
    mx = group_max(mx, WAVE);
    double s = 0.0;
    if (mx != -__builtin_inf())
        for (int k = lane; k < K; k += WAVE) s += exp(ut[i * K + k] - mx);
    s = group_sum(s, WAVE);
    if (lane == 0) L[i] = (mx == -__builtin_inf()) ? mx : mx + log(s);
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

// Single workgroup: strided partial sums in index order, then a fixed tree.
__global__ void __launch_bounds__(BLOCK) k_sum_L(const double* __restrict__ L, long nL, double* __restrict__ out,
                                                 uint32_t* __restrict__ status) {
    __shared__ double red[BLOCK];
    double s = 0.0;
    for (long j = threadIdx.x; j < nL; j += BLOCK) s += L[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = red[0];
        *out = v;
        if (!isfinite(v)) atomicOr(status, 0x1u);
    }
}

// ---------------------------------------------------------------- chains
// One workgroup per series g; steps t = T-1 .. 1 are eliminated in order.
// ut[g*T + t, :] holds u plus child messages on entry; on exit it holds the
// full u-tilde of every step (needed by the reverse pass).

template <typename T, int VEC, int NCH>
__global__ void __launch_bounds__(BLOCK) k_chain_fwd(const T* __restrict__ F, double* __restrict__ ut,
                                                     double* __restrict__ m, double* __restrict__ L,
                                                     int T_, int K, int lpr, bool nt) {
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
        const T* Ft = F + (g * (T_ - 1) + (t - 1)) * tileKK;
        for (int kp0 = 0; kp0 < K; kp0 += ngrp * 2) {
            T v[2][NCH * VEC];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int kp = kp0 + r * ngrp + grp;
                if (kp < K) load_row_plus<T, VEC, NCH>(Ft + static_cast<long>(kp) * K, s_ut, sh, K, lane, lpr, v[r], nt);
                else {
#pragma unroll
                    for (int q = 0; q < NCH * VEC; ++q) v[r][q] = neg_inf<T>();
                }
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int kp = kp0 + r * ngrp + grp;
                const T res = lse_group<T, NCH * VEC>(v[r], lpr);
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

template <typename T, int VEC, int NCH>
__global__ void __launch_bounds__(BLOCK) k_chain_bwd(const T* __restrict__ F, const double* __restrict__ ut,
                                                     const double* __restrict__ m, const double* __restrict__ L,
                                                     T* __restrict__ w, int T_, int K, int lpr,
                                                     const double* __restrict__ gsc, bool nt) {
    __shared__ T s_w[512];
    __shared__ T red[BLOCK / WAVE][512];
    __shared__ double s_scr[BLOCK / WAVE];
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
        const double sh = finite_or_zero(block_max(utt, K, s_scr));
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
            const T wk = s_w[kp];
            const T mk = static_cast<T>(mt[kp] - sh);
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int e0 = (c * lpr + lane) * VEC;
                if (e0 < K) {
                    T f[VEC];
                    load_vec_hint<T, VEC>(Ft + static_cast<long>(kp) * K + e0, f, nt);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) {
                        const T e = fexp(f[q] + utv[c * VEC + q] - mk);
                        acc[c * VEC + q] += (wk > T(0)) ? wk * e : T(0);
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

// ---------------------------------------------------------------- dispatch

template <typename T, int VEC, int NCH>
hipError_t launch_fwd(hipStream_t s, const void* F, const double* ut, void* m, long n, int K, int Kp, int lpr) {
    constexpr int RPI = (NCH <= 2) ? 4 : 2;
    const int rows_per_pass = (BLOCK / lpr) * RPI;
    const int ipb = std::max(1, rows_per_pass / Kp);
    const int kp_shift = (Kp & (Kp - 1)) == 0 ? __builtin_ctz(static_cast<unsigned>(Kp)) : -1;
    const dim3 grid((n + ipb - 1) / ipb);
    const size_t sm = static_cast<size_t>(ipb) * (8 + static_cast<size_t>(K) * sizeof(T));
    const bool nt = static_cast<size_t>(n) * Kp * K * sizeof(T) > STREAM_BYTES;
    hipLaunchKernelGGL((k_plate_fwd<T, VEC, NCH, RPI>), grid, dim3(BLOCK), sm, s, (const T*)F, ut, (double*)m, n, K,
                       Kp, lpr, ipb, kp_shift, nt);
    return hipGetLastError();
}

template <typename T, int VEC>
hipError_t fwd_nch(hipStream_t s, const RowPlan& p, const void* F, const double* ut, void* m, long R, int K, int Kp) {
    switch (p.nch) {
        case 1: return launch_fwd<T, VEC, 1>(s, F, ut, m, R, K, Kp, p.lpr);
        case 2: return launch_fwd<T, VEC, 2>(s, F, ut, m, R, K, Kp, p.lpr);
        case 4: return launch_fwd<T, VEC, 4>(s, F, ut, m, R, K, Kp, p.lpr);
        case 8: return launch_fwd<T, VEC, 8>(s, F, ut, m, R, K, Kp, p.lpr);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int VEC, int NCH>
hipError_t launch_bwd(hipStream_t s, const void* F, const double* ut, const void* m, const void* wp,
                      const int32_t* pidx, void* w, long n, int K, int Kp, int lpr, const void* z, double* mone,
                      int d) {
    const bool nt = static_cast<size_t>(n) * Kp * K * sizeof(T) > STREAM_BYTES;
    hipLaunchKernelGGL((k_plate_bwd<T, VEC, NCH>), dim3(n), dim3(BLOCK), 0, s, (const T*)F, ut, (const double*)m,
                       (const T*)wp, pidx, (T*)w, K, Kp, lpr, nt, (const T*)z, mone, d);
    return hipGetLastError();
}

template <typename T, int VEC>
hipError_t bwd_nch(hipStream_t s, const RowPlan& p, const void* F, const double* ut, const void* m, const void* wp,
                   const int32_t* pidx, void* w, long n, int K, int Kp, const void* z, double* mone, int d) {
    switch (p.nch) {
        case 1: return launch_bwd<T, VEC, 1>(s, F, ut, m, wp, pidx, w, n, K, Kp, p.lpr, z, mone, d);
        case 2: return launch_bwd<T, VEC, 2>(s, F, ut, m, wp, pidx, w, n, K, Kp, p.lpr, z, mone, d);
        case 4: return launch_bwd<T, VEC, 4>(s, F, ut, m, wp, pidx, w, n, K, Kp, p.lpr, z, mone, d);
        case 8: return launch_bwd<T, VEC, 8>(s, F, ut, m, wp, pidx, w, n, K, Kp, p.lpr, z, mone, d);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int VEC, int NCH>
hipError_t launch_chain(hipStream_t s, bool fwd, const void* F, double* ut, const void* m_in, void* m_out,
                        double* L, void* w, long G, int T_, int K, int lpr, const double* g) {
    const bool nt = static_cast<size_t>(G) * (T_ - 1) * K * K * sizeof(T) > STREAM_BYTES;
    if (fwd)
        hipLaunchKernelGGL((k_chain_fwd<T, VEC, NCH>), dim3(G), dim3(BLOCK), 0, s, (const T*)F, ut, (double*)m_out, L, T_,
                           K, lpr, nt);
    else
        hipLaunchKernelGGL((k_chain_bwd<T, VEC, NCH>), dim3(G), dim3(BLOCK), 0, s, (const T*)F, (const double*)ut,
                           (const double*)m_in, (const double*)L, (T*)w, T_, K, lpr, g, nt);
    return hipGetLastError();
}

template <typename T, int VEC>
hipError_t chain_nch(hipStream_t s, const RowPlan& p, bool fwd, const void* F, double* ut, const void* m_in,
                     void* m_out, double* L, void* w, long G, int T_, int K, const double* g) {
    switch (p.nch) {
        case 1: return launch_chain<T, VEC, 1>(s, fwd, F, ut, m_in, m_out, L, w, G, T_, K, p.lpr, g);
        case 2: return launch_chain<T, VEC, 2>(s, fwd, F, ut, m_in, m_out, L, w, G, T_, K, p.lpr, g);
        case 4: return launch_chain<T, VEC, 4>(s, fwd, F, ut, m_in, m_out, L, w, G, T_, K, p.lpr, g);
        case 8: return launch_chain<T, VEC, 8>(s, fwd, F, ut, m_in, m_out, L, w, G, T_, K, p.lpr, g);
        default: return hipErrorInvalidValue;
    }
}

hipError_t chain_any(hipStream_t s, bool f64, bool fwd, const void* F, double* ut, const void* m_in, void* m_out,
                     double* L, void* w, long G, int T_, int K, const double* g) {
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    if (f64) {
        if (p.vec == 2) return chain_nch<double, 2>(s, p, fwd, F, ut, m_in, m_out, L, w, G, T_, K, g);
        return chain_nch<double, 1>(s, p, fwd, F, ut, m_in, m_out, L, w, G, T_, K, g);
    }
    if (p.vec == 4) return chain_nch<float, 4>(s, p, fwd, F, ut, m_in, m_out, L, w, G, T_, K, g);
    return chain_nch<float, 1>(s, p, fwd, F, ut, m_in, m_out, L, w, G, T_, K, g);
}

}  // namespace

hipError_t child_sum(hipStream_t s, bool f64, double* ut, const void* u, const void* mc,
                     const int32_t* off, const int32_t* idx, int n_par, int K) {
    if (mc) {
        if (f64) hipLaunchKernelGGL(k_child_sum_par<double>, dim3(n_par), dim3(CS_BLOCK), 0, s, ut, (const double*)u,
                                    (const double*)mc, off, idx, K);
        else hipLaunchKernelGGL(k_child_sum_par<float>, dim3(n_par), dim3(CS_BLOCK), 0, s, ut, (const float*)u,
                                (const double*)mc, off, idx, K);
        return hipGetLastError();
    }
    const long total = static_cast<long>(n_par) * K;
    const dim3 grid((total + BLOCK - 1) / BLOCK);
    if (f64) hipLaunchKernelGGL(k_child_sum_f64, grid, dim3(BLOCK), 0, s, ut, (const double*)u, (const double*)mc, off, idx, n_par, K);
    else hipLaunchKernelGGL(k_child_sum_f32, grid, dim3(BLOCK), 0, s, ut, (const float*)u, (const double*)mc, off, idx, n_par, K);
    return hipGetLastError();
}

hipError_t plate_fwd(hipStream_t s, bool f64, const void* F, const double* ut, void* m, long n, int Kp, int K) {
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    if (f64) return p.vec == 2 ? fwd_nch<double, 2>(s, p, F, ut, m, n, K, Kp) : fwd_nch<double, 1>(s, p, F, ut, m, n, K, Kp);
    return p.vec == 4 ? fwd_nch<float, 4>(s, p, F, ut, m, n, K, Kp) : fwd_nch<float, 1>(s, p, F, ut, m, n, K, Kp);
}

hipError_t plate_bwd(hipStream_t s, bool f64, const void* F, const double* ut, const void* m,
                     const void* wp, const int32_t* pidx, void* w, long n, int Kp, int K, const void* z,
                     double* mone, int d) {
    const RowPlan p = plan_rows(K, f64 ? 8 : 4);
    if (f64) return p.vec == 2 ? bwd_nch<double, 2>(s, p, F, ut, m, wp, pidx, w, n, K, Kp, z, mone, d)
                               : bwd_nch<double, 1>(s, p, F, ut, m, wp, pidx, w, n, K, Kp, z, mone, d);
    return p.vec == 4 ? bwd_nch<float, 4>(s, p, F, ut, m, wp, pidx, w, n, K, Kp, z, mone, d)
                      : bwd_nch<float, 1>(s, p, F, ut, m, wp, pidx, w, n, K, Kp, z, mone, d);
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

hipError_t chain_fwd(hipStream_t s, bool f64, const void* F, double* ut, void* m, double* L,
                     long G, int T, int K) {
    return chain_any(s, f64, true, F, ut, nullptr, m, L, nullptr, G, T, K, nullptr);
}

hipError_t chain_bwd(hipStream_t s, bool f64, const void* F, const double* ut, const void* m,
                     const double* L, void* w, long G, int T, int K, const double* g) {
    return chain_any(s, f64, false, F, const_cast<double*>(ut), m, nullptr, const_cast<double*>(L), w, G, T, K, g);
}

}  // namespace qemk
