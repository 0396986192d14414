// Device pieces of the elimination's root level and of the closing M-step,
// shared by the one-purpose kernels of the stage calls and by the fused
// kernels of the iteration pipeline, so that both produce the same bits:
//   block_gather    ut[q,:] = u[q,:] + the messages of q's child instances
//   wave_lse        LSE of a row of FP64 log-weights, one wave
//   block_sum       the log P_MP sum over components
//   moment_sums     sum_k w (z, z^2), or (z, log z), of one (instance, dimension), index order
//   mstep_entry     EMA of the mean parameters and the closed-form Q update
//   digamma_d, trigamma_d, ef_gamma_shape   the exponential-family Gamma M-step
#pragma once
#include "qem_internal.h"
#include "dev_common.h"

namespace qemk {

constexpr double VAR_FLOOR = 1e-12;
constexpr double EF_GAP_FLOOR = 1e-12;   // floor of log m1 - m2 (exponential-family Gamma)

// psi(x) for x > 0 in FP64: psi(x) = psi(x + 1) - 1/x up to x >= 10, then the
// asymptotic series ln x - 1/(2x) - sum_n B_2n / (2n x^2n) (Abramowitz and
// Stegun 6.3.18) through B_14; the first omitted term is below 5e-17 at x = 10.
// The recurrence terms are summed as one fraction num/den (adding 1/y gives
// (num y + den) / (den y)), so the at most ten steps take one division.
__device__ __forceinline__ double digamma_d(double x) {
    double num = 0.0, den = 1.0;
    while (x < 10.0) {
        num = num * x + den;
        den *= x;
        x += 1.0;
    }
    const double r = -(num / den);
    const double f = 1.0 / (x * x);
    const double t = f * (-1.0 / 12 + f * (1.0 / 120 + f * (-1.0 / 252 + f * (1.0 / 240 + f * (-1.0 / 132 +
                     f * (691.0 / 32760 + f * (-1.0 / 12)))))));
    return r + log(x) - 0.5 / x + t;
}

// psi'(x) for x > 0: psi'(x) = psi'(x + 1) + 1/x^2 up to x >= 10, then
// 1/x + 1/(2x^2) + sum_n B_2n / x^(2n+1) (Abramowitz and Stegun 6.4.12).
// The recurrence terms are summed as one fraction, as in digamma_d.
__device__ __forceinline__ double trigamma_d(double x) {
    double num = 0.0, den = 1.0;
    while (x < 10.0) {
        const double y2 = x * x;
        num = num * y2 + den;
        den *= y2;
        x += 1.0;
    }
    const double r = num / den;
    const double f = 1.0 / (x * x);
    const double t = 1.0 / 6 + f * (-1.0 / 30 + f * (1.0 / 42 + f * (-1.0 / 30 + f * (5.0 / 66 +
                     f * (-691.0 / 2730 + f * (7.0 / 6))))));
    return r + 1.0 / x + 0.5 * f + t * f / x;
}

// log a - psi(a), without the cancellation of the two logarithms for large a:
// from a >= 10 the series 1/(2a) + sum_n B_2n / (2n a^2n).
__device__ __forceinline__ double log_minus_digamma(double a) {
    if (a < 10.0) return log(a) - digamma_d(a);
    const double f = 1.0 / (a * a);
    const double t = f * (1.0 / 12 + f * (-1.0 / 120 + f * (1.0 / 252 + f * (-1.0 / 240 + f * (1.0 / 132 +
                     f * (-691.0 / 32760 + f * (1.0 / 12)))))));
    return 0.5 / a + t;
}

// The shape a of the Gamma with log a - psi(a) = gap > 0, i.e. the one whose
// mean parameters (E z, E log z) have log E z - E log z = gap: Minka's
// closed-form start and his Newton iteration on 1/a ("Estimating a Gamma
// distribution", 2002), a fixed 12 steps (converged to FP64 after about 5).
__device__ __forceinline__ double ef_gamma_shape(double gap) {
    double a = (3.0 - gap + sqrt((gap - 3.0) * (gap - 3.0) + 24.0 * gap)) / (12.0 * gap);
    for (int it = 0; it < 12; ++it) {
        const double g = log_minus_digamma(a) - gap;
        const double dg = 1.0 / a - trigamma_d(a);
        const double inv = 1.0 / a + g / (a * a * dg);
        if (inv > 0.0) a = 1.0 / inv;
    }
    return a;
}

// a + mc[row(0) K + k] + mc[row(1) K + k] + ... (n rows, added in that
// order), row(t) = rows[t stride], or r0 + t stride when rows is null (a
// child list that holds the children of every parent in index order).  The
// loads of a batch are issued before any of them is added, so a wave has a
// batch of misses in flight rather than one.
__device__ __forceinline__ double sum_rows_in_order(double a, const double* __restrict__ mc,
                                                    const int32_t* rows, long r0, int n, int stride, int K, int k) {
    constexpr int B = 16;
    int t = 0;
    for (; t + B <= n; t += B) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const long row = rows ? static_cast<long>(rows[(t + u) * stride]) : r0 + static_cast<long>(t + u) * stride;
            v[u] = mc[row * K + k];
        }
#pragma unroll
        for (int u = 0; u < B; ++u) a += v[u];
    }
    for (; t < n; ++t) {
        const long row = rows ? static_cast<long>(rows[t * stride]) : r0 + static_cast<long>(t) * stride;
        a += mc[row * K + k];
    }
    return a;
}

// The children of parent instance q are split into S = 1024 / K strided
// subsets (subset p: children j0 + p, j0 + p + S, ... in index order); the
// subset sums are added to the running row in subset order, list after list.
// The child indices are staged in LDS a chunk at a time, so the message loads
// of a subset do not wait on each other; a list with cl.per set (every parent
// has cl.per children, in index order) needs neither its offsets nor its
// indices, and its message loads go out at once.  Every thread of the block calls
// it; s_ut [K], red [1024] (doubles) and s_idx [1024] (ints) are LDS.  The
// result does not depend on the block size (any multiple of 64 up to 1024).
template <typename BaseT>
__device__ void block_gather(double* s_ut, const BaseT* __restrict__ base, const ChildLists& cl, long q, int K,
                             double* red, int32_t* s_idx) {
    constexpr int RMAX = 8;   // subsets per thread: ceil(S / (blockDim / min(K, blockDim))) <= 8
    for (int k = threadIdx.x; k < K; k += blockDim.x) s_ut[k] = static_cast<double>(base[q * K + k]);
    const int splits = 1024 / K;
    const int chunk = splits * (1024 / splits);
    const int cols = K < static_cast<int>(blockDim.x) ? K : static_cast<int>(blockDim.x);
    const int tpc = blockDim.x / cols;
    const int tk = threadIdx.x % cols, sp = threadIdx.x / cols;
    for (int c = 0; c < cl.n; ++c) {
        const int per = cl.per[c];
        const int j0 = per ? static_cast<int>(q) * per : cl.off[c][q];
        const int j1 = per ? j0 + per : cl.off[c][q + 1];
        const double* __restrict__ mc = cl.mc[c];
        for (int k0 = 0; k0 < K; k0 += cols) {
            const int k = k0 + tk;
            const bool active = sp < tpc && k < K;
            double acc[RMAX];
#pragma unroll
            for (int r = 0; r < RMAX; ++r) acc[r] = 0.0;
            for (int cb = j0; cb < j1; cb += chunk) {
                const int ce = cb + chunk < j1 ? cb + chunk : j1;
                if (!per) {
                    __syncthreads();
                    for (int e = threadIdx.x; e < ce - cb; e += blockDim.x) s_idx[e] = cl.idx[c][cb + e];
                    __syncthreads();
                }
                if (active) {
#pragma unroll
                    for (int r = 0; r < RMAX; ++r) {
                        const int p = sp + r * tpc;
                        if (p < splits && p < ce - cb) {
                            const int nr = (ce - cb - p + splits - 1) / splits;
                            acc[r] = sum_rows_in_order(acc[r], mc, per ? nullptr : s_idx + p, cb + p, nr, splits,
                                                       K, k);
                        }
                    }
                }
            }
            if (active) {
#pragma unroll
                for (int r = 0; r < RMAX; ++r) {
                    const int p = sp + r * tpc;
                    if (p < splits) red[p * cols + tk] = acc[r];
                }
            }
            __syncthreads();
            if (sp == 0 && k < K) {
                double sum = s_ut[k];
                for (int p = 0; p < splits; ++p) sum += red[p * cols + tk];
                s_ut[k] = sum;
            }
            __syncthreads();
        }
    }
    __syncthreads();
}

// LSE_k row[k] by one wave (lanes strided over k); every lane gets it.
__device__ __forceinline__ double wave_lse(const double* row, int K) {
    const int lane = threadIdx.x & (WAVE - 1);
    double mx = -__builtin_inf();
    for (int k = lane; k < K; k += WAVE) mx = fmax(mx, row[k]);
    mx = group_max(mx, WAVE);
    double s = 0.0;
    if (mx != -__builtin_inf())
        for (int k = lane; k < K; k += WAVE) s += exp(row[k] - mx);
    s = group_sum(s, WAVE);
    return (mx == -__builtin_inf()) ? mx : mx + log(s);
}

// sum_j L[j] by the first BLOCK threads of a workgroup: strided partial sums
// in index order, then a fixed tree.  Every thread calls it; the result is
// valid in thread 0.  red: LDS of BLOCK doubles.
__device__ __forceinline__ double block_sum(const double* L, long nL, double* red) {
    if (threadIdx.x < BLOCK) {
        double s = 0.0;
        for (long j = threadIdx.x; j < nL; j += BLOCK) s += L[j];
        red[threadIdx.x] = s;
    }
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    return red[0];
}

// (sum_k w z, sum_k w z^2) of one instance, dimension j, in index order, or
// (sum_k w z, sum_k w log z) when logz (exponential-family Gamma);
// zrow = the instance's [K, d] samples, wrow = its K weights (global or LDS).
template <typename T>
__device__ __forceinline__ void moment_sums(const T* zrow, const T* wrow, int j, int K, int d, double& s1,
                                            double& s2, bool logz = false) {
    s1 = 0.0;
    s2 = 0.0;
    if (logz) {
        for (int k = 0; k < K; ++k) {
            const double wk = static_cast<double>(wrow[k]);
            const double zk = static_cast<double>(zrow[k * d + j]);
            s1 += wk * zk;
            s2 += wk * log(zk);
        }
        return;
    }
#pragma unroll 8
    for (int k = 0; k < K; ++k) {
        const double wk = static_cast<double>(wrow[k]);
        const double zk = static_cast<double>(zrow[k * d + j]);
        s1 += wk * zk;
        s2 += wk * zk * zk;
    }
}

// M-step of mean-parameter entry t (instance-dimension) from its previous
// mean parameters (m1, m2) and this iteration's moments (o1, o2): EMA
// (skipped when `skip`, i.e. log P_MP was not finite), then the closed-form
// Q parameters.
__device__ __forceinline__ void mstep_update(double* __restrict__ mema, double* __restrict__ qp, long t, double m1,
                                             double m2, double o1, double o2, int qfamily, double lam, bool skip,
                                             uint32_t* __restrict__ status) {
    if (lam != 0.0 && !skip) {
        m1 = (1.0 - lam) * m1 + lam * o1;
        m2 = (1.0 - lam) * m2 + lam * o2;
        mema[t * 2] = m1;
        mema[t * 2 + 1] = m2;
    }
    if (qfamily == QF_GAMMA_EF) {
        // mean parameters (E z, E log z): shape from log a - psi(a) = log m1 - m2
        if (!(m1 > 0.0)) {
            atomicOr(status, 0x4u);
            return;
        }
        const double gap = log(m1) - m2;
        if (gap < EF_GAP_FLOOR) {
            atomicAdd(status + 1, 1u);
            atomicOr(status, 0x2u);
        }
        const double a = ef_gamma_shape(fmax(gap, EF_GAP_FLOOR));
        qp[t * 2] = a;
        qp[t * 2 + 1] = a / m1;
        return;
    }
    if (qfamily == QF_CATEGORICAL) {
        // per category (E z_c, E z_c^2) = (p_c, p_c); p_c = m1 clamped to [floor, 1]
        if (m1 < BERN_FLOOR || m1 > 1.0) {
            atomicAdd(status + 1, 1u);
            atomicOr(status, 0x2u);
        }
        qp[t * 2] = fmin(fmax(m1, BERN_FLOOR), 1.0);
        qp[t * 2 + 1] = 1.0;
        return;
    }
    if (qfamily == QF_BERNOULLI) {
        // mean parameters (E z, E z^2) = (p, p)
        if (m1 < BERN_FLOOR || m1 > 1.0 - BERN_FLOOR) {
            atomicAdd(status + 1, 1u);
            atomicOr(status, 0x2u);
        }
        qp[t * 2] = fmin(fmax(m1, BERN_FLOOR), 1.0 - BERN_FLOOR);
        qp[t * 2 + 1] = 1.0;
        return;
    }
    const double raw = m2 - m1 * m1;
    if (raw < VAR_FLOOR) {
        atomicAdd(status + 1, 1u);
        atomicOr(status, 0x2u);
    }
    const double v = fmax(raw, VAR_FLOOR);
    if (qfamily == 0) {
        qp[t * 2] = m1;
        qp[t * 2 + 1] = v;
    } else if (m1 > 0.0) {
        qp[t * 2] = m1 * m1 / v;
        qp[t * 2 + 1] = m1 / v;
    } else {
        atomicOr(status, 0x4u);
    }
}

// Dirichlet concentration alpha [C] with psi(alpha_c) - psi(alpha_0) = L_c
// (needs sum_c exp(L_c) < 1): Newton's method in x = log alpha.  The Jacobian
// diag(psi'(alpha_c) alpha_c) - psi'(alpha_0) 1 alpha^T is inverted by
// Sherman-Morrison; steps are capped at 2 in log alpha.  Start: alpha = s m
// with the precision s that psi(x) ~ log x - 1/(2x) implies for the means m.
// Stops after a step below 1e-9 (quadratic convergence) or 100 steps.
// Returns false when no finite root was reached.
__device__ __forceinline__ bool dirichlet_solve(const double* __restrict__ L, const double* __restrict__ mbar, int C,
                                                double* __restrict__ alpha) {
    double msum = 0.0;
    for (int c = 0; c < C; ++c) msum += fmax(mbar[c], 1e-300);
    double num = 0.0, gap = 0.0;
    for (int c = 0; c < C; ++c) {
        const double m = fmax(mbar[c], 1e-300) / msum;
        num += 1.0 - m;
        gap += m * fmax(log(m) - L[c], 1e-300);
        alpha[c] = m;
    }
    const double s0 = fmax(num / (2.0 * gap), 1e-6);
    double x[MAX_DIM];
    for (int c = 0; c < C; ++c) x[c] = log(s0 * alpha[c]);
    for (int it = 0; it < 100; ++it) {
        double a0 = 0.0;
        for (int c = 0; c < C; ++c) { alpha[c] = exp(x[c]); a0 += alpha[c]; }
        const double p0 = digamma_d(a0), z0 = trigamma_d(a0);
        double F[MAX_DIM], q[MAX_DIM];
        double sf = 0.0, sa = 0.0;
        for (int c = 0; c < C; ++c) {
            F[c] = digamma_d(alpha[c]) - p0 - L[c];
            q[c] = trigamma_d(alpha[c]) * alpha[c];
            sf += alpha[c] * F[c] / q[c];
            sa += alpha[c] / q[c];
        }
        const double corr = z0 * sf / (1.0 - z0 * sa);
        double step = 0.0;
        for (int c = 0; c < C; ++c) {
            const double dx = fmin(fmax((F[c] + corr) / q[c], -2.0), 2.0);
            x[c] -= dx;
            step = fmax(step, fabs(dx));
        }
        if (!(step == step)) return false;
        // quadratic convergence: after a step below 1e-9 the error is ~1e-18
        // (a bound like 1e-15 sits at the rounding noise of the step itself)
        if (step < 1e-9) break;
    }
    bool ok = true;
    for (int c = 0; c < C; ++c) {
        alpha[c] = exp(x[c]);
        ok = ok && alpha[c] > 0.0 && alpha[c] < __builtin_inf();
    }
    return ok;
}

// EMA and M-step of one Dirichlet instance: mean parameters (E z_c, E log z_c)
// of its C components at mema[c*2], moments o (scaled by rho) at mone[c*2].
__device__ __forceinline__ void mstep_dirichlet(double* __restrict__ mema, const double* __restrict__ mone,
                                                double* __restrict__ qp, int C, double rho, double lam, bool skip,
                                                uint32_t* __restrict__ status) {
    double m1[MAX_DIM], L[MAX_DIM], alpha[MAX_DIM];
    double se = 0.0;
    for (int c = 0; c < C; ++c) {
        double a1 = mema[c * 2], a2 = mema[c * 2 + 1];
        if (lam != 0.0 && !skip) {
            a1 = (1.0 - lam) * a1 + lam * (rho * mone[c * 2]);
            a2 = (1.0 - lam) * a2 + lam * (rho * mone[c * 2 + 1]);
            mema[c * 2] = a1;
            mema[c * 2 + 1] = a2;
        }
        m1[c] = a1;
        L[c] = a2;
        se += exp(a2);
    }
    if (1.0 - se < DIR_GAP_FLOOR) {
        atomicAdd(status + 1, 1u);
        atomicOr(status, 0x2u);
        const double sh = log(se) - log1p(-DIR_GAP_FLOOR);
        for (int c = 0; c < C; ++c) L[c] -= sh;
    }
    if (!dirichlet_solve(L, m1, C, alpha)) {
        atomicOr(status, 0x4u);
        return;
    }
    for (int c = 0; c < C; ++c) {
        qp[c * 2] = alpha[c];
        qp[c * 2 + 1] = 1.0;
    }
}

__device__ __forceinline__ void mstep_entry(double* __restrict__ mema, const double* __restrict__ mone,
                                            double* __restrict__ qp, long t, int qfamily, double lam, bool skip,
                                            uint32_t* __restrict__ status) {
    mstep_update(mema, qp, t, mema[t * 2], mema[t * 2 + 1], mone[t * 2], mone[t * 2 + 1], qfamily, lam, skip, status);
}

}  // namespace qemk
