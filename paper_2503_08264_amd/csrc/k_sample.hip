// Sampling z ~ Q_t (Algorithm 1): counter-based Philox4x32-10 (Salmon et al.,
// SC'11) with Box-Muller normals and Marsaglia-Tsang (2000) Gamma variates.
//
// Counter (c, sub, iter, node), key (seed lo, seed hi); element e = (i*K+k)*d+j.
// Gaussian proposals draw normals in Box-Muller pairs: elements 2p and 2p+1
// take the cosine and sine branch of the block at counter (p, 0, iter, node).
// Gamma proposals use counter (e, sub): sub = 0 the shape-boost uniform,
// sub = 1+2a, 2+2a the normal (cosine branch) and uniform of Marsaglia-Tsang
// attempt a.  Bernoulli proposals: z = 1 when the uniform on (0, 1] of the
// block at counter (e, 0) is at most p.
// All sampler arithmetic is FP64 with contraction off, so accept/reject
// decisions follow the definition's rounding sequence exactly.
#include <algorithm>

#include "qem_internal.h"
#include "dev_common.h"
#include "dev_unary.h"
#include "dev_sample.h"

#pragma clang fp contract(off)

namespace qemk {

namespace {

constexpr int MT_MAX_ATTEMPTS = 32;

__device__ double gamma_unit(double shape, uint32_t e, const Stream& st) {
    const bool boost = shape < 1.0;
    const double a = boost ? shape + 1.0 : shape;
    const double d = a - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    double out = d;
    for (int att = 0; att < MT_MAX_ATTEMPTS; ++att) {
        const double x = std_normal(e, 1u + 2u * att, st);
        const double t = 1.0 + c * x;
        const double v = t * t * t;
        const double u = uniform_oc(e, 2u + 2u * att, st);
        if (v > 0.0) {
            const double lv = log(v);
            if (log(u) < 0.5 * x * x + d - d * v + d * lv) { out = d * v; break; }
        }
    }
    if (boost) out = out * pow(uniform_oc(e, 0u, st), 1.0 / shape);
    return out;
}

// log of the Gamma(shape, 1) draw of gamma_unit (same counters and steps)
// formed in log space, so draws too small for FP64 keep a finite logarithm.
__device__ double gamma_log_unit(double shape, uint32_t e, const Stream& st) {
    const bool boost = shape < 1.0;
    const double a = boost ? shape + 1.0 : shape;
    const double d = a - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    double out = log(d);
    for (int att = 0; att < MT_MAX_ATTEMPTS; ++att) {
        const double x = std_normal(e, 1u + 2u * att, st);
        const double t = 1.0 + c * x;
        const double v = t * t * t;
        const double u = uniform_oc(e, 2u + 2u * att, st);
        if (v > 0.0) {
            const double lv = log(v);
            if (log(u) < 0.5 * x * x + d - d * v + d * lv) { out = log(d) + lv; break; }
        }
    }
    if (boost) out += log(uniform_oc(e, 0u, st)) / shape;
    return out;
}

// One Dirichlet sample of C components at sample index t (elements t*C + c):
// z = softmax(log G), each component at least T's smallest normal value.
template <typename T>
__device__ __forceinline__ void dirichlet_draw(const double* __restrict__ qp, uint32_t i, uint32_t t, int C,
                                               const Stream& st, double* __restrict__ zd) {
    double mx = -__builtin_inf();
    for (int c = 0; c < C; ++c) {
        zd[c] = gamma_log_unit(qp[(static_cast<size_t>(i) * C + c) * 2], t * static_cast<uint32_t>(C) + c, st);
        mx = fmax(mx, zd[c]);
    }
    double s = 0.0;
    for (int c = 0; c < C; ++c) {
        zd[c] = exp(zd[c] - mx);
        s += zd[c];
    }
    for (int c = 0; c < C; ++c) {
        double v = zd[c] / s;
        if constexpr (sizeof(T) == 4) v = fmax(v, 1.17549435082228750797e-38);
        else v = fmax(v, 2.2250738585072013831e-308);
        zd[c] = v;
    }
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_sample_dirichlet(T* __restrict__ z, const double* __restrict__ qp,
                                                            long total, int K, int C, Stream st,
                                                            const uint64_t* __restrict__ it_dev) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= total) return;
    if (it_dev) st.it = static_cast<uint32_t>(*it_dev);
    double zd[MAX_DIM];
    dirichlet_draw<T>(qp, static_cast<uint32_t>(t / K), static_cast<uint32_t>(t), C, st, zd);
    for (int c = 0; c < C; ++c) z[t * C + c] = static_cast<T>(zd[c]);
}

// The category of sample e under (unnormalised) probabilities p [C].
__device__ __forceinline__ int categorical_draw(const double* __restrict__ p, int C, uint32_t e, const Stream& st) {
    double tot = 0.0;
    for (int c = 0; c < C; ++c) tot += p[c * 2];
    const double target = uniform_oc(e, 0u, st) * tot;
    double run = 0.0;
    for (int c = 0; c < C; ++c) {
        run += p[c * 2];
        if (target <= run) return c;
    }
    return C - 1;
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_sample_categorical(T* __restrict__ z, const double* __restrict__ qp,
                                                              long total, int K, int C, Stream st,
                                                              const uint64_t* __restrict__ it_dev) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= total) return;
    if (it_dev) st.it = static_cast<uint32_t>(*it_dev);
    const int cat = categorical_draw(qp + (t / K) * C * 2, C, static_cast<uint32_t>(t), st);
    for (int c = 0; c < C; ++c) z[t * C + c] = static_cast<T>(c == cat ? 1.0 : 0.0);
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_sample_gauss(T* __restrict__ z, const double* __restrict__ qp,
                                                        long total, int K, int d, Stream st,
                                                        const uint64_t* __restrict__ it_dev) {
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= total) return;
    if (it_dev) st.it = static_cast<uint32_t>(*it_dev);
    const long j = e % d;
    const long i = e / (static_cast<long>(K) * d);
    const double mean = qp[(i * d + j) * 2 + 0];
    const double var = qp[(i * d + j) * 2 + 1];
    const double eps = paired_normal(static_cast<uint32_t>(e), st);
    z[e] = static_cast<T>(mean + sqrt(var) * eps);
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_sample_gamma(T* __restrict__ z, const double* __restrict__ qp,
                                                        long total, int K, Stream st,
                                                        const uint64_t* __restrict__ it_dev) {
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= total) return;
    if (it_dev) st.it = static_cast<uint32_t>(*it_dev);
    const long i = e / K;
    const double shape = qp[i * 2 + 0];
    const double rate = qp[i * 2 + 1];
    double g = gamma_unit(shape, static_cast<uint32_t>(e), st) / rate;
    // A proposal with shape well below 1 can draw values below the smallest
    // normal number of T; they are raised to it so that log z stays finite.
    if constexpr (sizeof(T) == 4) g = fmax(g, 1.17549435082228750797e-38);
    else g = fmax(g, 2.2250738585072013831e-308);
    z[e] = static_cast<T>(g);
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_sample_bernoulli(T* __restrict__ z, const double* __restrict__ qp,
                                                            long total, int K, Stream st,
                                                            const uint64_t* __restrict__ it_dev) {
    const long e = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= total) return;
    if (it_dev) st.it = static_cast<uint32_t>(*it_dev);
    z[e] = static_cast<T>(uniform_oc(static_cast<uint32_t>(e), 0u, st) <= qp[(e / K) * 2] ? 1.0 : 0.0);
}

// Sampling and the unary log-factor of the same (instance, sample) in one
// pass: identical samples to k_sample_* and identical factors to the
// log-factor kernel (both use unary_value on the stored sample values).
// One launch covers up to SAMPLE_NODES nodes of the same dimension and
// family (node q takes blocks [boff[q], boff[q+1])).  Optionally writes
// ut = u (nodes without children); block 0 clears the status word and writes
// the iteration's EMA weight.
struct SampleTable {
    UnaryArgs a[SAMPLE_NODES];
    double* ut[SAMPLE_NODES];
    uint32_t node[SAMPLE_NODES];
    uint32_t boff[SAMPLE_NODES + 1];
    int n;
};

// Sampler families of the fused kernel
constexpr int FAM_GAUSS = 0, FAM_GAMMA = 1, FAM_BERN = 2, FAM_DIR = 3, FAM_CAT = 4;

// the proposal family each sampler family serves (QF_GAMMA: both Gamma families)
template <int FAM>
constexpr int fam_qf() {
    return FAM == FAM_GAUSS ? QF_GAUSS : FAM == FAM_GAMMA ? QF_GAMMA : FAM == FAM_BERN ? QF_BERNOULLI
         : FAM == FAM_DIR ? QF_DIRICHLET : QF_CATEGORICAL;
}

template <typename T, int D, int FAM>
__device__ __forceinline__ void sample_one(const UnaryArgs& a, const Stream& st, double* __restrict__ ut, uint32_t t) {
    const int d = D > 0 ? D : a.d;
    const uint32_t i = t / static_cast<uint32_t>(a.K);
    T* z = static_cast<T*>(const_cast<void*>(a.z)) + static_cast<size_t>(t) * d;
    double zd[D > 0 ? D : MAX_DIM];
    double u;
    if constexpr (FAM == FAM_GAUSS) {
        if constexpr (D > 0) {
            if (a.K % WAVE == 0) {   // the wave holds whole instances
                T zw[D > 0 ? D : 1];
                const T uT = gauss_sample_in_wave<T, D>(a, st, t, zw);
#pragma unroll
                for (int j = 0; j < D; ++j) z[j] = zw[j];
                static_cast<T*>(a.u)[t] = uT;
                if (ut) ut[t] = static_cast<double>(uT);
                return;
            }
        }
        double eps[D > 0 ? D : MAX_DIM];
        const uint32_t e0 = t * static_cast<uint32_t>(d);
        if constexpr (D > 0 && D % 2 == 0) {
            // e0 is even: the thread's elements form whole pairs
#pragma unroll
            for (int j = 0; j < D; j += 2) normal_pair((e0 + j) >> 1, st, eps[j], eps[j + 1]);
        } else {
            uint32_t cur = 0xffffffffu;
            double c = 0.0, s = 0.0;
#pragma unroll
            for (int j = 0; j < d; ++j) {
                const uint32_t e = e0 + j;
                if ((e >> 1) != cur) {
                    cur = e >> 1;
                    normal_pair(cur, st, c, s);
                }
                eps[j] = (e & 1u) ? s : c;
            }
        }
        // Per dimension: the mean, then sd = sqrt(var) and the log-density
        // constants (qc, qh), which depend on the instance only.  When a wave
        // holds whole instances (K a divisor of the wave with d <= K; K a
        // multiple of it takes gauss_sample_in_wave), lane j of an instance's
        // lane group computes them for dimension j and the other lanes read
        // them from it; otherwise each thread computes its own.  Either way
        // the values are the same bits.
        double q[D > 0 ? D : MAX_DIM][3], sd[D > 0 ? D : MAX_DIM];
#pragma unroll
        for (int j = 0; j < d; ++j) q[j][0] = a.qp[(static_cast<size_t>(i) * d + j) * 2];
        bool done = false;
        if constexpr (D > 0) {
            const int lane = threadIdx.x & (WAVE - 1);
            if (WAVE % a.K == 0 && D <= a.K) {
                const int base = (lane / a.K) * a.K;
                double s0 = 0.0, c0 = 0.0, h0 = 0.0;
                if (lane - base < D) q_consts(a.qp, i, D, lane - base, s0, c0, h0);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    sd[j] = __shfl(s0, base + j, WAVE);
                    q[j][1] = __shfl(c0, base + j, WAVE);
                    q[j][2] = __shfl(h0, base + j, WAVE);
                }
                done = true;
            }
        }
        if (!done)
            for (int j = 0; j < d; ++j) q_consts(a.qp, i, d, j, sd[j], q[j][1], q[j][2]);
#pragma unroll
        for (int j = 0; j < d; ++j) {
            const T zv = static_cast<T>(q[j][0] + sd[j] * eps[j]);
            z[j] = zv;
            zd[j] = static_cast<double>(zv);
        }
        u = unary_value<D, fam_qf<FAM>()>(a, i, zd, q);
    } else if constexpr (FAM == FAM_CAT) {
        const int cat = categorical_draw(a.qp + static_cast<size_t>(i) * d * 2, d, t, st);
        for (int c = 0; c < d; ++c) {
            const T zv = static_cast<T>(c == cat ? 1.0 : 0.0);
            z[c] = zv;
            zd[c] = static_cast<double>(zv);
        }
        u = unary_value<D, fam_qf<FAM>()>(a, i, zd);
    } else if constexpr (FAM == FAM_DIR) {
        dirichlet_draw<T>(a.qp, i, t, d, st, zd);
        for (int c = 0; c < d; ++c) {
            const T zv = static_cast<T>(zd[c]);
            z[c] = zv;
            zd[c] = static_cast<double>(zv);
        }
        u = unary_value<D, fam_qf<FAM>()>(a, i, zd);
    } else if constexpr (FAM == FAM_BERN) {
        const T zv = static_cast<T>(uniform_oc(t, 0u, st) <= a.qp[i * 2] ? 1.0 : 0.0);
        z[0] = zv;
        zd[0] = static_cast<double>(zv);
        u = unary_value<D, fam_qf<FAM>()>(a, i, zd);
    } else {
        double g = gamma_unit(a.qp[i * 2 + 0], t, st) / a.qp[i * 2 + 1];
        if constexpr (sizeof(T) == 4) g = fmax(g, 1.17549435082228750797e-38);
        else g = fmax(g, 2.2250738585072013831e-308);
        const T zv = static_cast<T>(g);
        z[0] = zv;
        zd[0] = static_cast<double>(zv);
        u = unary_value<D, fam_qf<FAM>()>(a, i, zd);
    }
    const T uT = static_cast<T>(u);
    static_cast<T*>(a.u)[t] = uT;
    if (ut) ut[t] = static_cast<double>(uT);
}

template <typename T, int D, int FAM>
__global__ void __launch_bounds__(BLOCK) k_sample_unary(SampleTable tb, Stream st, const uint64_t* __restrict__ it_dev,
                                                        uint32_t* __restrict__ status, IterTerms itt) {
    if (it_dev) st.it = static_cast<uint32_t>(*it_dev);
    if (blockIdx.x == 0) {
        if (status && threadIdx.x < 4) status[threadIdx.x] = 0u;
        if (itt.lam_out && threadIdx.x == 0)
            *itt.lam_out = itt.p > 0.0 ? pow(static_cast<double>(st.it), -itt.p) : itt.lam;
    }
    st.it ^= itt.it_xor;
    // the node of this block (uniform branches; the table stays in kernel arguments)
#pragma unroll
    for (int q = 0; q < SAMPLE_NODES; ++q) {
        if (q < tb.n && blockIdx.x >= tb.boff[q] && blockIdx.x < tb.boff[q + 1]) {
            // n*K*d < 2^32 (checked at create), so 32-bit indices suffice
            const uint32_t t = (blockIdx.x - tb.boff[q]) * BLOCK + threadIdx.x;
            if (t >= static_cast<uint32_t>(tb.a[q].n) * static_cast<uint32_t>(tb.a[q].K)) return;
            st.node = tb.node[q];
            sample_one<T, D, FAM>(tb.a[q], st, tb.ut[q], t);
            return;
        }
    }
}

}  // namespace

Stream make_stream(uint64_t seed, uint32_t iter, uint32_t node) {
    return Stream{iter, node, static_cast<uint32_t>(seed & 0xffffffffu), static_cast<uint32_t>(seed >> 32)};
}

template <typename T>
void launch_sample_unary(hipStream_t s, dim3 grid, const SampleTable& tb, int qfamily, int d, const Stream& st,
                         const uint64_t* iter_dev, uint32_t* status, const IterTerms& itt) {
    if (qfamily == QF_CATEGORICAL) {   // one-hot over C categories
        hipLaunchKernelGGL((k_sample_unary<T, 0, FAM_CAT>), grid, dim3(BLOCK), 0, s, tb, st, iter_dev, status, itt);
        return;
    }
    if (qfamily == QF_DIRICHLET) {   // C components, C from the node
        hipLaunchKernelGGL((k_sample_unary<T, 0, FAM_DIR>), grid, dim3(BLOCK), 0, s, tb, st, iter_dev, status, itt);
        return;
    }
    if (qfamily == QF_BERNOULLI) {   // scalar discrete latents
        hipLaunchKernelGGL((k_sample_unary<T, 1, FAM_BERN>), grid, dim3(BLOCK), 0, s, tb, st, iter_dev, status, itt);
        return;
    }
    if (qfamily != QF_GAUSS) {   // Gamma proposals are scalar
        hipLaunchKernelGGL((k_sample_unary<T, 1, FAM_GAMMA>), grid, dim3(BLOCK), 0, s, tb, st, iter_dev, status, itt);
        return;
    }
    switch (d) {
        case 1: hipLaunchKernelGGL((k_sample_unary<T, 1, FAM_GAUSS>), grid, dim3(BLOCK), 0, s, tb, st, iter_dev, status, itt); break;
        case 2: hipLaunchKernelGGL((k_sample_unary<T, 2, FAM_GAUSS>), grid, dim3(BLOCK), 0, s, tb, st, iter_dev, status, itt); break;
        case 4: hipLaunchKernelGGL((k_sample_unary<T, 4, FAM_GAUSS>), grid, dim3(BLOCK), 0, s, tb, st, iter_dev, status, itt); break;
        case 8: hipLaunchKernelGGL((k_sample_unary<T, 8, FAM_GAUSS>), grid, dim3(BLOCK), 0, s, tb, st, iter_dev, status, itt); break;
        default: hipLaunchKernelGGL((k_sample_unary<T, 0, FAM_GAUSS>), grid, dim3(BLOCK), 0, s, tb, st, iter_dev, status, itt); break;
    }
}

bool sample_group_compatible(const UnaryArgs& x, const UnaryArgs& y) {
    if (x.qfamily != y.qfamily) return false;
    if (x.qfamily != QF_GAUSS) return true;
    const auto fixed = [](int d) { return d == 1 || d == 2 || d == 4 || d == 8; };
    return x.d == y.d || (!fixed(x.d) && !fixed(y.d));
}

hipError_t sample_unary_multi(hipStream_t s, bool f64, const SampleNode* nodes, int n, uint64_t seed, uint32_t iter,
                              const uint64_t* iter_dev, uint32_t* status, const IterTerms& itt) {
    if (n < 1 || n > SAMPLE_NODES) return hipErrorInvalidValue;
    SampleTable tb{};
    tb.n = n;
    uint64_t blocks = 0;
    for (int q = 0; q < n; ++q) {
        if (!sample_group_compatible(nodes[0].a, nodes[q].a)) return hipErrorInvalidValue;
        tb.a[q] = nodes[q].a;
        tb.ut[q] = nodes[q].ut;
        tb.node[q] = nodes[q].node;
        tb.boff[q] = static_cast<uint32_t>(blocks);
        const uint64_t total = static_cast<uint64_t>(nodes[q].a.n) * nodes[q].a.K;
        blocks += std::max<uint64_t>(1, (total + BLOCK - 1) / BLOCK);
    }
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    for (int q = n; q <= SAMPLE_NODES; ++q) tb.boff[q] = static_cast<uint32_t>(blocks);
    const Stream st = make_stream(seed, iter, 0u);
    const dim3 grid(static_cast<unsigned>(blocks));
    if (f64) launch_sample_unary<double>(s, grid, tb, nodes[0].a.qfamily, nodes[0].a.d, st, iter_dev, status, itt);
    else launch_sample_unary<float>(s, grid, tb, nodes[0].a.qfamily, nodes[0].a.d, st, iter_dev, status, itt);
    return hipGetLastError();
}

hipError_t sample_unary(hipStream_t s, bool f64, const UnaryArgs& a, uint64_t seed, uint32_t iter, uint32_t node,
                        const uint64_t* iter_dev, double* ut, uint32_t* status, const IterTerms& itt) {
    const SampleNode one{a, ut, node};
    return sample_unary_multi(s, f64, &one, 1, seed, iter, iter_dev, status, itt);
}

hipError_t sample_gauss(hipStream_t s, bool f64, void* z, const double* qp, int n, int K, int d,
                        uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev) {
    const long total = static_cast<long>(n) * K * d;
    const dim3 grid(static_cast<unsigned>((total + BLOCK - 1) / BLOCK));
    const Stream st = make_stream(seed, iter, node);
    if (f64) hipLaunchKernelGGL(k_sample_gauss<double>, grid, dim3(BLOCK), 0, s, (double*)z, qp, total, K, d, st, iter_dev);
    else hipLaunchKernelGGL(k_sample_gauss<float>, grid, dim3(BLOCK), 0, s, (float*)z, qp, total, K, d, st, iter_dev);
    return hipGetLastError();
}

hipError_t sample_bernoulli(hipStream_t s, bool f64, void* z, const double* qp, int n, int K,
                            uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev) {
    const long total = static_cast<long>(n) * K;
    const dim3 grid(static_cast<unsigned>((total + BLOCK - 1) / BLOCK));
    const Stream st = make_stream(seed, iter, node);
    if (f64) hipLaunchKernelGGL(k_sample_bernoulli<double>, grid, dim3(BLOCK), 0, s, (double*)z, qp, total, K, st, iter_dev);
    else hipLaunchKernelGGL(k_sample_bernoulli<float>, grid, dim3(BLOCK), 0, s, (float*)z, qp, total, K, st, iter_dev);
    return hipGetLastError();
}

hipError_t sample_gamma(hipStream_t s, bool f64, void* z, const double* qp, int n, int K,
                        uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev) {
    const long total = static_cast<long>(n) * K;
    const dim3 grid(static_cast<unsigned>((total + BLOCK - 1) / BLOCK));
    const Stream st = make_stream(seed, iter, node);
    if (f64) hipLaunchKernelGGL(k_sample_gamma<double>, grid, dim3(BLOCK), 0, s, (double*)z, qp, total, K, st, iter_dev);
    else hipLaunchKernelGGL(k_sample_gamma<float>, grid, dim3(BLOCK), 0, s, (float*)z, qp, total, K, st, iter_dev);
    return hipGetLastError();
}

hipError_t sample_categorical(hipStream_t s, bool f64, void* z, const double* qp, int n, int K, int C,
                              uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev) {
    if (C < 2 || C > MAX_DIM) return hipErrorInvalidValue;
    const long total = static_cast<long>(n) * K;
    const dim3 grid(static_cast<unsigned>((total + BLOCK - 1) / BLOCK));
    const Stream st = make_stream(seed, iter, node);
    if (f64)
        hipLaunchKernelGGL(k_sample_categorical<double>, grid, dim3(BLOCK), 0, s, (double*)z, qp, total, K, C, st,
                           iter_dev);
    else
        hipLaunchKernelGGL(k_sample_categorical<float>, grid, dim3(BLOCK), 0, s, (float*)z, qp, total, K, C, st,
                           iter_dev);
    return hipGetLastError();
}

hipError_t sample_dirichlet(hipStream_t s, bool f64, void* z, const double* qp, int n, int K, int C,
                            uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev) {
    if (C < 2 || C > MAX_DIM) return hipErrorInvalidValue;
    const long total = static_cast<long>(n) * K;
    const dim3 grid(static_cast<unsigned>((total + BLOCK - 1) / BLOCK));
    const Stream st = make_stream(seed, iter, node);
    if (f64)
        hipLaunchKernelGGL(k_sample_dirichlet<double>, grid, dim3(BLOCK), 0, s, (double*)z, qp, total, K, C, st,
                           iter_dev);
    else
        hipLaunchKernelGGL(k_sample_dirichlet<float>, grid, dim3(BLOCK), 0, s, (float*)z, qp, total, K, C, st,
                           iter_dev);
    return hipGetLastError();
}

}  // namespace qemk
