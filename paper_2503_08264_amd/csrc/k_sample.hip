// Sampling z ~ Q_t (Algorithm 1): counter-based Philox4x32-10 (Salmon et al.,
// SC'11) with Box-Muller normals and Marsaglia-Tsang (2000) Gamma variates.
//
// Counter (c, sub, iter, node), key (seed lo, seed hi); element e = (i*K+k)*d+j.
// Gaussian proposals draw normals in Box-Muller pairs: elements 2p and 2p+1
// take the cosine and sine branch of the block at counter (p, 0, iter, node).
// Gamma proposals use counter (e, sub): sub = 0 the shape-boost uniform,
// sub = 1+2a, 2+2a the normal (cosine branch) and uniform of Marsaglia-Tsang
// attempt a.
// All sampler arithmetic is FP64 with contraction off, so accept/reject
// decisions follow the definition's rounding sequence exactly.
#include "qem_internal.h"
#include "dev_common.h"
#include "dev_unary.h"

#pragma clang fp contract(off)

namespace qemk {

namespace {

constexpr uint32_t PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
constexpr uint32_t PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;
constexpr int MT_MAX_ATTEMPTS = 32;

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit product gives both halves (a single v_mad_u64_u32)
        const uint64_t p0 = static_cast<uint64_t>(PH_M0) * c0;
        const uint64_t p1 = static_cast<uint64_t>(PH_M1) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = static_cast<uint32_t>(p1); c2 = n2; c3 = static_cast<uint32_t>(p0);
        k0 += PH_W0; k1 += PH_W1;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ uint64_t bits53(uint32_t hi, uint32_t lo) {
    return ((static_cast<uint64_t>(hi) << 32) | lo) >> 11;
}
__device__ __forceinline__ double u_oc(uint32_t hi, uint32_t lo) {   // (0, 1]
    return (static_cast<double>(bits53(hi, lo)) + 1.0) * 0x1.0p-53;
}
__device__ __forceinline__ double u_co(uint32_t hi, uint32_t lo) {   // [0, 1)
    return static_cast<double>(bits53(hi, lo)) * 0x1.0p-53;
}

struct Stream { uint32_t it, node, k0, k1; };

__device__ __forceinline__ double std_normal(uint32_t e, uint32_t sub, const Stream& st) {
    const U4 r = philox10(e, sub, st.it, st.node, st.k0, st.k1);
    const double u1 = u_oc(r.x, r.y), u2 = u_co(r.z, r.w);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}
// Both Box-Muller branches of the block at counter (pair, 0, iter, node).
__device__ __forceinline__ void normal_pair(uint32_t pair, const Stream& st, double& c, double& s) {
    const U4 r = philox10(pair, 0u, st.it, st.node, st.k0, st.k1);
    const double u1 = u_oc(r.x, r.y), u2 = u_co(r.z, r.w);
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(2.0 * M_PI * u2, &sn, &cs);
    c = rad * cs;
    s = rad * sn;
}
// The normal of Gaussian-proposal element e.
__device__ __forceinline__ double paired_normal(uint32_t e, const Stream& st) {
    double c, s;
    normal_pair(e >> 1, st, c, s);
    return (e & 1u) ? s : c;
}

__device__ __forceinline__ double uniform_oc(uint32_t e, uint32_t sub, const Stream& st) {
    const U4 r = philox10(e, sub, st.it, st.node, st.k0, st.k1);
    return u_oc(r.x, r.y);
}

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

// Sampling and the unary log-factor of the same (instance, sample) in one
// pass: identical samples to k_sample_* and identical factors to the
// log-factor kernel (both use unary_value on the stored sample values).
// Optionally writes ut = u (nodes without children) and clears the status
// word (the first node of an iteration).
template <typename T, int D, bool GAMMA>
__global__ void __launch_bounds__(BLOCK) k_sample_unary(UnaryArgs a, Stream st, const uint64_t* __restrict__ it_dev,
                                                        double* __restrict__ ut, uint32_t* __restrict__ status,
                                                        IterTerms itt) {
    const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (it_dev) st.it = static_cast<uint32_t>(*it_dev);
    if (status && t < 4) status[t] = 0u;
    if (itt.lam_out && t == 0)
        *itt.lam_out = itt.p > 0.0 ? pow(static_cast<double>(st.it), -itt.p) : itt.lam;
    st.it ^= itt.it_xor;
    if (t >= static_cast<long>(a.n) * a.K) return;
    const int d = D > 0 ? D : a.d;
    const long i = t / a.K;
    T* z = static_cast<T*>(const_cast<void*>(a.z)) + t * d;
    double zd[D > 0 ? D : MAX_DIM];
    if constexpr (!GAMMA) {
        double eps[D > 0 ? D : MAX_DIM];
        const uint32_t e0 = static_cast<uint32_t>(t * d);
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
#pragma unroll
        for (int j = 0; j < d; ++j) {
            const double mean = a.qp[(i * d + j) * 2 + 0];
            const double var = a.qp[(i * d + j) * 2 + 1];
            const T zv = static_cast<T>(mean + sqrt(var) * eps[j]);
            z[j] = zv;
            zd[j] = static_cast<double>(zv);
        }
    } else {
        double g = gamma_unit(a.qp[i * 2 + 0], static_cast<uint32_t>(t), st) / a.qp[i * 2 + 1];
        if constexpr (sizeof(T) == 4) g = fmax(g, 1.17549435082228750797e-38);
        else g = fmax(g, 2.2250738585072013831e-308);
        const T zv = static_cast<T>(g);
        z[0] = zv;
        zd[0] = static_cast<double>(zv);
    }
    const T u = static_cast<T>(unary_value<D>(a, i, zd));
    static_cast<T*>(a.u)[t] = u;
    if (ut) ut[t] = static_cast<double>(u);
}

Stream make_stream(uint64_t seed, uint32_t iter, uint32_t node) {
    return Stream{iter, node, static_cast<uint32_t>(seed & 0xffffffffu), static_cast<uint32_t>(seed >> 32)};
}

}  // namespace

template <typename T>
void launch_sample_unary(hipStream_t s, dim3 grid, const UnaryArgs& a, const Stream& st, const uint64_t* iter_dev,
                         double* ut, uint32_t* status, const IterTerms& itt) {
    if (a.qfamily != 0) {   // Gamma proposals are scalar
        hipLaunchKernelGGL((k_sample_unary<T, 1, true>), grid, dim3(BLOCK), 0, s, a, st, iter_dev, ut, status, itt);
        return;
    }
    switch (a.d) {
        case 1: hipLaunchKernelGGL((k_sample_unary<T, 1, false>), grid, dim3(BLOCK), 0, s, a, st, iter_dev, ut, status, itt); break;
        case 2: hipLaunchKernelGGL((k_sample_unary<T, 2, false>), grid, dim3(BLOCK), 0, s, a, st, iter_dev, ut, status, itt); break;
        case 4: hipLaunchKernelGGL((k_sample_unary<T, 4, false>), grid, dim3(BLOCK), 0, s, a, st, iter_dev, ut, status, itt); break;
        case 8: hipLaunchKernelGGL((k_sample_unary<T, 8, false>), grid, dim3(BLOCK), 0, s, a, st, iter_dev, ut, status, itt); break;
        default: hipLaunchKernelGGL((k_sample_unary<T, 0, false>), grid, dim3(BLOCK), 0, s, a, st, iter_dev, ut, status, itt); break;
    }
}

hipError_t sample_unary(hipStream_t s, bool f64, const UnaryArgs& a, uint64_t seed, uint32_t iter, uint32_t node,
                        const uint64_t* iter_dev, double* ut, uint32_t* status, const IterTerms& itt) {
    const long total = static_cast<long>(a.n) * a.K;
    const dim3 grid(static_cast<unsigned>((total + BLOCK - 1) / BLOCK));
    const Stream st = make_stream(seed, iter, node);
    if (f64) launch_sample_unary<double>(s, grid, a, st, iter_dev, ut, status, itt);
    else launch_sample_unary<float>(s, grid, a, st, iter_dev, ut, status, itt);
    return hipGetLastError();
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

hipError_t sample_gamma(hipStream_t s, bool f64, void* z, const double* qp, int n, int K,
                        uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev) {
    const long total = static_cast<long>(n) * K;
    const dim3 grid(static_cast<unsigned>((total + BLOCK - 1) / BLOCK));
    const Stream st = make_stream(seed, iter, node);
    if (f64) hipLaunchKernelGGL(k_sample_gamma<double>, grid, dim3(BLOCK), 0, s, (double*)z, qp, total, K, st, iter_dev);
    else hipLaunchKernelGGL(k_sample_gamma<float>, grid, dim3(BLOCK), 0, s, (float*)z, qp, total, K, st, iter_dev);
    return hipGetLastError();
}

}  // namespace qemk
