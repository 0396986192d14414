// Counter-based draws shared by the sampling kernels and by the plate forward
// kernel that draws its own node's samples: Philox4x32-10 (Salmon et al.,
// SC'11) on the counter (c, sub, iter, node) with the key (seed lo, seed hi),
// Box-Muller normals (elements 2p and 2p + 1 take the cosine and sine branch
// of the block at counter (p, 0, iter, node)), and the Gaussian sample of one
// (instance, sample) element with its unary factor when a wave holds whole
// instances.  All FP64 with contraction off, so every kernel that draws an
// element forms the same bits.
#pragma once
#include "qem_internal.h"
#include "dev_common.h"
#include "dev_unary.h"

namespace qemk {

namespace {

constexpr uint32_t PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
constexpr uint32_t PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;

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
#pragma clang fp contract(off)
    return (static_cast<double>(bits53(hi, lo)) + 1.0) * 0x1.0p-53;
}
__device__ __forceinline__ double u_co(uint32_t hi, uint32_t lo) {   // [0, 1)
#pragma clang fp contract(off)
    return static_cast<double>(bits53(hi, lo)) * 0x1.0p-53;
}

__device__ __forceinline__ double std_normal(uint32_t e, uint32_t sub, const Stream& st) {
#pragma clang fp contract(off)
    const U4 r = philox10(e, sub, st.it, st.node, st.k0, st.k1);
    const double u1 = u_oc(r.x, r.y), u2 = u_co(r.z, r.w);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}
// Both Box-Muller branches of the block at counter (pair, 0, iter, node).
__device__ __forceinline__ void normal_pair(uint32_t pair, const Stream& st, double& c, double& s) {
#pragma clang fp contract(off)
    const U4 r = philox10(pair, 0u, st.it, st.node, st.k0, st.k1);
    const double u1 = u_oc(r.x, r.y), u2 = u_co(r.z, r.w);
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    // the angle 2 pi u2 as sincospi(2 u2): the argument is exact and in [0, 2),
    // so no general range reduction is needed
    sincospi(2.0 * u2, &sn, &cs);
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

__device__ __forceinline__ double readlane_d(double x, int l) {
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(b), l);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(b >> 32), l);
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

// The Q constants of dimension j of instance i: sd = sqrt(var), and qc, qh of
// the Gaussian log-density.
__device__ __forceinline__ void q_consts(const double* __restrict__ qp, uint32_t i, int d, int j, double& sd,
                                         double& qc, double& qh) {
#pragma clang fp contract(off)
    const double v = qp[(static_cast<size_t>(i) * d + j) * 2 + 1];
    sd = sqrt(v);
    qc = normal_qc(v);
    qh = normal_qh(v);
}

// The global values the Gaussian sample of an instance's element needs: per
// dimension the proposal mean, the variance of dimension `lane` (lanes
// 0..D-1; the others hold 1), and the Gaussian observations' (xbar, ss).
// Loaded apart from gauss_sample_from so that a kernel can issue the loads
// before other work.
template <int D>
struct GaussInst {
    double mean[D], var_l, xb[D], ss[D];
    bool gobs;
};

template <int D>
__device__ __forceinline__ GaussInst<D> gauss_inst_load(const UnaryArgs& a, uint32_t i) {
    GaussInst<D> g;
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int j = 0; j < D; ++j) g.mean[j] = a.qp[(static_cast<size_t>(i) * D + j) * 2];
    g.var_l = lane < D ? a.qp[(static_cast<size_t>(i) * D + lane) * 2 + 1] : 1.0;
    g.gobs = a.g_xbar != nullptr;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        g.xb[j] = g.gobs ? a.g_xbar[static_cast<size_t>(i) * D + j] : 0.0;
        g.ss[j] = g.gobs ? a.g_ss[static_cast<size_t>(i) * D + j] : 0.0;
    }
    return g;
}

// The Gaussian sample of element t = i K + k of a node with D-dimensional
// proposals and K a multiple of the wave (the wave holds instance i whole):
// the normals of its D elements (Box-Muller pairs), per dimension the mean,
// then sd = sqrt(var) and the log-density constants (qc, qh), formed by lane
// j for dimension j and read by every lane, z = mean + sd eps rounded to T.
// Writes z[] and returns the unary factor (rounded to T).
template <typename T, int D>
__device__ __forceinline__ T gauss_sample_from(const UnaryArgs& a, const Stream& st, uint32_t t,
                                               const GaussInst<D>& g, T (&z)[D]) {
#pragma clang fp contract(off)
    const uint32_t i = t / static_cast<uint32_t>(a.K);
    double eps[D];
    const uint32_t e0 = t * static_cast<uint32_t>(D);
    if constexpr (D % 2 == 0) {
        // e0 is even: the element's dimensions form whole pairs
#pragma unroll
        for (int j = 0; j < D; j += 2) normal_pair((e0 + j) >> 1, st, eps[j], eps[j + 1]);
    } else {
        uint32_t cur = 0xffffffffu;
        double c = 0.0, s = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const uint32_t e = e0 + j;
            if ((e >> 1) != cur) {
                cur = e >> 1;
                normal_pair(cur, st, c, s);
            }
            eps[j] = (e & 1u) ? s : c;
        }
    }
    double q[D][3], sd[D], zd[D], go[D][2];
    const int lane = threadIdx.x & (WAVE - 1);
    double s0 = 0.0, c0 = 0.0, h0 = 0.0;
    if (lane < D) {
        s0 = sqrt(g.var_l);
        c0 = normal_qc(g.var_l);
        h0 = normal_qh(g.var_l);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        q[j][0] = g.mean[j];
        sd[j] = readlane_d(s0, j);
        q[j][1] = readlane_d(c0, j);
        q[j][2] = readlane_d(h0, j);
        go[j][0] = g.xb[j];
        go[j][1] = g.ss[j];
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const T zv = static_cast<T>(q[j][0] + sd[j] * eps[j]);
        z[j] = zv;
        zd[j] = static_cast<double>(zv);
    }
    return static_cast<T>(unary_value<D, QF_GAUSS>(a, i, zd, q, g.gobs ? go : nullptr));
}

template <typename T, int D>
__device__ __forceinline__ T gauss_sample_in_wave(const UnaryArgs& a, const Stream& st, uint32_t t, T (&z)[D]) {
    return gauss_sample_from<T, D>(a, st, t, gauss_inst_load<D>(a, t / static_cast<uint32_t>(a.K)), z);
}

}  // namespace

}  // namespace qemk
