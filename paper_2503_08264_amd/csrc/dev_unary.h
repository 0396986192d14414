// The unary log-factor of one (instance, sample), shared by the log-factor
// kernel and the fused sample-and-factor kernel so both produce the same bits:
//   u = sum_obs log p(x | z) + root prior - log Q(z) - log K,
// evaluated in FP64 from the sample values as stored (T rounded to double).
#pragma once
#include "qem_internal.h"

namespace qemk {

constexpr double LOG_2PI_D = 1.8378770664093454835606594728112;

// log N(x; mean, var) = qc - (x - mean)^2 qh with the constants of the
// (instance, dimension): qc = -(log(2 pi) + log var) / 2, qh = 1 / (2 var)
__device__ __forceinline__ double normal_qc(double var) {
#pragma clang fp contract(off)
    return -0.5 * (LOG_2PI_D + log(var));
}
__device__ __forceinline__ double normal_qh(double var) { return 0.5 / var; }
__device__ __forceinline__ double log_normal_ch(double x, double mean, double qc, double qh) {
#pragma clang fp contract(off)
    const double d = x - mean;
    return qc - d * d * qh;
}

__device__ __forceinline__ double log_normal_d(double x, double mean, double var) {
    return log_normal_ch(x, mean, normal_qc(var), normal_qh(var));
}

__device__ __forceinline__ double log_gamma_pdf_d(double x, double shape, double rate) {
#pragma clang fp contract(off)
    return shape * log(rate) - lgamma(shape) + (shape - 1.0) * log(x) - rate * x;
}

// z: the d sample values of (instance i, sample k) as doubles.  D > 0 fixes
// d at compile time (the loops unroll and z stays in registers); D = 0 reads
// it from the arguments.  qch (optional, Gaussian Q): the instance's
// (mean, qc, qh) per dimension already at hand, the same values this
// function would load and compute; gobs (optional, Gaussian observations):
// the instance's (xbar, ss) per dimension already loaded.  QF >= 0 fixes the
// proposal family at compile time (QF_GAMMA standing for both Gamma
// families): the terms that node creation rules out for that family are not
// compiled, which keeps the register count of the fused sampler down; the
// arithmetic is unchanged.  QF = -1 reads the family from the arguments.
template <int QF>
__device__ __forceinline__ constexpr bool fam_may(int f) {
    return QF < 0 || QF == f || (f == QF_GAMMA && QF == QF_GAMMA_EF) || (f == QF_GAMMA_EF && QF == QF_GAMMA);
}

template <int D, int QF = -1>
__device__ __forceinline__ double unary_value(const UnaryArgs& a, long i, const double* z,
                                              const double (*qch)[3] = nullptr, const double (*gobs)[2] = nullptr) {
#pragma clang fp contract(off)
    const int d = D > 0 ? D : a.d;
    const int qf = QF >= 0 ? QF : a.qfamily;
    double u = a.neg_log_K;
    if (qf == QF_BERNOULLI) {
        const double pq = a.qp[i * 2];
        u -= (z[0] != 0.0) ? log(pq) : log1p(-pq);
    } else if (qf == QF_CATEGORICAL) {
        // log of the normalised probability of the sample's category
        double tot = 0.0, pc = 0.0;
        for (int j = 0; j < d; ++j) {
            const double pj = a.qp[(i * d + j) * 2];
            tot += pj;
            if (z[j] != 0.0) pc = pj;
        }
        u -= log(pc / tot);
    } else if (qf == QF_DIRICHLET) {
        // log Dir(z; alpha) = lgamma(alpha_0) - sum lgamma(alpha_c) + sum (alpha_c - 1) log z_c
        double a0 = 0.0, lq = 0.0;
        for (int j = 0; j < d; ++j) {
            const double al = a.qp[(i * d + j) * 2];
            a0 += al;
            lq += (al - 1.0) * log(z[j]) - lgamma(al);
        }
        u -= lq + lgamma(a0);
    } else if (qf == QF_GAUSS) {
        if (qch) {
            for (int j = 0; j < d; ++j) u -= log_normal_ch(z[j], qch[j][0], qch[j][1], qch[j][2]);
        } else {
            for (int j = 0; j < d; ++j) u -= log_normal_d(z[j], a.qp[(i * d + j) * 2], a.qp[(i * d + j) * 2 + 1]);
        }
    } else {
        u -= log_gamma_pdf_d(z[0], a.qp[i * 2], a.qp[i * 2 + 1]);
    }
    if (a.prior_term == PT_NORMAL) {
        for (int j = 0; j < d; ++j) {
            const double e = z[j] - a.pb;
            u += a.prior_c0 - e * e * a.prior_hp;
        }
    } else if (fam_may<QF>(QF_GAMMA) && a.prior_term == PT_GAMMA) {
        u += a.prior_c0 + (a.pshape - 1.0) * log(z[0]) - a.prate * z[0];
    } else if (fam_may<QF>(QF_BERNOULLI) && a.prior_term == PT_BERN) {
        u += (z[0] != 0.0) ? a.prior_c0 : a.prior_hp;
    } else if (fam_may<QF>(QF_CATEGORICAL) && a.prior_term == PT_CAT) {
        u += a.prior_c0;   // uniform over the d categories: -log d
    } else if (fam_may<QF>(QF_DIRICHLET) && a.prior_term == PT_DIR) {
        // symmetric Dir(s): prior_c0 = lgamma(C s) - C lgamma(s), prior_hp = s - 1
        double sl = 0.0;
        for (int j = 0; j < d; ++j) sl += log(z[j]);
        u += a.prior_c0 + a.prior_hp * sl;
    } else if (fam_may<QF>(QF_GAUSS) && a.prior_term == PT_CHAIN_START) {
        if (i % a.chain_T == 0) {
            const double e = z[0] - a.pb;
            u += a.prior_c0 - e * e * a.prior_hp;
        }
    }
    if (fam_may<QF>(QF_GAUSS) && a.g_xbar) {
        for (int j = 0; j < d; ++j) {
            const double xb = gobs ? gobs[j][0] : a.g_xbar[i * d + j];
            const double ss = gobs ? gobs[j][1] : a.g_ss[i * d + j];
            const double e = xb - z[j];
            u += a.g_c0 - (ss + a.g_J * e * e) * a.g_hp;
        }
    }
    if (fam_may<QF>(QF_GAMMA) && a.p_sy) u += a.p_sy[i] * log(z[0]) - a.p_J * z[0] - a.p_slg[i];
    if (fam_may<QF>(QF_DIRICHLET) && a.c_cnt)
        for (int j = 0; j < d; ++j) u += a.c_cnt[i * d + j] * log(z[j]);
    if (fam_may<QF>(QF_CATEGORICAL) && a.m_lik)
        for (int j = 0; j < d; ++j)
            if (z[j] != 0.0) u += a.m_lik[i * d + j];
    if (fam_may<QF>(QF_BERNOULLI) && a.d_sy) {
        // detections y_r ~ Bernoulli(p z): z = 1 gives S log p + (R - S) log(1 - p); z = 0 is
        // impossible once anything was detected
        const double sy = a.d_sy[i];
        u += (z[0] != 0.0) ? sy * a.d_l1 + (a.d_R - sy) * a.d_l0 : (sy > 0.0 ? -__builtin_inf() : 0.0);
    }
    return u;
}

}  // namespace qemk
