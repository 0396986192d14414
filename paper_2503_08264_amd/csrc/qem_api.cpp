// Host side of the C ABI declared in include/qem.h: validation of the model
// description, workspace planning, and the order in which the E-step kernels
// are enqueued.
//
// Elimination order.  Nodes are listed parents first, so the forward pass
// walks node ids downwards (children before parents) and the reverse pass
// upwards.  Node kinds:
//   ROOT       no factor parent: every instance is its own component,
//              L_i = LSE_k ut[i,k]
//   CHAIN      series of steps, eliminated from the last step to the first
//   SINGLE     one factor parent: plate log-sum-exp into the parent's ut
//   PAIRCHILD  two single-instance root parents (a, b): K_a x K_b messages
//   PAIRROOT   a or b above: summed jointly with the pair's messages
// log P_MP is the FP64 sum, in a fixed order, of every component's L.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qem.h"
#include "qem_internal.h"

namespace {

thread_local std::string g_create_err;

// K_CHAINP: a chain whose series each hang under one instance of a sampled
// scalar parent (eliminated once per parent sample).
enum Kind { K_ROOT, K_CHAIN, K_CHAINP, K_SINGLE, K_PAIRCHILD, K_PAIRROOT };

struct Csr {                       // child instances of each parent instance
    int child = -1;
    std::vector<int32_t> off, idx;
    size_t o_off = 0, o_idx = 0;
    int32_t per = 0;               // > 0: every parent has `per` children, in index order
};

// The children per parent instance when the list holds the same number of
// children for every parent, in index order (idx[j] = j, off[q] = q r); else 0.
int32_t regular_per(const Csr& cs) {
    const size_t np = cs.off.size() - 1;
    if (np == 0 || cs.idx.empty() || cs.idx.size() % np != 0) return 0;
    const size_t r = cs.idx.size() / np;
    for (size_t q = 0; q <= np; ++q)
        if (static_cast<size_t>(cs.off[q]) != q * r) return 0;
    for (size_t j = 0; j < cs.idx.size(); ++j)
        if (static_cast<size_t>(cs.idx[j]) != j) return 0;
    return static_cast<int32_t>(r);
}

struct NodeP {
    qem_node_desc d{};
    std::vector<int32_t> pidx;
    std::vector<int32_t> sp;       // K_CHAINP: parent instance of each series
    int fp[2] = {-1, -1};
    int nfp = 0;
    Kind kind = K_ROOT;
    int gobs = -1, pobs = -1, bobs = -1, dobs = -1, cobs = -1, mobs = -1;
    std::vector<Csr> children;
    size_t o_qp = 0, o_mema = 0, o_mone = 0, o_z = 0, o_u = 0, o_F = 0, o_ut = 0, o_msg = 0, o_w = 0;
    size_t o_pidx = 0, o_gxbar = 0, o_gss = 0, o_psy = 0, o_pslg = 0, o_dsy = 0, o_dslg = 0, o_ccnt = 0, o_mlik = 0;
    size_t o_ga0 = 0, o_ga1 = 0, o_gk = 0, o_hb = 0, o_hk = 0, o_C = 0;
    // K_CHAINP: series -> parent instance, and per virtual series (g, kb):
    // u-tilde and weights [G * K, T, K], the message to the parent [G, K]
    size_t o_sp = 0, o_vut = 0, o_vw = 0, o_vL = 0;
    size_t o_tpflag = 0;           // K_PAIRCHILD on MFMA: instances left to the exact kernels
    bool has_F = false, has_pidx = false;
    long Lslot = -1;
    long nL = 0;
};

}  // namespace

struct qem_ctx_s {
    std::vector<NodeP> nodes;
    std::vector<qem_obs_desc> obs;
    int K = 0, prec = 0;
    hipStream_t s = nullptr;
    size_t bytes = 0;
    char* ws = nullptr;
    size_t o_logphat = 0, o_status = 0, o_iter = 0, o_Lall = 0, o_pairM = 0, o_pairW = 0, o_pairScr = 0;
    size_t o_lamt = 0, o_lp1 = 0;   // this iteration's EMA weight; log P_MP of the first sample
    size_t o_rootpart = 0;          // subset sums of a wide root's child gather
    // captured iterations of Algorithm 1 (qem_run): one, and RUN_UNROLL in a row
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr, graph_u = nullptr;
    hipGraphExec_t gexec = nullptr, gexec_u = nullptr;
    uint64_t g_seed = 0;
    double g_lam = -1.0;
    // EMA options of qem_step / qem_run (qem_set_ema)
    double ema_p = 0.0;
    bool second_sample = false;
    // QEM_CREATE_NO_TABLES: linear-Gaussian plate and chain factors recomputed, not kept
    bool no_tables = false;
    // QEM_CREATE_CHAIN_TABLES: FP32/FP64 chains keep their step-factor table
    bool chain_tables = false;
    long nL = 0, pair_slot = -1;
    int pa = -1, pb = -1;
    std::string err;
    std::vector<std::pair<size_t, const std::vector<int32_t>*>> uploads;
    // tracing: event pairs per (node + 1, phase), resolved on read
    bool timing = false;
    struct Rec { int slot; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    std::vector<double> tms;
    std::vector<int64_t> tcount;

    bool f64() const { return prec == QEM_FP64; }
    bool bexp() const { return prec == QEM_BF16EXP; }
    size_t eb() const { return f64() ? 8 : 4; }
    template <typename P = void> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
    double* d(size_t off) const { return at<double>(off); }
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

bool is_gamma_q(int32_t qfamily) { return qfamily == QEM_Q_GAMMA || qfamily == QEM_Q_GAMMA_EF; }

// Families whose mean parameters are (E z, E log z).
bool uses_log_moments(int32_t qfamily) { return qfamily == QEM_Q_GAMMA_EF || qfamily == QEM_Q_DIRICHLET; }

qem_status fail(qem_ctx c, qem_status st, const std::string& msg) {
    if (c) c->err = msg; else g_create_err = msg;
    return st;
}

// A node whose pairwise factor the forward (and, without a kept table, the
// reverse) kernels evaluate from the samples: linear-Gaussian plates of the
// supported shapes, and chains outside BF16-exp mode.
bool factor_in_kernel(const qem_ctx c, const NodeP& p) {
    if (p.kind == K_CHAINP) return true;
    if (p.kind == K_CHAIN) return true;
    return p.kind == K_SINGLE && p.bobs < 0 && p.d.prior == QEM_PRIOR_NORMAL &&
           qemk::plate_fwd_pn_supported(c->f64(), c->K, c->K, p.d.dim);
}

#define QEM_HIP(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(c, QEM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// A launch bracketed by tracing events (see qem_timing).
#define QEM_LAUNCH(node, phase, expr)          \
    do {                                       \
        Timed t_(c, (node), (phase));          \
        QEM_HIP(expr);                         \
    } while (0)

qem_status validate_and_plan(qem_ctx c, const qem_model_desc* m) {
    const int N = m->n_nodes;
    const int K = c->K;
    if (N < 1 || !m->nodes) return fail(c, QEM_E_INVALID, "model needs at least one node");
    if (m->n_obs < 0 || (m->n_obs > 0 && !m->obs)) return fail(c, QEM_E_INVALID, "bad observation list");
    c->nodes.resize(N);
    for (int v = 0; v < N; ++v) {
        NodeP& p = c->nodes[v];
        p.d = m->nodes[v];
        const qem_node_desc& d = p.d;
        if (d.n < 1 || d.dim < 1) return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": n and dim must be >= 1");
        if (d.dim > qemk::MAX_DIM)
            return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": dim must be <= " + std::to_string(qemk::MAX_DIM));
        if (d.qfamily < QEM_Q_GAUSS || d.qfamily > QEM_Q_CATEGORICAL)
            return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": bad qfamily");
        if (is_gamma_q(d.qfamily) && d.dim != 1)
            return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": Gamma proposals are scalar");
        if (d.prior < QEM_PRIOR_NORMAL || d.prior > QEM_PRIOR_CATEGORICAL)
            return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": bad prior kind");
        if ((d.qfamily == QEM_Q_BERNOULLI) != (d.prior == QEM_PRIOR_BERNOULLI_LOGIT))
            return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": Bernoulli latents take the Bernoulli-logit prior, and only they do");
        if (d.qfamily == QEM_Q_BERNOULLI && (d.dim != 1 || !(d.q0a > 0.0 && d.q0a < 1.0)))
            return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": Bernoulli latents are scalar with 0 < q0a < 1");
        if ((d.qfamily == QEM_Q_DIRICHLET) != (d.prior == QEM_PRIOR_DIRICHLET))
            return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": Dirichlet latents take the Dirichlet prior, and only they do");
        if ((d.qfamily == QEM_Q_CATEGORICAL) != (d.prior == QEM_PRIOR_CATEGORICAL))
            return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": categorical latents take the categorical prior, and only they do");
        if (d.qfamily == QEM_Q_CATEGORICAL) {
            if (d.dim < 2) return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": a categorical latent has dim = C >= 2 categories");
            if (!(d.q0a > 0.0)) return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": categorical initial weight q0a must be > 0");
            if (d.parent0 >= 0) {
                const qem_node_desc& pd = m->nodes[d.parent0];
                if (pd.qfamily != QEM_Q_DIRICHLET || pd.dim != d.dim)
                    return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": a categorical latent's parent is a Dirichlet latent over the same categories");
            }
        }
        if (d.qfamily == QEM_Q_DIRICHLET) {
            if (d.dim < 2) return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": a Dirichlet latent has dim = C >= 2 components");
            if (d.parent0 >= 0) return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": the Dirichlet prior takes no parent");
            if (!(d.q0a > 0.0) || !(d.shape > 0.0))
                return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": Dirichlet concentrations (q0a, shape) must be > 0");
        }
        for (int q : {d.parent0, d.parent1})
            if (q < -1 || q >= v) return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": parents must precede the node");
        if (static_cast<long long>(d.n) * K * d.dim >= (1LL << 32))
            return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": n*K*dim must be below 2^32");
        const bool needs0 = d.prior == QEM_PRIOR_GAMMA_PARENTS || d.prior == QEM_PRIOR_NORMAL_LOGSCALE;
        if (needs0 && d.parent0 < 0) return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": prior needs parent0");
        if (d.prior == QEM_PRIOR_GAMMA_PARENTS && d.parent1 < 0)
            return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": Gamma(shape, rate) prior needs two parents");
        if (d.prior == QEM_PRIOR_GAMMA && d.parent0 >= 0)
            return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": constant Gamma prior takes no parent");
        if (d.prior != QEM_PRIOR_GAMMA_PARENTS && d.parent1 >= 0)
            return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": parent1 only for Gamma(shape, rate)");
        if (d.prior == QEM_PRIOR_NORMAL && d.var <= 0.0) return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": var must be > 0");
        if (!(d.q0b > 0.0) || (is_gamma_q(d.qfamily) && !(d.q0a > 0.0)))
            return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": initial proposal needs var (rate, shape) > 0");
        if (d.prior == QEM_PRIOR_GAMMA && (d.shape <= 0.0 || d.rate <= 0.0))
            return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": Gamma constants must be > 0");
        if (d.parent0 >= 0) {
            const int np = m->nodes[d.parent0].n;
            if (np > 1) {
                if (!d.parent_index) return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": parent_index required");
                p.pidx.assign(d.parent_index, d.parent_index + d.n);
                for (int32_t x : p.pidx)
                    if (x < 0 || x >= np) return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": parent_index out of range");
                p.has_pidx = true;
            }
            if (d.prior == QEM_PRIOR_NORMAL && m->nodes[d.parent0].dim != d.dim)
                return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": parent dimension differs");
            if (d.prior == QEM_PRIOR_BERNOULLI_LOGIT && m->nodes[d.parent0].dim != 1)
                return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": the Bernoulli logit parent must be scalar");
        }
        p.d.parent_index = nullptr;
        if (d.chain_len > 1) {
            if (d.n % d.chain_len) return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": n must be a multiple of chain_len");
            if (d.prior != QEM_PRIOR_NORMAL || d.qfamily != QEM_Q_GAUSS || d.dim != 1)
                return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": chains are scalar Gaussian random walks");
            if (d.init_var <= 0.0) return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": init_var must be > 0");
            if (p.has_pidx)
                for (int i = 0; i < d.n; ++i)
                    if (p.pidx[i] != p.pidx[i - i % d.chain_len])
                        return fail(c, QEM_E_INVALID, "node " + std::to_string(v) + ": a series takes one parent instance");
        }
    }
    c->obs.assign(m->obs, m->obs + m->n_obs);
    for (int o = 0; o < m->n_obs; ++o) {
        const qem_obs_desc& ob = c->obs[o];
        if (ob.node < 0 || ob.node >= N) return fail(c, QEM_E_INVALID, "observation " + std::to_string(o) + ": bad node");
        if (ob.n_per < 1 || !ob.x) return fail(c, QEM_E_INVALID, "observation " + std::to_string(o) + ": needs n_per >= 1 and data");
        NodeP& p = c->nodes[ob.node];
        if (ob.kind == QEM_OBS_GAUSS) {
            if (p.gobs >= 0) return fail(c, QEM_E_UNSUPPORTED, "one Gaussian observation set per node");
            if (ob.var <= 0.0) return fail(c, QEM_E_INVALID, "observation variance must be > 0");
            if (p.d.qfamily != QEM_Q_GAUSS) return fail(c, QEM_E_UNSUPPORTED, "Gaussian observations of a Gamma node");
            p.gobs = o;
        } else if (ob.kind == QEM_OBS_POISSON) {
            if (p.pobs >= 0) return fail(c, QEM_E_UNSUPPORTED, "one Poisson observation set per node");
            if (!is_gamma_q(p.d.qfamily)) return fail(c, QEM_E_UNSUPPORTED, "Poisson rates need a Gamma proposal");
            p.pobs = o;
        } else if (ob.kind == QEM_OBS_BERNOULLI_LOGIT) {
            if (p.bobs >= 0) return fail(c, QEM_E_UNSUPPORTED, "one Bernoulli observation set per node");
            if (ob.coef < 0 || ob.coef >= ob.node) return fail(c, QEM_E_INVALID, "Bernoulli coefficient node must precede the node");
            const qem_node_desc& cd = c->nodes[ob.coef].d;
            if (cd.n != 1 || cd.dim != ob.n_cov || ob.n_cov < 1 || !ob.cov)
                return fail(c, QEM_E_SHAPE, "Bernoulli coefficients: one instance of dimension n_cov and covariates");
            if (p.d.dim != 1 || p.d.qfamily != QEM_Q_GAUSS) return fail(c, QEM_E_UNSUPPORTED, "Bernoulli-logit offsets are scalar Gaussian");
            p.bobs = o;
        } else if (ob.kind == QEM_OBS_GAUSS_MIXTURE) {
            if (p.mobs >= 0) return fail(c, QEM_E_UNSUPPORTED, "one Gaussian-mixture observation set per node");
            if (p.d.qfamily != QEM_Q_CATEGORICAL) return fail(c, QEM_E_UNSUPPORTED, "Gaussian-mixture observations need a categorical latent");
            if (!ob.cov || !(ob.var > 0.0)) return fail(c, QEM_E_INVALID, "Gaussian-mixture observations need the component means and var > 0");
            p.mobs = o;
        } else if (ob.kind == QEM_OBS_CATEGORICAL) {
            if (p.cobs >= 0) return fail(c, QEM_E_UNSUPPORTED, "one categorical observation set per node");
            if (p.d.qfamily != QEM_Q_DIRICHLET) return fail(c, QEM_E_UNSUPPORTED, "categorical observations need a Dirichlet latent");
            p.cobs = o;
        } else if (ob.kind == QEM_OBS_DETECTION) {
            if (p.dobs >= 0) return fail(c, QEM_E_UNSUPPORTED, "one detection set per node");
            if (p.d.qfamily != QEM_Q_BERNOULLI) return fail(c, QEM_E_UNSUPPORTED, "detections need a Bernoulli latent");
            if (!(ob.var > 0.0 && ob.var < 1.0)) return fail(c, QEM_E_INVALID, "detection probability must be in (0, 1)");
            p.dobs = o;
        } else {
            return fail(c, QEM_E_INVALID, "observation " + std::to_string(o) + ": bad kind");
        }
    }
    // factor parents and kinds
    for (int v = 0; v < N; ++v) {
        NodeP& p = c->nodes[v];
        auto add = [&](int q) { if (q >= 0 && q != p.fp[0] && q != p.fp[1]) p.fp[p.nfp++] = q; };
        add(p.d.parent0);
        add(p.d.parent1);
        if (p.bobs >= 0) {
            if (p.nfp == 2) return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": more than two factor parents");
            add(c->obs[p.bobs].coef);
        }
        for (int q = 0; q < p.nfp; ++q)
            if (c->nodes[p.fp[q]].d.qfamily == QEM_Q_DIRICHLET && p.d.prior != QEM_PRIOR_CATEGORICAL)
                return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": nodes under a Dirichlet latent other than categorical ones");
        if (p.d.chain_len > 1) {
            if (p.bobs >= 0) return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": chains take no Bernoulli-logit observations");
            p.kind = p.nfp ? K_CHAINP : K_CHAIN;
            if (p.nfp && c->nodes[p.fp[0]].d.chain_len > 1)
                return fail(c, QEM_E_UNSUPPORTED, "children of chain nodes");
            continue;
        }
        if (p.nfp == 0) p.kind = K_ROOT;
        else if (p.nfp == 1) {
            p.kind = K_SINGLE;
            if (p.bobs >= 0 && p.d.parent0 >= 0)
                return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": Bernoulli coefficient node and prior parent must differ");
            if (c->nodes[p.fp[0]].d.chain_len > 1) return fail(c, QEM_E_UNSUPPORTED, "children of chain nodes");
            if (p.d.prior == QEM_PRIOR_NORMAL_LOGSCALE &&
                (p.d.dim != 1 || c->nodes[p.d.parent0].d.n != 1 || c->nodes[p.d.parent0].d.dim != 1))
                return fail(c, QEM_E_UNSUPPORTED, "log-scale prior: scalar node with a scalar single-instance parent");
        } else {
            p.kind = K_PAIRCHILD;
            for (int q : p.fp) {
                const NodeP& r = c->nodes[q];
                if (r.nfp != 0 || r.d.chain_len > 1 || r.d.n != 1)
                    return fail(c, QEM_E_UNSUPPORTED, "two-parent node " + std::to_string(v) + ": parents must be single-instance roots");
            }
            const bool gp = p.d.prior == QEM_PRIOR_GAMMA_PARENTS && p.bobs < 0;
            const bool lb = p.d.prior == QEM_PRIOR_NORMAL_LOGSCALE && p.bobs >= 0;
            if (!gp && !lb) return fail(c, QEM_E_UNSUPPORTED, "two-parent node " + std::to_string(v) + ": unsupported factor combination");
            if (gp && (!is_gamma_q(c->nodes[p.fp[0]].d.qfamily) || !is_gamma_q(c->nodes[p.fp[1]].d.qfamily)))
                return fail(c, QEM_E_UNSUPPORTED, "Gamma(shape, rate) parents need Gamma proposals (positive samples)");
            if (lb && c->nodes[p.fp[0]].d.dim != 1) return fail(c, QEM_E_UNSUPPORTED, "log-scale parent must be scalar");
            if (c->pa < 0) { c->pa = p.fp[0]; c->pb = p.fp[1]; }
            else if (c->pa != p.fp[0] || c->pb != p.fp[1])
                return fail(c, QEM_E_UNSUPPORTED, "all two-parent nodes must share one root pair");
            if (K > 256) return fail(c, QEM_E_SHAPE, "two-parent nodes support K <= 256");
            if (p.bobs >= 0 && static_cast<size_t>(K) * K * c->eb() > 48 * 1024)
                return fail(c, QEM_E_SHAPE, "two-parent likelihood table of K*K entries must fit 48 KiB of LDS");
        }
    }
    if (c->pa >= 0) {
        c->nodes[c->pa].kind = K_PAIRROOT;
        c->nodes[c->pb].kind = K_PAIRROOT;
    }
    const size_t lds_cap = 64 * 1024;
    for (int v = 0; v < N; ++v) {
        const NodeP& p = c->nodes[v];
        if ((p.kind == K_CHAIN || p.kind == K_CHAINP) && K > 512) return fail(c, QEM_E_SHAPE, "chains support K <= 512");
        if (p.kind == K_CHAINP) {
            if (c->bexp()) return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": chains under a parent in BF16-exp mode");
            const Kind pk = c->nodes[p.fp[0]].kind;
            if (pk != K_ROOT && pk != K_SINGLE)
                return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": a chain's parent must be a root or plate node");
        }
        if (p.kind == K_CHAIN && c->bexp() && !qemk::chain_bexp_supported(K))
            return fail(c, QEM_E_UNSUPPORTED, "BF16-exp chains need K in {64, 128, 256}");
        if (p.kind == K_SINGLE && p.d.prior == QEM_PRIOR_NORMAL && p.bobs < 0 &&
            static_cast<size_t>(2) * K * p.d.dim * c->eb() > lds_cap)
            return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": 2*K*dim samples must fit 64 KiB of LDS");
        if (p.bobs >= 0) {
            const size_t J = c->obs[p.bobs].n_per, D = static_cast<size_t>(c->obs[p.bobs].n_cov);
            if ((((J + 3) & ~static_cast<size_t>(3)) * K + J + K) * c->eb() + (J * D + K * (D + 1)) * 8 > lds_cap)
                return fail(c, QEM_E_SHAPE, "node " + std::to_string(v) + ": Bernoulli table of n_per*K entries (n_per rounded up to a multiple of 4) plus the FP64 covariates (n_per*n_cov) and beta samples (K*(n_cov+1)) must fit 64 KiB of LDS");
        }
        if (p.kind == K_ROOT && p.d.prior != QEM_PRIOR_NORMAL && p.d.prior != QEM_PRIOR_GAMMA &&
            p.d.prior != QEM_PRIOR_BERNOULLI_LOGIT && p.d.prior != QEM_PRIOR_DIRICHLET &&
            p.d.prior != QEM_PRIOR_CATEGORICAL)
            return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": root prior must be Normal, Gamma, Bernoulli-logit, Dirichlet or categorical");
        if (p.d.prior == QEM_PRIOR_GAMMA && !is_gamma_q(p.d.qfamily))
            return fail(c, QEM_E_UNSUPPORTED, "node " + std::to_string(v) + ": Gamma prior needs a Gamma proposal");
    }
    // children lists (single-parent children, grouped by parent instance, stable
    // order); a chain under a parent contributes one message per series
    for (int v = 0; v < N; ++v) {
        NodeP& ch = c->nodes[v];
        if (ch.kind == K_CHAINP) {
            NodeP& par = c->nodes[ch.fp[0]];
            const int T = ch.d.chain_len, G = ch.d.n / T;
            ch.sp.assign(G, 0);
            if (ch.has_pidx)
                for (int g = 0; g < G; ++g) ch.sp[g] = ch.pidx[static_cast<size_t>(g) * T];
            Csr cs;
            cs.child = v;
            cs.off.assign(par.d.n + 1, 0);
            for (int g = 0; g < G; ++g) cs.off[ch.sp[g] + 1]++;
            for (int q = 0; q < par.d.n; ++q) cs.off[q + 1] += cs.off[q];
            cs.idx.assign(G, 0);
            std::vector<int32_t> fill(cs.off.begin(), cs.off.end() - 1);
            for (int g = 0; g < G; ++g) cs.idx[fill[ch.sp[g]]++] = g;
            cs.per = regular_per(cs);
            par.children.push_back(std::move(cs));
            continue;
        }
        if (ch.kind != K_SINGLE) continue;
        NodeP& par = c->nodes[ch.fp[0]];
        Csr cs;
        cs.child = v;
        cs.off.assign(par.d.n + 1, 0);
        for (int i = 0; i < ch.d.n; ++i) cs.off[(ch.has_pidx && ch.d.parent0 == ch.fp[0] ? ch.pidx[i] : 0) + 1]++;
        for (int q = 0; q < par.d.n; ++q) cs.off[q + 1] += cs.off[q];
        cs.idx.assign(ch.d.n, 0);
        std::vector<int32_t> fill(cs.off.begin(), cs.off.end() - 1);
        for (int i = 0; i < ch.d.n; ++i) {
            const int q = (ch.has_pidx && ch.d.parent0 == ch.fp[0]) ? ch.pidx[i] : 0;
            cs.idx[fill[q]++] = i;
        }
        cs.per = regular_per(cs);
        par.children.push_back(std::move(cs));
    }
    // workspace plan
    size_t off = 0;
    auto take = [&](size_t b) { const size_t o = off; off = align256(off + std::max<size_t>(b, 1)); return o; };
    const size_t eb = c->eb();
    c->o_logphat = take(8);
    c->o_status = take(16);
    c->o_iter = take(8);
    c->o_lamt = take(8);
    c->o_lp1 = take(8);
    c->o_rootpart = take(static_cast<size_t>(qemk::MAX_CHILD_LISTS) * 1024 * 8);
    long nL = 0;
    for (int v = 0; v < N; ++v) {
        NodeP& p = c->nodes[v];
        const long n = p.d.n, d = p.d.dim;
        p.o_qp = take(n * d * 2 * 8);
        p.o_mema = take(n * d * 2 * 8);
        p.o_mone = take(n * d * 2 * 8);
        p.o_z = take(n * K * d * eb);
        p.o_u = take(n * K * eb);
        p.o_ut = take(n * K * 8);
        p.o_w = take(n * K * eb);
        if (p.has_pidx) p.o_pidx = take(n * 4);
        if (p.gobs >= 0) { p.o_gxbar = take(n * d * 8); p.o_gss = take(n * d * 8); }
        if (p.pobs >= 0) { p.o_psy = take(n * 8); p.o_pslg = take(n * 8); }
        if (p.dobs >= 0) { p.o_dsy = take(n * 8); p.o_dslg = take(n * 8); }
        if (p.cobs >= 0) p.o_ccnt = take(n * d * 8);
        if (p.mobs >= 0) p.o_mlik = take(n * d * 8);
        switch (p.kind) {
            case K_ROOT: p.Lslot = nL; p.nL = n; nL += n; break;
            case K_CHAIN: {
                const long T = p.d.chain_len, G = n / T;
                // chains evaluate their step factors in the kernels; FP32/FP64 ones keep
                // the table only when asked (BF16-exp never: its fold forms the tiles)
                p.has_F = c->chain_tables && !c->no_tables && !c->bexp();
                if (p.has_F) p.o_F = take(static_cast<size_t>(G) * (T - 1) * K * K * eb);
                p.o_msg = take(static_cast<size_t>(n) * K * 8);
                p.Lslot = nL; p.nL = G; nL += G;
                break;
            }
            case K_CHAINP: {
                const long T = p.d.chain_len, G = n / T;
                const size_t rows = static_cast<size_t>(G) * K * T * K;   // virtual series x steps x K
                p.o_sp = take(G * 4);
                p.o_msg = take(rows * 8);
                p.o_vL = take(static_cast<size_t>(G) * K * 8);
                if (qemk::chainp_mfma_supported(K)) {
                    // per-block FP64 weight sums; u-tilde is rebuilt from the messages
                    p.o_vw = take(static_cast<size_t>(G) * qemk::chainp_mfma_blocks(K) * T * K * 8);
                } else {
                    p.o_vut = take(rows * 8);
                    p.o_vw = take(rows * eb);
                }
                break;
            }
            case K_SINGLE:
                p.has_F = !(c->no_tables && factor_in_kernel(c, p));
                if (p.has_F) p.o_F = take(static_cast<size_t>(n) * K * K * eb);
                p.o_msg = take(static_cast<size_t>(n) * K * 8);
                break;
            case K_PAIRCHILD:
                p.o_msg = take(static_cast<size_t>(n) * K * K * 8);
                p.o_ga0 = take(K * 8); p.o_ga1 = take(K * 8); p.o_hb = take(K * 8);
                p.o_gk = take(n * K * 8); p.o_hk = take(n * K * 8);
                p.o_C = take(static_cast<size_t>(K) * K * 8);
                if (qemk::twoparent_mfma_supported(c->f64(), K, K, K)) p.o_tpflag = take(static_cast<size_t>(n));
                if (p.bobs >= 0) { p.o_F = take(static_cast<size_t>(n) * K * K * eb); p.has_F = true; }
                break;
            case K_PAIRROOT: break;
        }
        for (Csr& cs : p.children) { cs.o_off = take(cs.off.size() * 4); cs.o_idx = take(cs.idx.size() * 4); }
    }
    if (c->pa >= 0) {
        c->pair_slot = nL++;
        c->o_pairM = take(static_cast<size_t>(K) * K * 8);
        c->o_pairW = take(static_cast<size_t>(K) * K * 8);
        c->o_pairScr = take(static_cast<size_t>(32) * K * K * 8);
    }
    c->nL = nL;
    c->o_Lall = take(nL * 8);
    c->bytes = off;
    for (NodeP& p : c->nodes) {
        if (p.has_pidx) c->uploads.push_back({p.o_pidx, &p.pidx});
        if (p.kind == K_CHAINP) c->uploads.push_back({p.o_sp, &p.sp});
        for (Csr& cs : p.children) {
            c->uploads.push_back({cs.o_off, &cs.off});
            c->uploads.push_back({cs.o_idx, &cs.idx});
        }
    }
    return QEM_OK;
}

hipEvent_t take_event(qem_ctx c) {
    if (!c->pool.empty()) { hipEvent_t e = c->pool.back(); c->pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one kernel launch with events when tracing is on.
struct Timed {
    qem_ctx c; int slot; hipEvent_t a = nullptr;
    Timed(qem_ctx c_, int node, int phase) : c(c_), slot((node + 1) * QEM_PH_COUNT + phase) {
        if (c->timing && (a = take_event(c))) hipEventRecord(a, c->s);
    }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) { c->pool.push_back(a); return; }
        hipEventRecord(b, c->s);
        c->recs.push_back({slot, a, b});
    }
};

qem_status need_ws(qem_ctx c) {
    if (!c) return QEM_E_INVALID;
    if (!c->ws) return fail(c, QEM_E_STATE, "workspace not bound");
    return QEM_OK;
}

void drop_graphs(qem_ctx c) {
    if (c->gexec) { hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
    if (c->graph) { hipGraphDestroy(c->graph); c->graph = nullptr; }
    if (c->gexec_u) { hipGraphExecDestroy(c->gexec_u); c->gexec_u = nullptr; }
    if (c->graph_u) { hipGraphDestroy(c->graph_u); c->graph_u = nullptr; }
}

}  // namespace

extern "C" {

qem_status qem_create(qem_ctx* out, const qem_model_desc* model, int32_t K, int32_t prec, void* stream) {
    return qem_create_ex(out, model, K, prec, 0, stream);
}

qem_status qem_create_ex(qem_ctx* out, const qem_model_desc* model, int32_t K, int32_t prec, uint32_t flags,
                         void* stream) {
    if (!out || !model) { g_create_err = "null argument"; return QEM_E_INVALID; }
    *out = nullptr;
    if (K < 1 || K > 512) { g_create_err = "K must be in [1, 512]"; return QEM_E_SHAPE; }
    if (prec < QEM_FP64 || prec > QEM_BF16EXP) { g_create_err = "bad precision"; return QEM_E_INVALID; }
    if (flags & ~(QEM_CREATE_NO_TABLES | QEM_CREATE_CHAIN_TABLES)) {
        g_create_err = "unknown create flags";
        return QEM_E_INVALID;
    }
    qem_ctx c = new qem_ctx_s();
    c->K = K;
    c->prec = prec;
    c->no_tables = (flags & QEM_CREATE_NO_TABLES) != 0;
    c->chain_tables = (flags & QEM_CREATE_CHAIN_TABLES) != 0;
    c->s = static_cast<hipStream_t>(stream);
    const qem_status st = validate_and_plan(c, model);
    if (st != QEM_OK) {
        g_create_err = c->err;
        delete c;
        return st;
    }
    *out = c;
    return QEM_OK;
}

void qem_destroy(qem_ctx ctx) {
    if (!ctx) return;
    drop_graphs(ctx);
    if (ctx->cap) hipStreamDestroy(ctx->cap);
    for (auto& r : ctx->recs) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
    for (hipEvent_t e : ctx->pool) hipEventDestroy(e);
    delete ctx;
}

qem_status qem_timing(qem_ctx c, int32_t enable) {
    if (!c) return QEM_E_INVALID;
    QEM_HIP(hipStreamSynchronize(c->s));
    for (auto& r : c->recs) { c->pool.push_back(r.a); c->pool.push_back(r.b); }
    c->recs.clear();
    c->tms.assign((c->nodes.size() + 1) * QEM_PH_COUNT, 0.0);
    c->tcount.assign((c->nodes.size() + 1) * QEM_PH_COUNT, 0);
    c->timing = enable != 0;
    return QEM_OK;
}

qem_status qem_timing_read(qem_ctx c, int32_t node, int32_t phase, double* total_ms, int64_t* launches) {
    if (!c) return QEM_E_INVALID;
    if (node < -1 || node >= static_cast<int>(c->nodes.size()) || phase < 0 || phase >= QEM_PH_COUNT)
        return fail(c, QEM_E_INVALID, "bad node or phase");
    if (c->tms.empty()) {
        c->tms.assign((c->nodes.size() + 1) * QEM_PH_COUNT, 0.0);
        c->tcount.assign((c->nodes.size() + 1) * QEM_PH_COUNT, 0);
    }
    QEM_HIP(hipStreamSynchronize(c->s));
    for (auto& r : c->recs) {
        float ms = 0.f;
        QEM_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        c->tms[r.slot] += ms;
        c->tcount[r.slot] += 1;
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->recs.clear();
    const int slot = (node + 1) * QEM_PH_COUNT + phase;
    if (total_ms) *total_ms = c->tms[slot];
    if (launches) *launches = c->tcount[slot];
    return QEM_OK;
}

const char* qem_last_error(qem_ctx ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

size_t qem_workspace_bytes(qem_ctx ctx) { return ctx ? ctx->bytes : 0; }

qem_status qem_bind_workspace(qem_ctx c, void* dev, size_t bytes) {
    if (!c || !dev) return fail(c, QEM_E_INVALID, "null workspace");
    if (bytes < c->bytes) return fail(c, QEM_E_STATE, "workspace smaller than qem_workspace_bytes()");
    if (reinterpret_cast<uintptr_t>(dev) % 256) return fail(c, QEM_E_INVALID, "workspace must be 256-byte aligned");
    // captured qem_run graphs hold the previous workspace's addresses
    drop_graphs(c);
    c->ws = static_cast<char*>(dev);
    for (auto& up : c->uploads)
        QEM_HIP(hipMemcpyAsync(c->ws + up.first, up.second->data(), up.second->size() * 4, hipMemcpyHostToDevice, c->s));
    for (NodeP& p : c->nodes) {
        if (p.gobs >= 0) {
            const qem_obs_desc& ob = c->obs[p.gobs];
            QEM_HIP(qemk::stats_gauss(c->s, ob.x, p.d.n, ob.n_per, p.d.dim, c->d(p.o_gxbar), c->d(p.o_gss)));
        }
        if (p.pobs >= 0) {
            const qem_obs_desc& ob = c->obs[p.pobs];
            QEM_HIP(qemk::stats_poisson(c->s, ob.x, p.d.n, ob.n_per, c->d(p.o_psy), c->d(p.o_pslg)));
        }
        if (p.dobs >= 0) {   // the detection count sum_r y per instance
            const qem_obs_desc& ob = c->obs[p.dobs];
            QEM_HIP(qemk::stats_poisson(c->s, ob.x, p.d.n, ob.n_per, c->d(p.o_dsy), c->d(p.o_dslg)));
        }
        if (p.mobs >= 0) {   // per-category log-likelihood of each instance's data
            const qem_obs_desc& ob = c->obs[p.mobs];
            QEM_HIP(qemk::stats_gauss_mixture(c->s, ob.x, ob.cov, p.d.n, ob.n_per, p.d.dim, ob.var, c->d(p.o_mlik)));
        }
        if (p.cobs >= 0) {   // per-category counts
            const qem_obs_desc& ob = c->obs[p.cobs];
            QEM_HIP(qemk::stats_categorical(c->s, ob.x, p.d.n, ob.n_per, p.d.dim, c->d(p.o_ccnt)));
        }
    }
    QEM_HIP(qemk::reset_status(c->s, c->at<uint32_t>(c->o_status)));
    if (qem_status st = qem_init(c, -1)) return st;
    QEM_HIP(hipStreamSynchronize(c->s));
    return QEM_OK;
}

namespace {
qem_status init_nodes(qem_ctx c, int32_t node, int set_q) {
    if (qem_status st = need_ws(c)) return st;
    if (node < -1 || node >= static_cast<int>(c->nodes.size())) return fail(c, QEM_E_INVALID, "bad node id");
    for (int v = 0; v < static_cast<int>(c->nodes.size()); ++v) {
        if (node >= 0 && v != node) continue;
        const NodeP& p = c->nodes[v];
        QEM_HIP(qemk::init_q(c->s, c->d(p.o_qp), c->d(p.o_mema), static_cast<long>(p.d.n) * p.d.dim, p.d.qfamily,
                             set_q, p.d.q0a, p.d.q0b, p.d.dim));
    }
    return QEM_OK;
}
}  // namespace

qem_status qem_init(qem_ctx c, int32_t node) { return init_nodes(c, node, 1); }

qem_status qem_init_from_q(qem_ctx c, int32_t node) { return init_nodes(c, node, 0); }

qem_status qem_tensor(qem_ctx c, int32_t node, int32_t kind, qem_tensor_info* out) {
    if (!c || !out) return QEM_E_INVALID;
    std::memset(out, 0, sizeof(*out));
    const int K = c->K;
    const int tdt = c->f64() ? QEM_DT_F64 : QEM_DT_F32;
    auto set = [&](size_t off, int dt, std::initializer_list<int64_t> sh) {
        out->offset = off;
        out->dtype = dt;
        out->ndim = static_cast<int32_t>(sh.size());
        size_t cnt = 1;
        int j = 0;
        for (int64_t x : sh) { out->shape[j++] = x; cnt *= static_cast<size_t>(x); }
        out->bytes = cnt * (dt == QEM_DT_F64 ? 8 : dt == QEM_DT_BF16 ? 2 : 4);
        return QEM_OK;
    };
    if (node == -1) {
        switch (kind) {
            case QEM_T_LOGPHAT: return set(c->o_logphat, QEM_DT_F64, {1});
            case QEM_T_STATUS: return set(c->o_status, QEM_DT_U32, {4});
            case QEM_T_PAIR_M: if (c->pa >= 0) return set(c->o_pairM, QEM_DT_F64, {K, K}); break;
            case QEM_T_PAIR_W: if (c->pa >= 0) return set(c->o_pairW, QEM_DT_F64, {K, K}); break;
            case QEM_T_ROOTL: return set(c->o_Lall, QEM_DT_F64, {c->nL});
            default: break;
        }
        return fail(c, QEM_E_INVALID, "no such global tensor");
    }
    if (node < 0 || node >= static_cast<int>(c->nodes.size())) return fail(c, QEM_E_INVALID, "bad node id");
    const NodeP& p = c->nodes[node];
    const int64_t n = p.d.n, d = p.d.dim;
    switch (kind) {
        case QEM_T_QPARAM: return set(p.o_qp, QEM_DT_F64, {n, d, 2});
        case QEM_T_MEMA: return set(p.o_mema, QEM_DT_F64, {n, d, 2});
        case QEM_T_MONE: return set(p.o_mone, QEM_DT_F64, {n, d, 2});
        case QEM_T_Z: return set(p.o_z, tdt, {n, K, d});
        case QEM_T_U: return set(p.o_u, tdt, {n, K});
        case QEM_T_UT: return set(p.o_ut, QEM_DT_F64, {n, K});
        case QEM_T_W: return set(p.o_w, tdt, {n, K});
        case QEM_T_F:
            if (!p.has_F) break;
            if (p.kind == K_CHAIN) {
                const int64_t T = p.d.chain_len;
                return set(p.o_F, tdt, {n / T, T - 1, K, K});
            }
            return set(p.o_F, tdt, {n, K, K});
        case QEM_T_MSG:
            if (p.kind == K_SINGLE) return set(p.o_msg, QEM_DT_F64, {n, K});
            if (p.kind == K_PAIRCHILD) return set(p.o_msg, QEM_DT_F64, {n, K, K});
            if (p.kind == K_CHAIN) return set(p.o_msg, QEM_DT_F64, {n / p.d.chain_len, p.d.chain_len, K});
            if (p.kind == K_CHAINP) return set(p.o_msg, QEM_DT_F64, {n / p.d.chain_len, K, p.d.chain_len, K});
            break;
        case QEM_T_ROOTL:
            if (p.nL > 0) return set(c->o_Lall + p.Lslot * 8, QEM_DT_F64, {p.nL});
            if (p.kind == K_CHAINP) return set(p.o_vL, QEM_DT_F64, {n / p.d.chain_len, K});
            break;
        default: break;
    }
    return fail(c, QEM_E_INVALID, "node " + std::to_string(node) + " has no tensor of kind " + std::to_string(kind));
}

namespace {
qem_status sample_impl(qem_ctx c, uint64_t seed, uint64_t iter, const uint64_t* iter_dev) {
    QEM_HIP(qemk::reset_status(c->s, c->at<uint32_t>(c->o_status)));
    for (size_t v = 0; v < c->nodes.size(); ++v) {
        const NodeP& p = c->nodes[v];
        if (p.d.qfamily == QEM_Q_GAUSS)
            QEM_LAUNCH(v, QEM_PH_SAMPLE, qemk::sample_gauss(c->s, c->f64(), c->at(p.o_z), c->d(p.o_qp), p.d.n, c->K, p.d.dim, seed,
                                       static_cast<uint32_t>(iter), static_cast<uint32_t>(v), iter_dev));
        else if (p.d.qfamily == QEM_Q_CATEGORICAL)
            QEM_LAUNCH(v, QEM_PH_SAMPLE, qemk::sample_categorical(c->s, c->f64(), c->at(p.o_z), c->d(p.o_qp), p.d.n, c->K, p.d.dim,
                                             seed, static_cast<uint32_t>(iter), static_cast<uint32_t>(v), iter_dev));
        else if (p.d.qfamily == QEM_Q_DIRICHLET)
            QEM_LAUNCH(v, QEM_PH_SAMPLE, qemk::sample_dirichlet(c->s, c->f64(), c->at(p.o_z), c->d(p.o_qp), p.d.n, c->K, p.d.dim,
                                           seed, static_cast<uint32_t>(iter), static_cast<uint32_t>(v), iter_dev));
        else if (p.d.qfamily == QEM_Q_BERNOULLI)
            QEM_LAUNCH(v, QEM_PH_SAMPLE, qemk::sample_bernoulli(c->s, c->f64(), c->at(p.o_z), c->d(p.o_qp), p.d.n, c->K, seed,
                                           static_cast<uint32_t>(iter), static_cast<uint32_t>(v), iter_dev));
        else
            QEM_LAUNCH(v, QEM_PH_SAMPLE, qemk::sample_gamma(c->s, c->f64(), c->at(p.o_z), c->d(p.o_qp), p.d.n, c->K, seed,
                                       static_cast<uint32_t>(iter), static_cast<uint32_t>(v), iter_dev));
    }
    return QEM_OK;
}
}  // namespace

qem_status qem_sample(qem_ctx c, uint64_t seed, uint64_t iter) {
    if (!c) return QEM_E_INVALID;
    if (iter > 0xFFFFFFFFull) return fail(c, QEM_E_INVALID, "iteration numbers are 32-bit Philox counter words");
    if (qem_status st = need_ws(c)) return st;
    return sample_impl(c, seed, iter, nullptr);
}

namespace {

qemk::UnaryArgs unary_args(qem_ctx c, const NodeP& p) {
    qemk::UnaryArgs a{};
    a.z = c->at(p.o_z); a.u = c->at(p.o_u); a.qp = c->d(p.o_qp);
    a.n = p.d.n; a.K = c->K; a.d = p.d.dim; a.qfamily = p.d.qfamily;
    a.prior_term = qemk::PT_NONE;
    if (p.kind == K_CHAIN) {
        a.prior_term = qemk::PT_CHAIN_START; a.pb = p.d.init_b; a.pvar = p.d.init_var; a.chain_T = p.d.chain_len;
    } else if (p.d.prior == QEM_PRIOR_NORMAL && p.d.parent0 < 0) {
        a.prior_term = qemk::PT_NORMAL; a.pb = p.d.b; a.pvar = p.d.var;
    } else if (p.d.prior == QEM_PRIOR_GAMMA) {
        a.prior_term = qemk::PT_GAMMA; a.pshape = p.d.shape; a.prate = p.d.rate;
    } else if (p.d.prior == QEM_PRIOR_BERNOULLI_LOGIT && p.d.parent0 < 0) {
        a.prior_term = qemk::PT_BERN; a.pb = p.d.b;
    } else if (p.d.prior == QEM_PRIOR_DIRICHLET) {
        a.prior_term = qemk::PT_DIR; a.pshape = p.d.shape;
    } else if (p.d.prior == QEM_PRIOR_CATEGORICAL && p.d.parent0 < 0) {
        a.prior_term = qemk::PT_CAT;
    }
    if (p.cobs >= 0) a.c_cnt = c->d(p.o_ccnt);
    if (p.mobs >= 0) a.m_lik = c->d(p.o_mlik);
    if (p.gobs >= 0) {
        a.g_xbar = c->d(p.o_gxbar); a.g_ss = c->d(p.o_gss);
        a.g_J = c->obs[p.gobs].n_per; a.g_var = c->obs[p.gobs].var;
    }
    if (p.pobs >= 0) { a.p_sy = c->d(p.o_psy); a.p_slg = c->d(p.o_pslg); a.p_J = c->obs[p.pobs].n_per; }
    if (p.dobs >= 0) {
        const qem_obs_desc& ob = c->obs[p.dobs];
        a.d_sy = c->d(p.o_dsy); a.d_R = ob.n_per;
        a.d_l1 = std::log(ob.var); a.d_l0 = std::log1p(-ob.var);
    }
    qemk::unary_consts(a);
    return a;
}

// A linear-Gaussian plate node or a chain (FP32/FP64) whose pair table the
// fused step evaluates inside the forward kernel.
bool table_in_fwd(qem_ctx c, const NodeP& p) { return factor_in_kernel(c, p); }

// The factor tables of node v that involve a parent (every log-factor but the
// unary one); none for a node whose table is not kept.
qem_status pair_tables(qem_ctx c, int v) {
    const int K = c->K;
    const bool f64 = c->f64();
    const NodeP& p = c->nodes[v];
    if (!p.has_F && factor_in_kernel(c, p)) return QEM_OK;
    if (p.kind == K_CHAIN) {
        const long T = p.d.chain_len, G = p.d.n / T;
        QEM_LAUNCH(v, QEM_PH_PAIRTABLE, qemk::pair_normal(c->s, f64, c->at(p.o_F), c->at(p.o_z), c->at(p.o_z), nullptr, G * (T - 1), K, K,
                                  1, p.d.a, p.d.b, p.d.var, static_cast<int>(T)));
    } else if (p.kind == K_SINGLE) {
        const NodeP& par = c->nodes[p.fp[0]];
        if (p.bobs >= 0) {
            const qem_obs_desc& ob = c->obs[p.bobs];
            QEM_LAUNCH(v, QEM_PH_PAIRTABLE, qemk::pair_bernoulli(c->s, f64, c->at(p.o_F), c->at(p.o_z), c->at(par.o_z), ob.x, ob.cov,
                                         nullptr, nullptr, p.d.n, K, K, ob.n_per, ob.n_cov));
        } else if (p.d.prior == QEM_PRIOR_NORMAL) {
            QEM_LAUNCH(v, QEM_PH_PAIRTABLE, qemk::pair_normal(c->s, f64, c->at(p.o_F), c->at(p.o_z), c->at(par.o_z),
                                      p.has_pidx ? c->at<int32_t>(p.o_pidx) : nullptr, p.d.n, K, K, p.d.dim,
                                      p.d.a, p.d.b, p.d.var, 0));
        } else if (p.d.prior == QEM_PRIOR_CATEGORICAL) {
            QEM_LAUNCH(v, QEM_PH_PAIRTABLE, qemk::pair_categorical(c->s, f64, c->at(p.o_F), c->at(p.o_z), c->at(par.o_z),
                                           p.has_pidx ? c->at<int32_t>(p.o_pidx) : nullptr, p.d.n, K, K,
                                           p.d.dim));
        } else if (p.d.prior == QEM_PRIOR_BERNOULLI_LOGIT) {
            QEM_LAUNCH(v, QEM_PH_PAIRTABLE, qemk::pair_bern_prior(c->s, f64, c->at(p.o_F), c->at(p.o_z), c->at(par.o_z),
                                          p.has_pidx ? c->at<int32_t>(p.o_pidx) : nullptr, p.d.n, K, K,
                                          p.d.a, p.d.b));
        } else {
            QEM_LAUNCH(v, QEM_PH_PAIRTABLE, qemk::pair_logscale(c->s, f64, c->at(p.o_F), c->at(p.o_z), c->at(par.o_z), p.d.n, K, K));
        }
    } else if (p.kind == K_PAIRCHILD) {
        const NodeP& A = c->nodes[p.fp[0]];
        const NodeP& B = c->nodes[p.fp[1]];
        QEM_LAUNCH(v, QEM_PH_PAIRTABLE, qemk::twoparent_prep(c->s, f64, p.d.prior, c->at(A.o_z), c->at(B.o_z), c->at(p.o_z), p.d.n, K, K,
                                     K, c->d(p.o_ga0), c->d(p.o_ga1), c->d(p.o_gk), c->d(p.o_hb), c->d(p.o_hk),
                                     c->d(p.o_C)));
        if (p.bobs >= 0) {
            const qem_obs_desc& ob = c->obs[p.bobs];
            QEM_LAUNCH(v, QEM_PH_PAIRTABLE, qemk::pair_bernoulli(c->s, f64, c->at(p.o_F), c->at(p.o_z), c->at(B.o_z), ob.x, ob.cov,
                                         nullptr, nullptr, p.d.n, K, K, ob.n_per, ob.n_cov));
        }
    }
    return QEM_OK;
}

}  // namespace

qem_status qem_logfactors(qem_ctx c) {
    if (qem_status st = need_ws(c)) return st;
    for (size_t v = 0; v < c->nodes.size(); ++v) {
        const qemk::UnaryArgs a = unary_args(c, c->nodes[v]);
        QEM_LAUNCH(v, QEM_PH_UNARY, qemk::unary(c->s, c->f64(), a));
        if (qem_status st = pair_tables(c, static_cast<int>(v))) return st;
    }
    return QEM_OK;
}

namespace {

qemk::TwoParentArgs tp_args(qem_ctx c, const NodeP& p) {
    qemk::TwoParentArgs a{};
    const bool gp = p.d.prior == QEM_PRIOR_GAMMA_PARENTS;
    a.ga0 = c->d(p.o_ga0); a.ga1 = c->d(p.o_ga1); a.gk = c->d(p.o_gk);
    a.hb = gp ? c->d(p.o_hb) : nullptr;
    a.hk = gp ? c->d(p.o_hk) : nullptr;
    a.hmat = gp ? nullptr : c->at(p.o_F);
    a.C = gp ? c->d(p.o_C) : nullptr;
    a.ut = c->d(p.o_ut); a.m = c->d(p.o_msg);
    a.n = p.d.n; a.Ka = c->K; a.Kb = c->K; a.K = c->K;
    a.flags = p.o_tpflag ? c->at<uint8_t>(p.o_tpflag) : nullptr;
    return a;
}

// Child messages above which the root finisher's gather is split into one
// workgroup per subset (a single workgroup gathers 128 KB in about 8 us).
constexpr long ROOT_WIDE_GATHER = 32768;

// What the fused iteration folds into neighbouring kernels; the stage calls
// pass none.
struct Fusion {
    double lam = 0.0;
    const double* lam_dev = nullptr;   // this iteration's EMA weight (device scalar)
    uint64_t* iter_dev = nullptr;
    int root_fin = -1;        // single-instance root finished by one kernel (k_root_fin)
    bool root_mstep = true;   // the root finisher also does the root's M-step
    std::vector<char> fwd_sample;   // nodes whose plate forward draws their samples (sample_in_plate_fwd)
    uint64_t seed = 0;
    uint32_t iter = 0;
};

// Whether a fused iteration lets the plate forward of node v draw the node's
// samples and unary factor (the FP32 K = 64 kernel, Gaussian proposals of at
// most 4 dimensions, the pair factor evaluated in the kernel, no child node
// to gather): its wave per instance then replaces the sampling launch's.
bool sample_in_plate_fwd(qem_ctx c, const NodeP& p) {
    return !c->f64() && p.kind == K_SINGLE && p.children.empty() && factor_in_kernel(c, p) &&
           p.d.qfamily == QEM_Q_GAUSS && qemk::plate_fwd_samples_supported(false, c->K, c->K, p.d.dim);
}

bool fwd_samples(const Fusion* fu, int v) {
    return fu && v >= 0 && static_cast<size_t>(v) < fu->fwd_sample.size() && fu->fwd_sample[v];
}

// The virtual-series description of a chain under a parent: K parent samples
// per series, the start term log N(x_0; beta + init_b, init_var).
qemk::VSeries vseries(qem_ctx c, const NodeP& p) {
    const NodeP& par = c->nodes[p.fp[0]];
    qemk::VSeries vs{};
    vs.Kb = c->K;
    vs.sp = c->at<int32_t>(p.o_sp);
    vs.zb = c->at(par.o_z);
    vs.wb = c->at(par.o_w);
    vs.usrc = c->d(p.o_ut);
    vs.a = p.d.a; vs.b = p.d.b;
    vs.ib = p.d.init_b;
    vs.ic0 = -0.5 * std::log(2.0 * M_PI * p.d.init_var);
    vs.ihp = 0.5 / p.d.init_var;
    return vs;
}

qemk::ChildLists child_lists(qem_ctx c, const NodeP& p, size_t first, size_t count) {
    qemk::ChildLists cl{};
    cl.n = static_cast<int>(count);
    for (size_t q = 0; q < count; ++q) {
        const Csr& cs = p.children[first + q];
        const NodeP& ch = c->nodes[cs.child];
        cl.mc[q] = c->d(ch.kind == K_CHAINP ? ch.o_vL : ch.o_msg);
        cl.off[q] = c->at<int32_t>(cs.o_off);
        cl.idx[q] = c->at<int32_t>(cs.o_idx);
        cl.per[q] = cs.per;
    }
    return cl;
}

// Whether the fused iteration's plate forward of node v (pair table in the
// kernel, at most MAX_CHILD_LISTS child lists) forms ut itself.
bool gather_in_plate_fwd(qem_ctx c, int v, const NodeP& p, const Fusion* fu) {
    return fu && v != fu->root_fin && p.kind == K_SINGLE && !p.children.empty() &&
           p.children.size() <= static_cast<size_t>(qemk::MAX_CHILD_LISTS) && c->K <= 512 && table_in_fwd(c, p);
}

// ut = u + child messages.  In the fused iteration nodes without children
// had ut written by their sampling kernel, and the root finisher and the
// in-kernel plate forwards gather their own.
qem_status gather_children(qem_ctx c, int v, NodeP& p, const Fusion* fu) {
    if (fu && (p.children.empty() || v == fu->root_fin || gather_in_plate_fwd(c, v, p, fu))) return QEM_OK;
    const bool f64 = c->f64();
    if (p.children.empty()) {
        QEM_LAUNCH(v, QEM_PH_CHILDSUM, qemk::gather(c->s, f64, c->d(p.o_ut), c->at(p.o_u), qemk::ChildLists{}, p.d.n, c->K));
        return QEM_OK;
    }
    if (p.d.n == 1 && p.children.size() <= static_cast<size_t>(qemk::MAX_CHILD_LISTS)) {
        // a single instance with a wide gather: one workgroup per subset, then the sum in order
        long entries = 0;
        for (const Csr& cs : p.children) entries += static_cast<long>(cs.idx.size()) * c->K;
        if (entries > ROOT_WIDE_GATHER) {
            QEM_LAUNCH(v, QEM_PH_CHILDSUM, qemk::gather_subsets(c->s, child_lists(c, p, 0, p.children.size()), 0, c->K,
                                                                c->d(c->o_rootpart)));
            QEM_LAUNCH(v, QEM_PH_CHILDSUM, qemk::gather_finish(c->s, f64, c->d(p.o_ut), c->at(p.o_u),
                                                               static_cast<int>(p.children.size()), c->K,
                                                               c->d(c->o_rootpart)));
            return QEM_OK;
        }
    }
    for (size_t first = 0; first < p.children.size(); first += qemk::MAX_CHILD_LISTS) {
        const size_t count = std::min(p.children.size() - first, static_cast<size_t>(qemk::MAX_CHILD_LISTS));
        QEM_LAUNCH(v, QEM_PH_CHILDSUM, qemk::gather(c->s, f64, c->d(p.o_ut), first == 0 ? c->at(p.o_u) : nullptr,
                                                   child_lists(c, p, first, count), p.d.n, c->K));
    }
    return QEM_OK;
}

// Whether a fused iteration computes node v's moments inside the plate
// backward kernel or the root finisher (plates with (z, z^2) statistics, and
// the finished root) rather than in a moments launch.
bool moments_fused(const NodeP& p, int v, const Fusion* fu) {
    return fu && ((p.kind == K_SINGLE && p.d.qfamily != QEM_Q_GAMMA_EF) || v == fu->root_fin);
}

qem_status contract_fwd_impl(qem_ctx c, const Fusion* fu) {
    const int K = c->K;
    const bool f64 = c->f64();
    double* Lall = c->d(c->o_Lall);
    bool pair_first = true;
    for (int v = static_cast<int>(c->nodes.size()) - 1; v >= 0; --v) {
        NodeP& p = c->nodes[v];
        if (qem_status st = gather_children(c, v, p, fu)) return st;
        switch (p.kind) {
            case K_SINGLE:
                if ((fu || !p.has_F) && table_in_fwd(c, p)) {
                    const NodeP& par = c->nodes[p.fp[0]];
                    const bool g = gather_in_plate_fwd(c, v, p, fu);
                    const qemk::ChildLists cl = g ? child_lists(c, p, 0, p.children.size()) : qemk::ChildLists{};
                    const bool fs_here = fwd_samples(fu, v);
                    const qemk::FwdSample fs = fs_here ? qemk::FwdSample{unary_args(c, p),
                                                                         qemk::make_stream(fu->seed, fu->iter,
                                                                                           static_cast<uint32_t>(v)),
                                                                         fu->iter_dev, 0u}
                                                       : qemk::FwdSample{};
                    QEM_LAUNCH(v, QEM_PH_PLATE_FWD,
                               qemk::plate_fwd_pn(c->s, f64, p.has_F ? c->at(p.o_F) : nullptr, c->at(p.o_z), c->at(par.o_z),
                                                  p.has_pidx ? c->at<int32_t>(p.o_pidx) : nullptr, c->d(p.o_ut),
                                                  c->at(p.o_msg), p.d.n, K, K, p.d.dim, p.d.a, p.d.b, p.d.var,
                                                  g ? c->at(p.o_u) : nullptr, g ? &cl : nullptr,
                                                  c->at<uint32_t>(c->o_status), fs_here ? &fs : nullptr));
                    break;
                }
                QEM_LAUNCH(v, QEM_PH_PLATE_FWD, qemk::plate_fwd(c->s, f64, c->at(p.o_F), c->d(p.o_ut), c->at(p.o_msg), p.d.n, K, K,
                                                                c->at<uint32_t>(c->o_status)));
                break;
            case K_CHAIN: {
                const long T = p.d.chain_len;
                if (c->bexp()) {
                    QEM_LAUNCH(v, QEM_PH_CHAIN_FWD, qemk::chain_bexp_fwd(c->s, c->at(p.o_z), c->d(p.o_ut),
                                                                        c->d(p.o_msg), Lall + p.Lslot, p.d.n / T,
                                                                        static_cast<int>(T), K, p.d.a, p.d.b, p.d.var));
                    break;
                }
                if ((fu || !p.has_F) && table_in_fwd(c, p)) {
                    QEM_LAUNCH(v, QEM_PH_CHAIN_FWD, qemk::chain_fwd_pn(c->s, f64, p.has_F ? c->at(p.o_F) : nullptr,
                                                                      c->at(p.o_z), c->d(p.o_ut),
                                                                      c->at(p.o_msg), Lall + p.Lslot, p.d.n / T,
                                                                      static_cast<int>(T), K, p.d.a, p.d.b, p.d.var));
                    break;
                }
                QEM_LAUNCH(v, QEM_PH_CHAIN_FWD, qemk::chain_fwd(c->s, f64, c->at(p.o_F), c->d(p.o_ut), c->at(p.o_msg), Lall + p.Lslot,
                                        p.d.n / T, static_cast<int>(T), K, p.d.var));
                break;
            }
            case K_CHAINP: {
                const long T = p.d.chain_len;
                if (qemk::chainp_mfma_supported(K)) {
                    const NodeP& par = c->nodes[p.fp[0]];
                    QEM_LAUNCH(v, QEM_PH_CHAIN_FWD,
                               qemk::chainp_fwd_mfma(c->s, f64, c->at(p.o_z), c->d(p.o_ut), c->at(par.o_z),
                                                     c->at<int32_t>(p.o_sp), c->d(p.o_msg), c->d(p.o_vL), p.d.n / T,
                                                     static_cast<int>(T), K, p.d.a, p.d.b, p.d.var, p.d.init_b,
                                                     p.d.init_var));
                    break;
                }
                QEM_LAUNCH(v, QEM_PH_CHAIN_FWD, qemk::chain_fwd_pn(c->s, f64, nullptr, c->at(p.o_z), c->d(p.o_vut),
                                                                  c->at(p.o_msg), c->d(p.o_vL), p.d.n / T,
                                                                  static_cast<int>(T), K, p.d.a, p.d.b, p.d.var,
                                                                  vseries(c, p)));
                break;
            }
            case K_ROOT:
                if (fu && v == fu->root_fin) {
                    qemk::RootFinArgs a{};
                    // a wide child gather (more than ROOT_WIDE_GATHER messages) runs as one
                    // workgroup per subset first
                    long entries = 0;
                    for (const Csr& cs : p.children) entries += static_cast<long>(cs.idx.size()) * K;
                    if (entries > ROOT_WIDE_GATHER) {
                        QEM_LAUNCH(v, QEM_PH_CHILDSUM, qemk::gather_subsets(c->s, child_lists(c, p, 0, p.children.size()), 0, K,
                                                                            c->d(c->o_rootpart)));
                        a.part = c->d(c->o_rootpart);
                    }
                    a.u = c->at(p.o_u); a.ut = c->d(p.o_ut);
                    a.cl = child_lists(c, p, 0, p.children.size());
                    a.K = K; a.d = p.d.dim; a.logz = uses_log_moments(p.d.qfamily);
                    a.L = Lall + p.Lslot; a.Lall = Lall; a.nL = c->nL;
                    a.logphat = c->d(c->o_logphat); a.status = c->at<uint32_t>(c->o_status);
                    a.w = c->at(p.o_w); a.g = nullptr; a.z = c->at(p.o_z); a.mone = c->d(p.o_mone);
                    if (fu->root_mstep)
                        a.ms = qemk::MstepArgs{c->d(p.o_mema), c->d(p.o_qp), p.d.qfamily, fu->lam, a.status,
                                               fu->lam_dev};
                    a.iter_dev = fu->root_mstep ? fu->iter_dev : nullptr;
                    QEM_LAUNCH(v, QEM_PH_ROOT, qemk::root_fin(c->s, f64, a));
                    break;
                }
                QEM_LAUNCH(v, QEM_PH_ROOT, qemk::root_lse(c->s, c->d(p.o_ut), Lall + p.Lslot, p.d.n, K));
                break;
            case K_PAIRCHILD: {
                const qemk::TwoParentArgs a = tp_args(c, p);
                QEM_LAUNCH(v, QEM_PH_TP_FWD, qemk::twoparent_fwd(c->s, f64, a));
                QEM_LAUNCH(v, QEM_PH_TP_FWD, qemk::pair_sum(c->s, f64, c->d(p.o_msg), p.d.n, K, K, c->d(c->o_pairM), c->d(c->o_pairScr),
                                       pair_first ? 0 : 1));
                pair_first = false;
                break;
            }
            case K_PAIRROOT: break;
        }
    }
    if (c->pa >= 0)
        QEM_LAUNCH(-1, QEM_PH_ROOT, qemk::pair_root_fwd(c->s, c->d(c->nodes[c->pa].o_ut), c->d(c->nodes[c->pb].o_ut), c->d(c->o_pairM), K,
                                    K, Lall + c->pair_slot));
    if (!(fu && fu->root_fin >= 0))
        QEM_LAUNCH(-1, QEM_PH_ROOT, qemk::sum_L(c->s, Lall, c->nL, c->d(c->o_logphat), c->at<uint32_t>(c->o_status)));
    return QEM_OK;
}

// In the fused iteration the plate backward kernel also writes the node's
// moments, and the root finisher has already written the root's weights.
qem_status contract_bwd_impl(qem_ctx c, const double* g, const Fusion* fu) {
    const int K = c->K;
    const bool f64 = c->f64();
    double* Lall = c->d(c->o_Lall);
    if (c->pa >= 0) {
        const NodeP& A = c->nodes[c->pa];
        const NodeP& B = c->nodes[c->pb];
        QEM_LAUNCH(-1, QEM_PH_ROOT, qemk::pair_root_bwd(c->s, f64, c->d(A.o_ut), c->d(B.o_ut), c->d(c->o_pairM), Lall + c->pair_slot, K, K,
                                    c->d(c->o_pairW), c->at(A.o_w), c->at(B.o_w), g));
    }
    for (int v = 0; v < static_cast<int>(c->nodes.size()); ++v) {
        const NodeP& p = c->nodes[v];
        switch (p.kind) {
            case K_ROOT:
                if (fu && v == fu->root_fin) break;
                QEM_LAUNCH(v, QEM_PH_ROOT, qemk::root_w(c->s, f64, c->d(p.o_ut), Lall + p.Lslot, c->at(p.o_w), p.d.n, K, g));
                break;
            case K_CHAIN: {
                const long T = p.d.chain_len;
                if (c->bexp()) {
                    QEM_LAUNCH(v, QEM_PH_CHAIN_BWD, qemk::chain_bwd_pn(c->s, false, c->at(p.o_z), c->d(p.o_ut),
                                                                      c->d(p.o_msg), Lall + p.Lslot, c->at(p.o_w),
                                                                      p.d.n / T, static_cast<int>(T), K, p.d.a, p.d.b,
                                                                      p.d.var, g, qemk::VSeries{}, true));
                    break;
                }
                if (!p.has_F) {
                    QEM_LAUNCH(v, QEM_PH_CHAIN_BWD, qemk::chain_bwd_pn(c->s, f64, c->at(p.o_z), c->d(p.o_ut), c->d(p.o_msg),
                                                                      Lall + p.Lslot, c->at(p.o_w), p.d.n / T,
                                                                      static_cast<int>(T), K, p.d.a, p.d.b, p.d.var, g));
                    break;
                }
                QEM_LAUNCH(v, QEM_PH_CHAIN_BWD, qemk::chain_bwd(c->s, f64, c->at(p.o_F), c->d(p.o_ut), c->at(p.o_msg), Lall + p.Lslot,
                                        c->at(p.o_w), p.d.n / T, static_cast<int>(T), K, g));
                break;
            }
            case K_CHAINP: {
                const long T = p.d.chain_len, G = p.d.n / T;
                if (qemk::chainp_mfma_supported(K)) {
                    const NodeP& par = c->nodes[p.fp[0]];
                    QEM_LAUNCH(v, QEM_PH_CHAIN_BWD,
                               qemk::chainp_bwd_mfma(c->s, f64, c->at(p.o_z), c->d(p.o_ut), c->at(par.o_z),
                                                     c->at(par.o_w), c->at<int32_t>(p.o_sp), c->d(p.o_msg),
                                                     c->d(p.o_vL), c->d(p.o_vw), G, static_cast<int>(T), K, p.d.a,
                                                     p.d.b, p.d.var, p.d.init_b, p.d.init_var));
                    QEM_LAUNCH(v, QEM_PH_CHAIN_BWD, qemk::chainp_wsum(c->s, f64, true, c->at(p.o_vw), c->at(p.o_w), G,
                                                                     qemk::chainp_mfma_blocks(K), static_cast<int>(T), K));
                    break;
                }
                QEM_LAUNCH(v, QEM_PH_CHAIN_BWD, qemk::chain_bwd_pn(c->s, f64, c->at(p.o_z), c->d(p.o_vut), c->d(p.o_msg),
                                                                  c->d(p.o_vL), c->at(p.o_vw), G, static_cast<int>(T),
                                                                  K, p.d.a, p.d.b, p.d.var, nullptr, vseries(c, p)));
                QEM_LAUNCH(v, QEM_PH_CHAIN_BWD, qemk::chainp_wsum(c->s, f64, false, c->at(p.o_vw), c->at(p.o_w), G, K,
                                                                 static_cast<int>(T), K));
                break;
            }
            case K_SINGLE: {
                const NodeP& par = c->nodes[p.fp[0]];
                if (!p.has_F) {
                    QEM_LAUNCH(v, QEM_PH_PLATE_BWD,
                               qemk::plate_bwd_pn(c->s, f64, c->at(p.o_z), c->at(par.o_z),
                                                  p.has_pidx ? c->at<int32_t>(p.o_pidx) : nullptr, c->d(p.o_ut),
                                                  c->d(p.o_msg), c->at(par.o_w), c->at(p.o_w), p.d.n, K, K, p.d.dim,
                                                  p.d.a, p.d.b, p.d.var,
                                                  moments_fused(p, v, fu) ? c->d(p.o_mone) : nullptr));
                    break;
                }
                const bool use_idx = p.has_pidx && p.d.parent0 == p.fp[0];
                QEM_LAUNCH(v, QEM_PH_PLATE_BWD, qemk::plate_bwd(c->s, f64, c->at(p.o_F), c->d(p.o_ut), c->at(p.o_msg), c->at(par.o_w),
                                        use_idx ? c->at<int32_t>(p.o_pidx) : nullptr, c->at(p.o_w), p.d.n, K, K,
                                        moments_fused(p, v, fu) ? c->at(p.o_z) : nullptr,
                                        moments_fused(p, v, fu) ? c->d(p.o_mone) : nullptr, p.d.dim));
                break;
            }
            case K_PAIRCHILD: {
                const qemk::TwoParentArgs a = tp_args(c, p);
                QEM_LAUNCH(v, QEM_PH_TP_BWD, qemk::twoparent_bwd(c->s, f64, a, c->d(c->o_pairW), c->at(p.o_w)));
                break;
            }
            case K_PAIRROOT: break;
        }
    }
    return QEM_OK;
}

// Nodes whose moments the fused iteration writes in another kernel.

qem_status moments_impl(qem_ctx c, const Fusion* fu) {
    for (int v = 0; v < static_cast<int>(c->nodes.size()); ++v) {
        const NodeP& p = c->nodes[v];
        if (moments_fused(p, v, fu)) continue;
        QEM_LAUNCH(v, QEM_PH_MOMENTS, qemk::moments(c->s, c->f64(), c->at(p.o_z), c->at(p.o_w), c->d(p.o_mone), p.d.n, c->K,
                                                    p.d.dim, uses_log_moments(p.d.qfamily)));
    }
    return QEM_OK;
}

}  // namespace

qem_status qem_contract_fwd(qem_ctx c) {
    if (qem_status st = need_ws(c)) return st;
    return contract_fwd_impl(c, nullptr);
}

qem_status qem_contract_bwd(qem_ctx c, const double* g) {
    if (qem_status st = need_ws(c)) return st;
    return contract_bwd_impl(c, g, nullptr);
}

qem_status qem_moments(qem_ctx c) {
    if (qem_status st = need_ws(c)) return st;
    return moments_impl(c, nullptr);
}

qem_status qem_ess(qem_ctx c, int32_t node, double* ess, double* mean) {
    if (qem_status st = need_ws(c)) return st;
    if (node < 0 || node >= static_cast<int>(c->nodes.size())) return fail(c, QEM_E_INVALID, "bad node id");
    if (!ess) return fail(c, QEM_E_INVALID, "ess must be a device buffer of n doubles");
    const NodeP& p = c->nodes[node];
    QEM_LAUNCH(node, QEM_PH_MOMENTS, qemk::ess(c->s, c->f64(), c->at(p.o_w), p.d.n, c->K, ess, mean));
    return QEM_OK;
}

qem_status qem_mstep(qem_ctx c, double lam) {
    if (qem_status st = need_ws(c)) return st;
    if (!(lam >= 0.0 && lam <= 1.0)) return fail(c, QEM_E_INVALID, "lam must be in [0, 1]");
    for (int v = 0; v < static_cast<int>(c->nodes.size()); ++v) {
        const NodeP& p = c->nodes[v];
        QEM_LAUNCH(v, QEM_PH_MSTEP, qemk::mstep(c->s, c->d(p.o_mema), c->d(p.o_mone), c->d(p.o_qp), static_cast<long>(p.d.n) * p.d.dim,
                            p.d.qfamily, lam, c->at<uint32_t>(c->o_status), p.d.dim));
    }
    return QEM_OK;
}

namespace {
// One iteration of Algorithm 1 with the stages fused where they meet:
//  - sampling and the unary factor in one kernel per node, which also writes
//    ut of nodes without children (the first one clears the status word);
//    an FP32 K = 64 leaf plate with Gaussian proposals draws its samples in
//    its own plate forward kernel instead (sample_in_plate_fwd);
//  - the linear-Gaussian pair tables inside the plate forward kernel (F is
//    still written, for the backward pass);
//  - a single-instance root node (listed first, no joint root pair) finished
//    by one kernel: gather, LSE, the log P_MP sum, weights, moments, M-step;
//  - the plate nodes' moments inside the plate backward kernel;
//  - one M-step launch for the remaining nodes.
// Each kernel does the same arithmetic as its standalone counterpart.  With
// iter_dev the iteration number is read from the device counter, which the
// root finisher or the last M-step launch advances.  The EMA weight of the
// iteration (lam, or t^-p with qem_set_ema) is written by the first sampling
// kernel; with the second-sample normaliser a second forward pass on an
// independent sample follows the moments and the M-step scales them by
// P_MP(z) / P_MP(z_new).
qem_status step_pipeline(qem_ctx c, uint64_t seed, uint64_t iter, uint64_t* iter_dev, double lam) {
    const int nv = static_cast<int>(c->nodes.size());
    const bool second = c->second_sample;
    double* lam_dev = c->d(c->o_lamt);
    Fusion fu;
    fu.lam = lam;
    fu.lam_dev = lam_dev;
    fu.iter_dev = iter_dev;
    fu.root_mstep = !second;   // with the second sample every M-step waits for its log P_MP
    fu.seed = seed;
    fu.iter = static_cast<uint32_t>(iter);
    fu.fwd_sample.assign(nv, 0);
    if (!second)   // the second sample's forward pass has no sampling of its own
        for (int v = 0; v < nv; ++v) fu.fwd_sample[v] = sample_in_plate_fwd(c, c->nodes[v]);
    const NodeP& n0 = c->nodes[0];
    if (n0.kind == K_ROOT && n0.d.n == 1 && c->pa < 0 && n0.d.qfamily != QEM_Q_DIRICHLET &&
        n0.children.size() <= static_cast<size_t>(qemk::MAX_CHILD_LISTS))
        fu.root_fin = 0;
    // consecutive nodes of the same proposal family and dimension share one
    // sampling launch (timed under the group's first node); the pair tables
    // that are not evaluated inside the forward kernels follow the group
    // (the first pass leaves out the nodes whose plate forward draws them)
    auto sample_all = [&](uint32_t it_xor, bool first) -> qem_status {
        for (int v0 = 0; v0 < nv;) {
            if (first && fwd_samples(&fu, v0)) {
                ++v0;
                continue;
            }
            qemk::SampleNode grp[qemk::SAMPLE_NODES];
            int n = 0;
            while (v0 + n < nv && n < qemk::SAMPLE_NODES) {
                if (first && fwd_samples(&fu, v0 + n)) break;
                const NodeP& p = c->nodes[v0 + n];
                const qemk::UnaryArgs a = unary_args(c, p);
                if (n > 0 && !qemk::sample_group_compatible(grp[0].a, a)) break;
                grp[n] = qemk::SampleNode{a, p.children.empty() ? c->d(p.o_ut) : nullptr, static_cast<uint32_t>(v0 + n)};
                ++n;
            }
            const qemk::IterTerms itt{it_xor, first && v0 == 0 ? lam_dev : nullptr, lam, c->ema_p};
            QEM_LAUNCH(v0, QEM_PH_SAMPLE, qemk::sample_unary_multi(c->s, c->f64(), grp, n, seed, static_cast<uint32_t>(iter),
                                                                  iter_dev,
                                                                  first && v0 == 0 ? c->at<uint32_t>(c->o_status) : nullptr,
                                                                  itt));
            for (int v = v0; v < v0 + n; ++v)
                if (!table_in_fwd(c, c->nodes[v]))
                    if (qem_status st = pair_tables(c, v)) return st;
            v0 += n;
        }
        return QEM_OK;
    };
    if (qem_status st = sample_all(0u, true)) return st;
    if (qem_status st = contract_fwd_impl(c, &fu)) return st;
    if (qem_status st = contract_bwd_impl(c, nullptr, &fu)) return st;
    if (qem_status st = moments_impl(c, &fu)) return st;
    if (second) {
        // log P_MP of a second, independent sample of this iteration's Q
        QEM_HIP(qemk::copy_scalar(c->s, c->d(c->o_logphat), c->d(c->o_lp1)));
        if (qem_status st = sample_all(QEM_SECOND_SAMPLE_STREAM, false)) return st;
        Fusion fu2;
        if (qem_status st = contract_fwd_impl(c, &fu2)) return st;
    }
    const bool root_done = fu.root_fin >= 0 && fu.root_mstep;
    std::vector<int> rest;   // nodes whose M-step is not done by the root finisher
    for (int v = 0; v < nv; ++v)
        if (!(root_done && v == fu.root_fin)) rest.push_back(v);
    // the counter still advances once when every node's M-step was fused
    const bool counter_left = iter_dev && !root_done;
    const int nrest = static_cast<int>(rest.size());
    for (int v0 = 0; v0 < nrest || (v0 == 0 && counter_left); v0 += qemk::MSTEP_NODES) {
        qemk::MstepTable tb{};
        tb.n = std::min(qemk::MSTEP_NODES, nrest - v0);
        for (int q = 0; q < tb.n; ++q) {
            const NodeP& p = c->nodes[rest[v0 + q]];
            tb.mema[q] = c->d(p.o_mema);
            tb.mone[q] = c->d(p.o_mone);
            tb.qp[q] = c->d(p.o_qp);
            tb.count[q] = static_cast<long>(p.d.n) * p.d.dim;
            tb.qfamily[q] = p.d.qfamily;
            tb.dim[q] = p.d.dim;
        }
        tb.lam_dev = lam_dev;
        tb.lp_z = second ? c->d(c->o_lp1) : nullptr;
        tb.lp_new = second ? c->d(c->o_logphat) : nullptr;
        const bool last = v0 + qemk::MSTEP_NODES >= nrest;
        QEM_LAUNCH(-1, QEM_PH_MSTEP, qemk::mstep_multi(c->s, tb, lam, c->at<uint32_t>(c->o_status),
                                                      last && counter_left ? iter_dev : nullptr));
    }
    // the reported log P_MP of the iteration is the first sample's
    if (second) QEM_HIP(qemk::copy_scalar(c->s, c->d(c->o_lp1), c->d(c->o_logphat)));
    return QEM_OK;
}
}  // namespace

qem_status qem_set_ema(qem_ctx c, double p, int32_t second_sample) {
    if (!c) return QEM_E_INVALID;
    if (!(p >= 0.0 && p < 1.0)) return fail(c, QEM_E_INVALID, "p must be in [0, 1)");
    if (second_sample != 0 && second_sample != 1) return fail(c, QEM_E_INVALID, "second_sample must be 0 or 1");
    c->ema_p = p;
    c->second_sample = second_sample != 0;
    // the captured iterations no longer match
    drop_graphs(c);
    return QEM_OK;
}

namespace {
// Iterations t0 .. t0 + n - 1 of qem_step / qem_run: the Theorem 1 step t^-p
// needs t >= 1; the iteration is a 32-bit Philox counter word whose top bit
// the second-sample stream flips, so with that option t < 2^31.
qem_status check_iters(qem_ctx c, uint64_t t0, uint64_t n) {
    if (c->ema_p > 0.0 && t0 == 0) return fail(c, QEM_E_INVALID, "the t^-p step size needs iterations t >= 1");
    const uint64_t lim = c->second_sample ? 0x7FFFFFFFull : 0xFFFFFFFFull;
    if (t0 > lim || n - 1 > lim - t0)
        return fail(c, QEM_E_INVALID, c->second_sample ? "iterations must stay below 2^31 with the second sample"
                                                       : "iterations must stay below 2^32");
    return QEM_OK;
}
}  // namespace

qem_status qem_step(qem_ctx c, uint64_t seed, uint64_t iter, double lam) {
    if (!c) return QEM_E_INVALID;
    if (qem_status st = check_iters(c, iter, 1)) return st;
    if (qem_status st = need_ws(c)) return st;
    if (!(lam >= 0.0 && lam <= 1.0)) return fail(c, QEM_E_INVALID, "lam must be in [0, 1]");
    return step_pipeline(c, seed, iter, nullptr, lam);
}

namespace {
// Iterations per graph launch of qem_run beyond the first few: consecutive
// iterations captured in one graph run back to back without a launch gap.
constexpr int RUN_UNROLL = 8;

// Capture `iters` iterations of the step pipeline (the iteration number is
// read from the device counter, which each iteration advances).
qem_status capture_iters(qem_ctx c, uint64_t seed, double lam, int iters, hipGraph_t* graph, hipGraphExec_t* exec) {
    if (!c->cap) QEM_HIP(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipStream_t saved = c->s;
    const bool timing = c->timing;
    c->s = c->cap;
    c->timing = false;
    qem_status st = QEM_OK;
    hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int k = 0; k < iters && st == QEM_OK; ++k)
            st = step_pipeline(c, seed, 0, c->at<uint64_t>(c->o_iter), lam);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->cap, &g);
        *graph = g;
    }
    c->s = saved;
    c->timing = timing;
    if (st != QEM_OK) return st;
    QEM_HIP(e);
    QEM_HIP(hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0));
    return QEM_OK;
}

qem_status capture(qem_ctx c, uint64_t seed, double lam) {
    drop_graphs(c);
    if (qem_status st = capture_iters(c, seed, lam, 1, &c->graph, &c->gexec)) return st;
    if (qem_status st = capture_iters(c, seed, lam, RUN_UNROLL, &c->graph_u, &c->gexec_u)) return st;
    c->g_seed = seed;
    c->g_lam = lam;
    return QEM_OK;
}
}  // namespace

qem_status qem_run(qem_ctx c, uint64_t seed, uint64_t iter0, double lam, int32_t n_iter) {
    if (!c) return QEM_E_INVALID;
    if (n_iter < 0) return fail(c, QEM_E_INVALID, "n_iter must be >= 0");
    if (n_iter > 0)
        if (qem_status st = check_iters(c, iter0, static_cast<uint64_t>(n_iter))) return st;
    if (qem_status st = need_ws(c)) return st;
    if (!(lam >= 0.0 && lam <= 1.0)) return fail(c, QEM_E_INVALID, "lam must be in [0, 1]");
    if (n_iter == 0) return QEM_OK;
    if (!c->gexec || c->g_seed != seed || c->g_lam != lam)
        if (qem_status st = capture(c, seed, lam)) return st;
    QEM_HIP(qemk::iter_set(c->s, c->at<uint64_t>(c->o_iter), iter0));
    int32_t t = 0;
    for (; t + RUN_UNROLL <= n_iter; t += RUN_UNROLL) QEM_HIP(hipGraphLaunch(c->gexec_u, c->s));
    for (; t < n_iter; ++t) QEM_HIP(hipGraphLaunch(c->gexec, c->s));
    return QEM_OK;
}

qem_status qem_read_status(qem_ctx c, uint32_t* flags, uint32_t* floor_hits, double* logphat) {
    if (qem_status st = need_ws(c)) return st;
    uint32_t sw[4];
    double lp;
    QEM_HIP(hipMemcpyAsync(sw, c->ws + c->o_status, sizeof(sw), hipMemcpyDeviceToHost, c->s));
    QEM_HIP(hipMemcpyAsync(&lp, c->ws + c->o_logphat, sizeof(lp), hipMemcpyDeviceToHost, c->s));
    QEM_HIP(hipStreamSynchronize(c->s));
    if (flags) *flags = sw[0];
    if (floor_hits) *floor_hits = sw[1];
    if (logphat) *logphat = lp;
    static_assert(QEM_FLAG_NEG_INF_ROW == qemk::FLAG_NEG_INF_ROW, "header and kernels agree on the flag");
    return (sw[0] & QEM_FLAG_NONFINITE_LOGPHAT) ? QEM_E_NONFINITE : QEM_OK;
}

// ---- stream-bandwidth calibration -------------------------------------------

qem_status qem_stream_probe(void* buf, size_t bytes, int32_t mode, float* sink, void* stream) {
    if (!buf || mode < 0 || mode > 3 || (mode >= 2 && !sink)) {
        g_create_err = "qem_stream_probe: null buffer or sink, or mode outside 0..3";
        return QEM_E_INVALID;
    }
    if (bytes == 0 || bytes % 16384 != 0 || bytes / 16384 > 0x7fffffffu) {
        g_create_err = "qem_stream_probe: bytes must be a positive multiple of 16384";
        return QEM_E_SHAPE;
    }
    const hipError_t e = qemk::stream_probe(static_cast<hipStream_t>(stream), buf, bytes, mode, sink);
    if (e != hipSuccess) {
        g_create_err = std::string("qem_stream_probe: ") + hipGetErrorString(e);
        return QEM_E_DEVICE;
    }
    return QEM_OK;
}

// ---- encoder ----------------------------------------------------------------

#define QEM_ENC_HIP(expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            g_create_err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
            return QEM_E_DEVICE;                                                             \
        }                                                                                    \
    } while (0)

static qem_status enc_fail(qem_status st, const char* msg) {
    g_create_err = msg;
    return st;
}

qem_status qem_enc_features(const double* y, const double* cov, int32_t n, int32_t n_per, int32_t n_cov, float* feat,
                            void* stream) {
    if (!y || !cov || !feat) return enc_fail(QEM_E_INVALID, "null pointer");
    if (n < 1 || n_per < 1 || 2 + 2 * n_cov != QEM_ENC_IN) return enc_fail(QEM_E_SHAPE, "features need n_cov == 8");
    QEM_ENC_HIP(qemk::enc_features(static_cast<hipStream_t>(stream), y, cov, n, n_per, n_cov, feat));
    return QEM_OK;
}

qem_status qem_enc_pool(const float* feat, int32_t n, int32_t n_per, float* rows, void* stream) {
    if (n < 1 || n_per < 1) return enc_fail(QEM_E_SHAPE, "n and n_per must be >= 1");
    if (!feat || !rows) return enc_fail(QEM_E_INVALID, "null pointer");
    QEM_ENC_HIP(qemk::enc_pool(static_cast<hipStream_t>(stream), feat, n, n_per, rows));
    return QEM_OK;
}

qem_status qem_enc_features_ctx(const float* feat, const float* rows, int32_t n, int32_t n_per, float* out,
                                void* stream) {
    if (n < 1 || n_per < 1) return enc_fail(QEM_E_SHAPE, "n and n_per must be >= 1");
    if (!feat || !rows || !out) return enc_fail(QEM_E_INVALID, "null pointer");
    QEM_ENC_HIP(qemk::enc_features_ctx(static_cast<hipStream_t>(stream), feat, rows, n, n_per, out));
    return QEM_OK;
}

qem_status qem_enc_fwd(const uint16_t* w, const float* feat, int32_t n, float* out, float* act, void* stream) {
    if (!w || !feat || !out) return enc_fail(QEM_E_INVALID, "null pointer");
    if (n < 1) return enc_fail(QEM_E_SHAPE, "n must be >= 1");
    QEM_ENC_HIP(qemk::enc_fwd(static_cast<hipStream_t>(stream), w, feat, n, out, act));
    return QEM_OK;
}

qem_status qem_enc_loss(const float* out, const double* target, int32_t n, float* dout, double* kl, double* loss,
                        void* stream) {
    if (!out || !target || !dout || !kl) return enc_fail(QEM_E_INVALID, "null pointer");
    if (n < 1) return enc_fail(QEM_E_SHAPE, "n must be >= 1");
    QEM_ENC_HIP(qemk::enc_kl(static_cast<hipStream_t>(stream), out, target, n, dout, kl, loss));
    return QEM_OK;
}

size_t qem_enc_scratch_bytes(int32_t n) { return n < 1 ? 0 : qemk::enc_scratch_bytes(n); }

qem_status qem_enc_bwd(const uint16_t* w, const float* feat, const float* act, const float* dout, int32_t n, float* grad,
                       void* scratch, void* stream) {
    if (!w || !feat || !act || !dout || !grad || !scratch) return enc_fail(QEM_E_INVALID, "null pointer");
    if (n < 1) return enc_fail(QEM_E_SHAPE, "n must be >= 1");
    QEM_ENC_HIP(qemk::enc_bwd(static_cast<hipStream_t>(stream), w, feat, act, dout, n, grad,
                              static_cast<float*>(scratch)));
    return QEM_OK;
}

qem_status qem_enc_bwd_noalloc(const uint16_t* w, const float* feat, const float* act, const float* dout, int32_t n,
                               float* grad, void* stream) {
    if (!w || !feat || !act || !dout || !grad) return enc_fail(QEM_E_INVALID, "null pointer");
    if (n < 1 || n > QEM_ENC_NOALLOC_MAX_N)
        return enc_fail(QEM_E_SHAPE, "n must be in [1, QEM_ENC_NOALLOC_MAX_N]: the library's scratch holds the "
                                     "partial gradients of at most 16384 groups");
    static_assert(QEM_ENC_NOALLOC_MAX_N == qemk::ENC_NOALLOC_MAX_N, "header and library agree on the scratch size");
    const hipError_t e = qemk::enc_bwd_noalloc(static_cast<hipStream_t>(stream), w, feat, act, dout, n, grad);
    if (e == hipErrorInvalidDevice)
        return enc_fail(QEM_E_INVALID, "the stream must belong to the current device");
    QEM_ENC_HIP(e);
    return QEM_OK;
}

qem_status qem_enc_adam(float* master, uint16_t* w, const float* grad, float* m1, float* m2, int32_t step, float lr,
                        float beta1, float beta2, float eps, void* stream) {
    if (!master || !w || !grad || !m1 || !m2) return enc_fail(QEM_E_INVALID, "null pointer");
    if (step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return enc_fail(QEM_E_INVALID, "bad Adam hyper-parameters");
    QEM_ENC_HIP(qemk::enc_adam(static_cast<hipStream_t>(stream), master, w, grad, m1, m2, step, lr, beta1, beta2, eps));
    return QEM_OK;
}

qem_status qem_enc_to_bf16(const float* master, uint16_t* w, void* stream) {
    if (!master || !w) return enc_fail(QEM_E_INVALID, "null pointer");
    QEM_ENC_HIP(qemk::enc_to_bf16(static_cast<hipStream_t>(stream), master, w));
    return QEM_OK;
}

qem_status qem_enc_targets(const double* mema, int32_t n, double var_floor, const float* rows, double* target,
                           void* stream) {
    if (!mema || !target) return enc_fail(QEM_E_INVALID, "null pointer");
    if (n < 1) return enc_fail(QEM_E_SHAPE, "n must be >= 1");
    if (!(var_floor >= 0.0)) return enc_fail(QEM_E_INVALID, "var_floor must be >= 0");
    QEM_ENC_HIP(qemk::enc_targets(static_cast<hipStream_t>(stream), mema, n, var_floor, rows, target));
    return QEM_OK;
}

qem_status qem_enc_apply(const float* out, int32_t n, double* qparam, void* stream) {
    if (!out || !qparam) return enc_fail(QEM_E_INVALID, "null pointer");
    if (n < 1) return enc_fail(QEM_E_SHAPE, "n must be >= 1");
    QEM_ENC_HIP(qemk::enc_apply(static_cast<hipStream_t>(stream), out, n, qparam));
    return QEM_OK;
}

qem_status qem_enc_apply_residual(const float* out, const float* rows, int32_t n, double* qparam, void* stream) {
    if (n < 1) return enc_fail(QEM_E_SHAPE, "n must be >= 1");
    if (!out || !rows || !qparam) return enc_fail(QEM_E_INVALID, "null pointer");
    QEM_ENC_HIP(qemk::enc_apply_res(static_cast<hipStream_t>(stream), out, rows, n, qparam));
    return QEM_OK;
}

}  // extern "C"
