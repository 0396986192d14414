// Kernel launchers of the QEM library (internal to the shared object).
// Every launcher enqueues on `s` and returns the launch status.  `f64`
// selects FP64 tensors (else FP32).  Shapes are validated by the caller
// (qem_api.cpp) before any launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <cmath>

namespace qemk {

// largest sample dimension of a latent node
constexpr int MAX_DIM = 32;

// ---- sampling -------------------------------------------------------------
// z[i,k,j] = mean[i,j] + sqrt(var[i,j]) * N(e), e = (i*K + k)*d + j.
// iter_dev (optional): read the iteration number from device memory instead.
hipError_t sample_gauss(hipStream_t s, bool f64, void* z, const double* qp, int n, int K, int d,
                        uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev);
// z[i,k] = Gamma(shape_i, 1) / rate_i by Marsaglia-Tsang.
hipError_t sample_gamma(hipStream_t s, bool f64, void* z, const double* qp, int n, int K,
                        uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev);
// z[i,k] = 1 if the uniform of counter (i*K + k, 0) is at most p_i, else 0
hipError_t sample_bernoulli(hipStream_t s, bool f64, void* z, const double* qp, int n, int K,
                            uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev);
// Dirichlet proposals, d = C components: sample (i, k) normalises the
// Gamma(alpha_c, 1) draws of its elements (i*K + k)*C + c in log space.
hipError_t sample_dirichlet(hipStream_t s, bool f64, void* z, const double* qp, int n, int K, int C,
                            uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev);
// Categorical proposals, one-hot over C categories: sample e takes the first
// c with u * P_{C-1} <= P_c (P the running sums of p, u the (0, 1] uniform of
// counter (e, 0)).
hipError_t sample_categorical(hipStream_t s, bool f64, void* z, const double* qp, int n, int K, int C,
                              uint64_t seed, uint32_t iter, uint32_t node, const uint64_t* iter_dev);

struct UnaryArgs;
// Per-iteration terms of the fused sampling kernel: the Philox iteration word
// is XOR-ed with it_xor (a second, independent sample of the same iteration),
// and, when lam_out is set, thread 0 writes the EMA weight of this iteration
// t there: t^-p for p > 0, else lam.
struct IterTerms {
    uint32_t it_xor;
    double* lam_out;
    double lam;
    double p;
};
// Sampling fused with the unary log-factor (see k_sample_unary); ut and status optional.
hipError_t sample_unary(hipStream_t s, bool f64, const UnaryArgs& a, uint64_t seed, uint32_t iter, uint32_t node,
                        const uint64_t* iter_dev, double* ut, uint32_t* status, const IterTerms& itt);

// ---- observation statistics (once per context) ----------------------------
// xbar[i,j] = mean_o x[i,o,j]; ss[i,j] = sum_o (x[i,o,j] - xbar[i,j])^2
hipError_t stats_gauss(hipStream_t s, const double* x, int n, int J, int d, double* xbar, double* ss);
// sy[i] = sum_o y[i,o]; slg[i] = sum_o lgamma(y[i,o] + 1)
hipError_t stats_poisson(hipStream_t s, const double* y, int n, int J, double* sy, double* slg);
// cnt[i, c] = the number of y[i, :] equal to c, c < C (other values are not counted)
hipError_t stats_categorical(hipStream_t s, const double* y, int n, int J, int C, double* cnt);
// lik[i, c] = sum_j log N(y[i, j]; mu[c], var)
hipError_t stats_gauss_mixture(hipStream_t s, const double* y, const double* mu, int n, int J, int C, double var,
                               double* lik);
// F[i, kp, k] = log pi^kp[c(z_i^k)]: a one-hot child under a Dirichlet parent
// (samples pi [n_parent, Kp, C]), c the child's category.
hipError_t pair_categorical(hipStream_t s, bool f64, void* F, const void* zc, const void* zp, const int32_t* pidx,
                            long n, int K, int Kp, int C);
// syx[i,:] = sum_o y[i,o] cov[i,o,:]; sy[i] = sum_o y[i,o]
hipError_t stats_bernoulli(hipStream_t s, const double* y, const double* cov, int n, int J, int D,
                           double* syx, double* sy);

// ---- log-factors ----------------------------------------------------------
// Constants of the linear-Gaussian pair factor of a d-dimensional latent
// (host side; every kernel that evaluates the factor receives these).
inline void normal_pair_consts(int d, double var, double* c0, double* hp) {
    *c0 = -0.5 * d * (1.8378770664093454835606594728112 + std::log(var));   // log(2 pi)
    *hp = 0.5 / var;
}

enum PriorTerm { PT_NONE = 0, PT_NORMAL = 1, PT_GAMMA = 2, PT_CHAIN_START = 3, PT_BERN = 4, PT_DIR = 5, PT_CAT = 6 };
// proposal families (the ABI's qem_qfamily values)
constexpr int QF_GAUSS = 0, QF_GAMMA = 1, QF_GAMMA_EF = 2, QF_BERNOULLI = 3, QF_DIRICHLET = 4, QF_CATEGORICAL = 5;
constexpr double BERN_FLOOR = 1e-9;   // the Bernoulli M-step keeps p in [floor, 1 - floor]
// The Dirichlet M-step moves mean parameters with 1 - sum_c exp(E log z_c)
// below this gap back to it before solving.
constexpr double DIR_GAP_FLOOR = 1e-12;

// Terms that do not depend on the sample are formed on the host once
// (unary_consts): -log K, the prior's normaliser and the Gaussian
// observations' normaliser and 1/(2 var).
struct UnaryArgs {
    const void* z; void* u; const double* qp;
    int n, K, d, qfamily;
    int prior_term; double pb, pvar, pshape, prate; int chain_T;
    const double* g_xbar; const double* g_ss; int g_J; double g_var;   // Gaussian obs or null
    const double* p_sy; const double* p_slg; int p_J;                  // Poisson obs or null
    const double* c_cnt;                                               // categorical counts [n, d] or null
    const double* m_lik;                                               // mixture log-likelihood [n, d] or null
    const double* d_sy; int d_R; double d_l1, d_l0;                    // detection obs or null:
                                                                       // sum_r y, visits, log p, log(1 - p)
    double neg_log_K;   // -log K
    double prior_c0;    // Normal: -1/2 log(2 pi var); Gamma: shape log rate - lgamma(shape);
                        // Bernoulli: log sigmoid(b)
    double prior_hp;    // Normal: 1 / (2 var); Bernoulli: log sigmoid(-b)
    double g_c0;        // -J/2 log(2 pi var_obs)
    double g_hp;        // 1 / (2 var_obs)
};
void unary_consts(UnaryArgs& a);

// The Philox word of a sampling launch: iteration, node and the two key
// words of the seed.
struct Stream { uint32_t it, node, k0, k1; };
Stream make_stream(uint64_t seed, uint32_t iter, uint32_t node);

// A plate node whose samples and unary factor the FP32 K = 64 plate forward
// kernel draws itself (its wave per instance takes the place of the sampling
// launch's): the node's unary arguments, its Philox word, the device
// iteration counter (when set, it replaces st.it) and the word XOR-ed into
// the iteration.
struct FwdSample {
    UnaryArgs a;
    Stream st;
    const uint64_t* it_dev;
    uint32_t it_xor;
};

// Several nodes sampled by one launch of the fused sample-and-factor kernel
// (same proposal family and, for Gaussian proposals, the same dimension when
// it is 1, 2, 4 or 8); the samples are those of one launch per node.
constexpr int SAMPLE_NODES = 4;
struct SampleNode {
    UnaryArgs a;
    double* ut;      // ut = u written here when set (nodes without children)
    uint32_t node;   // the node's Philox word
};
bool sample_group_compatible(const UnaryArgs& x, const UnaryArgs& y);
hipError_t sample_unary_multi(hipStream_t s, bool f64, const SampleNode* nodes, int n, uint64_t seed, uint32_t iter,
                              const uint64_t* iter_dev, uint32_t* status, const IterTerms& itt);
hipError_t unary(hipStream_t s, bool f64, const UnaryArgs& a);

// F[r,kp,k] = sum_j log N(zc[c(r),k,j]; a*zp[p(r),kp,j] + b, var).
// Tree (chain_T == 0): c(r) = r, p(r) = pidx ? pidx[r] : 0.
// Chain (chain_T > 1): r over series*(T-1), g = r/(T-1), t = r%(T-1)+1,
//   c(r) = g*T + t, p(r) = g*T + t - 1 (zp == zc).
hipError_t pair_normal(hipStream_t s, bool f64, void* F, const void* zc, const void* zp,
                       const int32_t* pidx, long R, int K, int Kp, int d,
                       double a, double b, double var, int chain_T);
// F[i,kp,k] = log N(zc[i,k]; 0, exp(2 zp[0,kp]))   (scalar nodes, root parent)
hipError_t pair_logscale(hipStream_t s, bool f64, void* F, const void* zc, const void* zp,
                         long n, int K, int Kp);
// F[i,kp,k] = z_k eta - softplus(eta), eta = a zp[p(i),kp] + b (Bernoulli-logit prior of a
// discrete child; p(i) = pidx ? pidx[i] : 0), in the tensor type's arithmetic
hipError_t pair_bern_prior(hipStream_t s, bool f64, void* F, const void* zc, const void* zp, const int32_t* pidx,
                           long n, int K, int Kp, double a, double b);
// F[i,kb,k] = sum_o [y_io eta - softplus(eta)], eta = cov[i,o,:] . beta[kb,:] + zc[i,k]
hipError_t pair_bernoulli(hipStream_t s, bool f64, void* F, const void* zc, const void* zbeta,
                          const double* y, const double* cov, const double* syx, const double* sy,
                          long n, int K, int Kb, int J, int D);

// ---- contraction ----------------------------------------------------------
// Child-message lists of a parent node (one CSR list per child node).
constexpr int MAX_CHILD_LISTS = 4;
// per[c] > 0: list c holds per[c] children of every parent instance, in
// index order (idx[j] = j, off[q] = q per[c]); the kernels then read neither.
struct ChildLists {
    int n;
    const double* mc[MAX_CHILD_LISTS];
    const int32_t* off[MAX_CHILD_LISTS];
    const int32_t* idx[MAX_CHILD_LISTS];
    int32_t per[MAX_CHILD_LISTS];
};
// M-step arguments of a node that the root finisher updates in place.
struct MstepArgs {
    double* mema;
    double* qp;
    int qfamily;
    double lam;
    uint32_t* status;
    const double* lam_dev;   // when set, the EMA weight is read here instead of lam
};
// ut[q,:] = (u ? u : ut)[q,:] + the messages of the listed children of q, for
// every parent instance q (FP64, fixed order).
hipError_t gather(hipStream_t s, bool f64, double* ut, const void* u, const ChildLists& cl, int n_par, int K);

// part[(c * S + p) * K + k] = the sum over subset p (positions p, p + S, ... of
// parent q's children in list c, S = 1024 / K) of the child messages, as the
// child gather forms it; one workgroup per (list, subset).
hipError_t gather_subsets(hipStream_t s, const ChildLists& cl, long q, int K, double* part);
// ut[0,:] = u[0,:] + the subset sums gather_subsets wrote for nl child lists of
// parent instance 0 (the bits of gather() for that instance).
hipError_t gather_finish(hipStream_t s, bool f64, double* ut, const void* u, int nl, int K, const double* part);

// The root level of a single-instance root node in one launch (see k_root_fin).
// part (optional): the root's subset sums from gather_subsets, which replace
// the gather inside the kernel (same additions, same order).
struct RootFinArgs {
    const void* u; double* ut; ChildLists cl; int K; int d; bool logz;   // logz: moments of (z, log z)
    const double* part;
    double* L; const double* Lall; long nL; double* logphat; uint32_t* status;
    void* w; const double* g; const void* z; double* mone;
    MstepArgs ms; uint64_t* iter_dev;
};
hipError_t root_fin(hipStream_t s, bool f64, const RootFinArgs& a);

// Messages m (plate, chain and two-parent) are FP64 in every precision mode.
// m[i,kp] = LSE_k (F[i,kp,k] + ut[i,k])
// status (optional): QEM_FLAG_NEG_INF_ROW is set when a row's log-sum-exp is -inf.
hipError_t plate_fwd(hipStream_t s, bool f64, const void* F, const double* ut, void* m,
                     long n, int Kp, int K, uint32_t* status = nullptr);
// Plate forward of a linear-Gaussian plate node with the pair table evaluated
// in place: writes F (as pair_normal; not kept when F is null) and m (as
// plate_fwd), same bits.  Only for the shapes plate_fwd_pn_supported accepts.
bool plate_fwd_pn_supported(bool f64, int K, int Kp, int d);
// With cl set (u: the node's unary factors, K <= 512) the kernel first forms
// ut = u + child messages itself, the bits of gather(), and writes it out.
// With fs (FP32, K = Kp = 64, d <= 4, no child lists) the kernel first draws
// the node's samples and unary factor (the bits of the sampling kernel) and
// writes z, u and ut = u itself.
hipError_t plate_fwd_pn(hipStream_t s, bool f64, void* F, const void* zc, const void* zp, const int32_t* pidx,
                        double* ut, void* m, long n, int Kp, int K, int d, double a, double b, double var,
                        const void* u = nullptr, const ChildLists* cl = nullptr, uint32_t* status = nullptr,
                        const FwdSample* fs = nullptr);
// Whether plate_fwd_pn can draw the node's samples (fs) at this shape.
bool plate_fwd_samples_supported(bool f64, int K, int Kp, int d);
// w[i,k] = sum_kp wp[p(i),kp] exp(F[i,kp,k] + ut[i,k] - m[i,kp])
// With z and mone non-null the same kernel also writes the instance's moments
// mone[i,j,:] = sum_k w (z, z^2) (FP64, fixed order).
hipError_t plate_bwd(hipStream_t s, bool f64, const void* F, const double* ut, const void* m,
                     const void* wp, const int32_t* pidx, void* w, long n, int Kp, int K,
                     const void* z = nullptr, double* mone = nullptr, int d = 0);
// L[i] = LSE_k ut[i,k]
hipError_t root_lse(hipStream_t s, const double* ut, double* L, long n, int K);
// w[i,k] = g * exp(ut[i,k] - L[i]),  g = dlogphat ? *dlogphat : 1
hipError_t root_w(hipStream_t s, bool f64, const double* ut, const double* L, void* w, long n, int K,
                  const double* dlogphat);
// logphat = sum_i L[i] in a fixed order; sets the non-finite flag.
hipError_t sum_L(hipStream_t s, const double* L, long nL, double* logphat, uint32_t* status);

// chains: one workgroup per series
// A chain whose series hang under a sampled scalar parent beta (one parent
// instance per series): each series is eliminated once per parent sample kb,
// as the virtual series vs = g * Kb + kb, with the step mean
// a x_{t-1} + (1 - a) beta^kb + b and the start term
// log N(x_0; beta^kb + ib, var0) = ic0 - ihp (x_0 - beta^kb - ib)^2.
// Kb = 0 marks an ordinary chain (every other field unused).
struct VSeries {
    int Kb;
    const int32_t* sp;     // parent instance of each series [G]
    const void* zb;        // parent samples [n_parent, Kb], element type of the path
    const void* wb;        // parent weights [n_parent, Kb] (reverse pass)
    const double* usrc;    // unary terms of the series [G, T, K] (forward pass)
    double a, b;
    double ib, ic0, ihp;
};
// Chain forward with the step factor evaluated in place (see k_chain_fwd_pn):
// writes F (as pair_normal with chain_T = T; not kept when F is null) and the
// messages (as chain_fwd).  With vs.Kb > 0 the launch covers G * Kb virtual
// series: ut, m [G * Kb, T, K] and L [G * Kb] are theirs, ut is written from
// vs.usrc plus the start term, and z stays [G, T, K].
hipError_t chain_fwd_pn(hipStream_t s, bool f64, void* F, const void* z, double* ut, void* m, double* L, long G,
                        int T, int K, double a, double b, double var, const VSeries& vs = VSeries{});
// w[g, t, k] = sum over q < np (in order, FP64) of vw[g, q, t, k]: the
// virtual series' weights (np = Kb, the path's element type) or per-block
// partial sums (parts_f64: FP64 parts).
hipError_t chainp_wsum(hipStream_t s, bool f64, bool parts_f64, const void* vw, void* w, long G, int np, int T,
                       int K);
// Chains under a sampled parent as FP64 exponential GEMMs on MFMA (see
// k_chainp_mfma.hip), K in {16, 32, 64, 128}: the forward writes the messages
// m [G * K, T, K] (rows t >= 1) and the messages into the parent L [G * K];
// the reverse writes, per series and block of chainp_mfma_blocks(K) parts,
// the sum of the block's weights part [G, parts, T, K] (FP64).
bool chainp_mfma_supported(int K);
int chainp_mfma_blocks(int K);
hipError_t chainp_fwd_mfma(hipStream_t s, bool f64, const void* z, const double* usrc, const void* zb,
                           const int32_t* sp, double* m, double* L, long G, int T, int K, double a, double b,
                           double var, double ib, double var0);
hipError_t chainp_bwd_mfma(hipStream_t s, bool f64, const void* z, const double* usrc, const void* zb, const void* wb,
                           const int32_t* sp, const double* m, const double* L, double* part, long G, int T, int K,
                           double a, double b, double var, double ib, double var0);
// Reverse passes with the linear-Gaussian factor recomputed from the samples
// instead of read (the factor table is not kept); same bits as chain_bwd /
// plate_bwd over the table the forward kernels write.  mone (optional): the
// plate node's moments, as plate_bwd writes them.
// With vs.Kb > 0: G * Kb virtual series, each scaled by its parent weight
// vs.wb[sp[g] * Kb + kb] (g unused); w [G * Kb, T, K].
// renorm: each step's weights are rescaled to sum to the series' scale (the
// reverse pass over messages of the BF16-exp fold, which are not exactly
// those of these FP32 factors).
hipError_t chain_bwd_pn(hipStream_t s, bool f64, const void* z, const double* ut, const double* m, const double* L,
                        void* w, long G, int T, int K, double a, double b, double var, const double* g,
                        const VSeries& vs = VSeries{}, bool renorm = false);
hipError_t plate_bwd_pn(hipStream_t s, bool f64, const void* zc, const void* zp, const int32_t* pidx,
                        const double* ut, const double* m, const void* wp, void* w, long n, int Kp, int K, int d,
                        double a, double b, double var, double* mone);
// var: the chain's step variance; F holds its linear-Gaussian step factors,
// which c0 = -log(2 pi var)/2 bounds (the forward's log-sum-exps use it).
hipError_t chain_fwd(hipStream_t s, bool f64, const void* F, double* ut, void* m, double* L,
                     long G, int T, int K, double var);
hipError_t chain_bwd(hipStream_t s, bool f64, const void* F, const double* ut, const void* m,
                     const double* L, void* w, long G, int T, int K, const double* dlogphat);

// chains in BF16-exp mode (K in {64, 128, 256}): MFMA transfer-matrix forward
// fold over BF16 exp-shifted factors formed in the kernel from the samples z
// (FP32 [series * T, K]); the reverse pass is chain_bwd_pn with renorm.
bool chain_bexp_supported(int K);
hipError_t chain_bexp_fwd(hipStream_t s, const void* z, double* ut, double* msg, double* L, long G, int T, int K,
                          double a, double b, double var);

// two root parents (a, b):  m[i,ka,kb] = C[ka,kb] + LSE_k (ga0[ka] + ga1[ka]*gk[i,k] + H + ut[i,k])
// with H = hb[kb]*hk[i,k] (hmat == null) or hmat[i,kb,k].
struct TwoParentArgs {
    const double* ga0; const double* ga1; const double* gk;   // [Ka], [Ka], [n,K]  (FP64)
    const double* hb; const double* hk;                       // [Kb], [n,K] or null
    const void* hmat;                                         // [n,Kb,K] T or null
    const double* C;                                          // [Ka,Kb] or null
    const double* ut; double* m;                              // [n,K], [n,Ka,Kb] (FP64)
    long n; int Ka, Kb, K;
    // FP32, K = 64 or 128: per instance the arithmetic it takes, 0 FP32 GEMM,
    // 1 FP64 GEMM, TP_FLAG_EXACT the exact VALU kernels (written by the FP32
    // forward; every kernel skips the others' instances); null: VALU only
    uint8_t* flags;
};
constexpr uint8_t TP_FLAG_EXACT = 2;
// Two-parent contraction as FP32 exponential GEMMs on MFMA (see
// k_twoparent_mfma.hip); instances beyond its range bound are flagged.
bool twoparent_mfma_supported(bool f64, int Ka, int Kb, int K);
hipError_t twoparent_fwd_mfma(hipStream_t s, const TwoParentArgs& a);
hipError_t twoparent_bwd_mfma(hipStream_t s, const TwoParentArgs& a, const double* W, void* w);
hipError_t twoparent_fwd(hipStream_t s, bool f64, const TwoParentArgs& a);
// w[i,k] = sum_{ka,kb} W[ka,kb] exp(G + H + C + ut[i,k] - m[i,ka,kb])
hipError_t twoparent_bwd(hipStream_t s, bool f64, const TwoParentArgs& a, const double* W, void* w);
// per-node vectors of the separable two-parent factors
hipError_t twoparent_prep(hipStream_t s, bool f64, int prior, const void* za, const void* zb,
                          const void* zc, long n, int Ka, int Kb, int K,
                          double* ga0, double* ga1, double* gk, double* hb, double* hk, double* C);
// M[ka,kb] = sum_i m[i,ka,kb] (FP64, fixed order); called per two-parent node, accumulate != 0 adds.
hipError_t pair_sum(hipStream_t s, bool f64, const double* m, long n, int Ka, int Kb, double* M,
                    double* scratch, int accumulate);
// joint root: L = LSE_{ka,kb} (uta[ka] + utb[kb] + M[ka,kb]); W = g*exp(... - L);
// wa[ka] = sum_kb W, wb[kb] = sum_ka W.
hipError_t pair_root_fwd(hipStream_t s, const double* uta, const double* utb, const double* M,
                         int Ka, int Kb, double* L);
hipError_t pair_root_bwd(hipStream_t s, bool f64, const double* uta, const double* utb,
                         const double* M, const double* L, int Ka, int Kb, double* W,
                         void* wa, void* wb, const double* dlogphat);

// ---- moments and M-step ---------------------------------------------------
// mone[i,j,:] = sum_k w[i,k] (z[i,k,j], z[i,k,j]^2), or (z, log z) when logz
hipError_t moments(hipStream_t s, bool f64, const void* z, const void* w, double* mone,
                   long n, int K, int d, bool logz);
// EMA (skipped when the non-finite flag is set) then Q parameters.
hipError_t mstep(hipStream_t s, double* mema, const double* mone, double* qp, long count,
                 int qfamily, double lam, uint32_t* status, int d = 1);
// M-step of up to MSTEP_NODES nodes in one launch; advances *iter_dev when non-null.
constexpr int MSTEP_NODES = 8;
struct MstepTable {
    int n;
    double* mema[MSTEP_NODES];
    const double* mone[MSTEP_NODES];
    double* qp[MSTEP_NODES];
    long count[MSTEP_NODES];
    int qfamily[MSTEP_NODES];
    int dim[MSTEP_NODES];
    const double* lam_dev;                   // when set, the EMA weight is read here
    const double* lp_z;                      // when set, the moments are scaled by
    const double* lp_new;                    //   exp(*lp_z - *lp_new) (second-sample normaliser)
};
// log P_MP of the first sample, kept for the second-sample normaliser.
hipError_t copy_scalar(hipStream_t s, const double* src, double* dst);
hipError_t mstep_multi(hipStream_t s, const MstepTable& tb, double lam, uint32_t* status, uint64_t* iter_dev);
hipError_t reset_status(hipStream_t s, uint32_t* status);
// device iteration counter of graph replays: set, and advance by one
hipError_t iter_set(hipStream_t s, uint64_t* it, uint64_t v);
// ess_out[i] = 1 / sum_k w[i,k]^2 (FP64); mean_out (optional) = their mean.
hipError_t ess(hipStream_t s, bool f64, const void* w, long n, int K, double* ess_out, double* mean_out);
// qp <- (q0a, q0b) when set_q; then mema <- mean parameters of qp.
hipError_t init_q(hipStream_t s, double* qp, double* mema, long count, int qfamily, int set_q,
                  double q0a, double q0b, int d = 1);

// Status word bit of a forward row whose log-sum-exp is -inf (every entry of
// the row -inf: a parent sample under which the child's data have probability
// zero for every child sample); the value of QEM_FLAG_NEG_INF_ROW.
constexpr uint32_t FLAG_NEG_INF_ROW = 0x8u;

// ---- stream-bandwidth calibration (k_probe.hip) -----------------------------
// mode 0 write, 1 nontemporal write, 2 read, 3 nontemporal read; bytes a
// multiple of 16 KB.
hipError_t stream_probe(hipStream_t s, void* buf, size_t bytes, int mode, float* sink);

// ---- amortised encoder ----------------------------------------------------
int enc_nparam();
size_t enc_scratch_bytes(int n);
hipError_t enc_features(hipStream_t s, const double* y, const double* cov, int n, int J, int D, float* feat);
hipError_t enc_pool(hipStream_t s, const float* feat, int n, int J, float* rows);
hipError_t enc_features_ctx(hipStream_t s, const float* feat, const float* rows, int n, int J, float* out);
hipError_t enc_apply_res(hipStream_t s, const float* out, const float* rows, int n, double* qp);
hipError_t enc_fwd(hipStream_t s, const uint16_t* w, const float* x, int n, float* out, float* act);
hipError_t enc_kl(hipStream_t s, const float* out, const double* target, int n, float* dout, double* kl,
                  double* loss);
hipError_t enc_bwd(hipStream_t s, const uint16_t* w, const float* x, const float* act, const float* dout, int n,
                   float* grad, float* scratch);
// enc_bwd with the partial gradients in the library's own device array
// (no workspace argument); n <= ENC_NOALLOC_MAX_N, the stream on the current
// device.  Calls that overlap on one GPU share that array and race.
constexpr int ENC_NOALLOC_MAX_N = 16384;
hipError_t enc_bwd_noalloc(hipStream_t s, const uint16_t* w, const float* x, const float* act, const float* dout,
                           int n, float* grad);
hipError_t enc_adam(hipStream_t s, float* master, uint16_t* w, const float* grad, float* m1, float* m2, int step,
                    float lr, float b1, float b2, float eps);
hipError_t enc_to_bf16(hipStream_t s, const float* master, uint16_t* w);
hipError_t enc_apply(hipStream_t s, const float* out, int n, double* qp);
hipError_t enc_targets(hipStream_t s, const double* m, int n, double floor_v, const float* rows, double* target);

}  // namespace qemk
