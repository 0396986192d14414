/*
 * qem.h - C ABI of the QEM E-step library for AMD MI355X (gfx950).
 *
 * QEM ("Massively Parallel Expectation Maximization for Approximate
 * Posteriors", arXiv 2503.08264) alternates an E-step that estimates posterior
 * moments by massively parallel importance weighting (MPIW, section 3.2,
 * Eq. mp_iw) with an M-step that sets an exponential-family proposal Q from
 * an exponential moving average of those moments (Eq. ema, Algorithm 1).
 *
 * The library runs one E-step as six stream-ordered calls:
 *   qem_sample        K draws per latent instance from Q_t   (Algorithm 1, z ~ Q_t)
 *   qem_logfactors    unary u and pairwise F log-factor tensors of log r_k (Eq. rmp)
 *   qem_contract_fwd  log-space sum over all K^n index tuples by elimination:
 *                     log P_MP (Eq. Prmp) and the per-level partial log-sum-exps
 *   qem_contract_bwd  reverse pass: marginal weights w_v[i,k] = d log P_MP / d u_v[i,k]
 *   qem_moments       m_one_v[i,j] = sum_k w (z, z^2)          (Eq. mmp)
 *   qem_mstep         m_t = (1-lam) m_{t-1} + lam m_one_t, then Q_{t+1} from m_t
 *                                                              (Eq. ema, Algorithm 1)
 * and qem_step chains them as one iteration of Algorithm 1.
 *
 * Conventions
 *   - Every call is asynchronous on the context's HIP stream and returns a
 *     status for errors that the host can detect (null pointers, sizes,
 *     unsupported structure, unbound workspace).  Conditions found on the
 *     device (non-finite log P_MP, variance floor hits, Gamma mean <= 0) are
 *     recorded in a device status word read with qem_read_status.
 *   - The caller owns all device memory: a single workspace of
 *     qem_workspace_bytes() bytes bound with qem_bind_workspace, and the
 *     observation arrays named in the model description, which must stay valid
 *     and unchanged while the context lives.  The library never allocates or
 *     frees device memory and never synchronises the stream, except in
 *     qem_bind_workspace (one upload of index tables), qem_read_status and
 *     the kernel-timing calls qem_timing and qem_timing_read.
 *   - Every tensor of the E-step (samples, factors, messages, weights, moments,
 *     proposal parameters, log P_MP) lives in the workspace; qem_tensor gives
 *     its byte offset, element type and shape.
 *   - Reductions have a fixed order and use no floating-point atomics, so FP64
 *     results are bitwise reproducible run to run.
 *   - Distributions: Normal(mean, variance), Gamma(shape, rate).
 *   - Not thread-safe per context; one context per stream.
 */
#ifndef QEM_H
#define QEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qem_ctx_s* qem_ctx;

typedef enum {
    QEM_OK = 0,
    QEM_E_INVALID = 1,      /* null pointer, bad enum, bad value */
    QEM_E_SHAPE = 2,        /* sizes out of range or inconsistent */
    QEM_E_UNSUPPORTED = 3,  /* model structure outside what the kernels cover */
    QEM_E_DEVICE = 4,       /* a HIP runtime call failed */
    QEM_E_NONFINITE = 5,    /* (qem_read_status) log P_MP was not finite */
    QEM_E_STATE = 6         /* workspace not bound, or too small */
} qem_status;

/* Arithmetic of the sample, factor, message and weight tensors.  Sums across
 * plate instances, log P_MP, moments, EMA and M-step are FP64 in every mode.
 * QEM_BF16EXP folds chains with BF16 MFMA products (FP32 accumulation) of
 * transition factors taken as BF16 exponentials with FP32 row shifts, formed
 * in the fold kernel from the samples (no factor tensor), and runs the
 * chain's reverse pass on its FP32 factors with those messages, renormalising
 * each step's weights; everything else runs as in QEM_FP32. */
typedef enum { QEM_FP64 = 0, QEM_FP32 = 1, QEM_BF16EXP = 2 } qem_prec;

/* Proposal family of a node and its mean parameters (Algorithm 1 keeps an
 * EMA of these; section 4 recovers the parameters from them):
 *  - QEM_Q_GAUSS: N(mean, var) per dimension; (E z, E z^2); mean = m1,
 *    var = m2 - m1^2;
 *  - QEM_Q_GAMMA: Gamma(shape, rate); (E z, E z^2) and moment matching,
 *    v = m2 - m1^2, shape = m1^2 / v, rate = m1 / v;
 *  - QEM_Q_GAMMA_EF: Gamma(shape, rate) with its exponential-family mean
 *    parameters (E z, E log z): shape from log shape - psi(shape) =
 *    log m1 - m2 (Newton iteration in FP64), rate = shape / m1;
 *  - QEM_Q_BERNOULLI: a discrete latent z in {0, 1} with Q(z = 1) = p;
 *    (E z, E z^2) = (p, p); p = m1 clamped to [1e-9, 1 - 1e-9].  Parameters
 *    [n, 1, 2] hold (p, 1); samples are 0 or 1 in the tensor type.
 *  - QEM_Q_DIRICHLET: z on the simplex of dim = C >= 2 components (C = 2:
 *    a Beta latent as (z, 1 - z)), Q = Dir(alpha); per component the
 *    exponential-family mean parameters (E z_c, E log z_c) =
 *    (alpha_c / alpha_0, psi(alpha_c) - psi(alpha_0)); the M-step solves
 *    psi(alpha_c) - psi(alpha_0) = m2_c for all c (Newton in log alpha,
 *    FP64).  Parameters [n, C, 2] hold (alpha_c, 1).  A sample normalises C
 *    Gamma(alpha_c, 1) draws (Philox elements (i*K + k)*C + c) in log space;
 *    components below the tensor type's smallest normal are raised to it.
 *  - QEM_Q_CATEGORICAL: a one-hot latent over dim = C >= 2 categories,
 *    Q(c) = p_c / sum_j p_j; per category (E z_c, E z_c^2) = (p_c, p_c);
 *    p_c = m1_c clamped to [1e-9, 1].  Parameters [n, C, 2] hold (p_c, 1);
 *    sample e is the first c with u * P_{C-1} <= P_c (P the running sums of
 *    p, u the (0, 1] uniform of Philox counter (e, 0)), written one-hot.
 * Each floor (variance, log m1 - m2 below 1e-12, the Bernoulli clamp, a
 * Dirichlet gap 1 - sum_c exp(m2_c) below 1e-12, closed by shifting m2 down)
 * counts a floor hit. */
typedef enum {
    QEM_Q_GAUSS = 0, QEM_Q_GAMMA = 1, QEM_Q_GAMMA_EF = 2, QEM_Q_BERNOULLI = 3, QEM_Q_DIRICHLET = 4,
    QEM_Q_CATEGORICAL = 5
} qem_qfamily;

typedef enum {
    QEM_PRIOR_NORMAL = 0,          /* z ~ N(a*z_parent0 + b, var) per dim; no parent: N(b, var) */
    QEM_PRIOR_GAMMA = 1,           /* z ~ Gamma(shape, rate), constants, root only */
    QEM_PRIOR_GAMMA_PARENTS = 2,   /* z ~ Gamma(z_parent0, z_parent1) (shape node, rate node) */
    QEM_PRIOR_NORMAL_LOGSCALE = 3, /* z ~ N(0, exp(z_parent0)^2) */
    QEM_PRIOR_BERNOULLI_LOGIT = 4, /* z in {0,1} ~ Bernoulli(sigmoid(a*z_parent0 + b)); no parent:
                                      Bernoulli(sigmoid(b)); QEM_Q_BERNOULLI nodes only */
    QEM_PRIOR_DIRICHLET = 5,       /* z ~ Dir(shape, ..., shape) over dim components, no parent;
                                      QEM_Q_DIRICHLET nodes only (only categorical nodes may hang
                                      under one) */
    QEM_PRIOR_CATEGORICAL = 6      /* one-hot z, P(c) = z_parent0[c] with parent0 a QEM_Q_DIRICHLET
                                      node of the same dim (mixture weights); no parent: 1 / dim;
                                      QEM_Q_CATEGORICAL nodes only */
} qem_prior;

typedef enum {
    QEM_OBS_GAUSS = 0,             /* x[n, n_per, dim] ~ N(z, var) */
    QEM_OBS_POISSON = 1,           /* y[n, n_per] ~ Poisson(z) */
    QEM_OBS_BERNOULLI_LOGIT = 2,   /* y[n, n_per] ~ Bernoulli(sigmoid(cov[n,n_per,:] . z_coef + z)) */
    QEM_OBS_DETECTION = 3,         /* y[n, n_per] in {0,1} ~ Bernoulli(p z), z a QEM_Q_BERNOULLI
                                      latent (occupancy with imperfect detection), p = var */
    QEM_OBS_CATEGORICAL = 4,       /* y[n, n_per] in {0, .., dim-1} ~ Categorical(z), z a
                                      QEM_Q_DIRICHLET latent; reduced to per-category counts at
                                      bind time (values outside the range are not counted) */
    QEM_OBS_GAUSS_MIXTURE = 5      /* y[n, n_per] ~ N(mu_c, var), c the category of a
                                      QEM_Q_CATEGORICAL latent; cov: device FP64 [dim], the
                                      component means; reduced at bind time to
                                      sum_j log N(y_ij; mu_c, var) per (instance, category) */
} qem_obs_kind;

/* One latent node replicated over a plate of n instances (section 3.1's
 * model P(x, z') organised as plates; each instance is one latent of
 * Eq. mp_iw with its own K samples).  Nodes must be listed parents first
 * (parent ids smaller than the node's id). */
typedef struct {
    int32_t n;                    /* instances, >= 1 */
    int32_t dim;                  /* dimension of one sample; 1 for the Gamma families */
    int32_t qfamily;              /* qem_qfamily of this node's proposal factor */
    int32_t prior;                /* qem_prior */
    int32_t parent0, parent1;     /* parent node ids or -1 */
    const int32_t* parent_index;  /* host, [n]: instance of parent0 for each instance;
                                     NULL when parent0 has a single instance */
    double a, b, var;             /* QEM_PRIOR_NORMAL constants */
    double shape, rate;           /* QEM_PRIOR_GAMMA constants */
    int32_t chain_len;            /* T > 1: the n instances are n/T series laid out
                                     [series, T]; step t's parent is step t-1 of its
                                     series, step 0 ~ N(init_b, init_var).  0 or 1: no chain.
                                     With parent0 >= 0 (a scalar root or plate node, K <= 512,
                                     FP32/FP64): each series takes one instance beta of parent0
                                     (parent_index constant over the series; the region level of
                                     the appendix F AR(1) chains), step 0 ~ N(beta + init_b,
                                     init_var), step t ~ N(a x_{t-1} + (1 - a) beta + b, var);
                                     the series is eliminated once per sample of beta */
    double init_b, init_var;
    double q0a, q0b;              /* initial proposal Q_0 of every instance and dimension:
                                     Gaussian (mean, var) or Gamma (shape, rate) */
} qem_node_desc;

/* Observations of one latent node.  Every instance has n_per observations. */
typedef struct {
    int32_t node;                 /* observed latent node */
    int32_t kind;                 /* qem_obs_kind */
    int32_t n_per;                /* observations per instance, >= 1 */
    int32_t n_cov;                /* covariate width (QEM_OBS_BERNOULLI_LOGIT), else 0 */
    int32_t coef;                 /* node holding the coefficient vector, or -1 */
    double var;                   /* QEM_OBS_GAUSS variance; QEM_OBS_DETECTION probability in (0, 1) */
    const double* x;              /* device, FP64: [n, n_per, dim] (GAUSS) or [n, n_per] */
    const double* cov;            /* device, FP64: [n, n_per, n_cov] (BERNOULLI_LOGIT) or NULL */
} qem_obs_desc;

typedef struct {
    int32_t n_nodes;
    int32_t n_obs;
    const qem_node_desc* nodes;
    const qem_obs_desc* obs;
} qem_model_desc;

/* Supported structure (else QEM_E_UNSUPPORTED): every node has at most two
 * factor parents (prior parents plus an observation's coefficient node).
 *  - one factor parent: any earlier node (a plate under its parent's plate);
 *  - two factor parents: both roots with one instance; all such nodes share
 *    the same pair, which is then summed jointly (K^2 combinations);
 *  - chains have no factor parent;
 *  - 1 <= K <= 512 (K <= 256 for two-parent nodes; chains in QEM_BF16EXP
 *    need K in {64, 128, 256}). */

/* Create a context for a model, K samples per latent instance, precision
 * prec (qem_prec), on HIP stream `stream` (a hipStream_t; NULL = default
 * stream).  Host-only: validates the description and plans the workspace. */
qem_status qem_create(qem_ctx* out, const qem_model_desc* model, int32_t K,
                      int32_t prec, void* stream);

/* Create flags of qem_create_ex. */
#define QEM_CREATE_NO_TABLES 0x1u
#define QEM_CREATE_CHAIN_TABLES 0x2u

/* qem_create with flags (0 = qem_create).
 * QEM_CREATE_NO_TABLES: the pairwise log-factor of a linear-Gaussian plate
 * node (one Normal prior parent, no observation coefficient, a shape the
 * recomputing kernels accept) is not kept in the workspace; the forward and
 * reverse passes evaluate it from the samples where they read it.  The K^2
 * table per instance is the workspace's largest part, so this trades its HBM
 * traffic and footprint for arithmetic.  Results are the same bits as with
 * the table (the same expression in the same order); QEM_T_F of such a node
 * returns QEM_E_INVALID.  Other nodes keep their tables.
 * Chains never keep their step-factor table unless QEM_CREATE_CHAIN_TABLES
 * is given (and QEM_CREATE_NO_TABLES is not; never in QEM_BF16EXP): the
 * [series, T-1, K, K] table is written and read once per pass at the memory
 * rate of one workgroup per series, while evaluating each entry where it is
 * used costs less (at 1024 series x 64 steps, K = 256, FP32: 3.4 ms per
 * iteration against 8.1 ms with the 17 GB table).  Same bits either way.
 * Unknown flags: QEM_E_INVALID. */
qem_status qem_create_ex(qem_ctx* out, const qem_model_desc* model, int32_t K,
                         int32_t prec, uint32_t flags, void* stream);
void qem_destroy(qem_ctx ctx);

/* Text of the last error on this context (or of the last failed qem_create
 * on this thread when ctx is NULL).  Valid until the next call. */
const char* qem_last_error(qem_ctx ctx);

/* Bytes of device memory the context needs (256-byte aligned sub-buffers). */
size_t qem_workspace_bytes(qem_ctx ctx);

/* Bind caller-owned device memory of at least qem_workspace_bytes() bytes,
 * 256-byte aligned.  Uploads the plate index tables, computes the
 * observations' sufficient statistics, applies qem_init(ctx, -1) and
 * synchronises the stream once.  Binding again (the same or another buffer)
 * starts over from Q_0 and discards the graphs qem_run captured, which hold
 * the previous buffer's addresses; the previous buffer is no longer used. */
qem_status qem_bind_workspace(qem_ctx ctx, void* dev, size_t bytes);

/* Algorithm 1's initial values: Q of node `node` (every node when -1) set to
 * the description's Q_0, and the EMA state m_0 to Q_0's mean parameters
 * (Gaussian: (mean, mean^2 + var); Gamma: (shape/rate, shape(shape+1)/rate^2);
 * exponential-family Gamma: (shape/rate, psi(shape) - log rate)). */
qem_status qem_init(qem_ctx ctx, int32_t node);

/* m_0 of node `node` (every node when -1) from the proposal parameters
 * currently in QEM_T_QPARAM, e.g. written by an amortised encoder. */
qem_status qem_init_from_q(qem_ctx ctx, int32_t node);

typedef enum {
    QEM_T_QPARAM = 0,   /* [n, dim, 2] f64: Gaussian (mean, var) | Gamma (shape, rate) | Bernoulli (p, 1)
                           | Dirichlet (alpha_c, 1) */
    QEM_T_MEMA = 1,     /* [n, dim, 2] f64: EMA mean parameters (E z, E z^2), (E z, E log z) for
                           QEM_Q_GAMMA_EF and QEM_Q_DIRICHLET */
    QEM_T_MONE = 2,     /* [n, dim, 2] f64: this E-step's moments (same statistics) */
    QEM_T_Z = 3,        /* [n, K, dim] T: samples */
    QEM_T_U = 4,        /* [n, K] T: unary log-factors (incl. -log Q - log K) */
    QEM_T_F = 5,        /* [n, Kp, K] T pairwise log-factors (one factor parent);
                           chains: [series, T-1, K, K]; two-parent nodes with a
                           likelihood term: [n, Kb, K] */
    QEM_T_UT = 6,       /* [n, K] f64: u plus the messages of all child instances */
    QEM_T_MSG = 7,      /* f64 partial log-sum-exps: [n, Kp] | two-parent [n, Ka, Kb] | chain [series, T, K]
                           | chain under a parent [series, Kb, T, K] (per parent sample kb)
                           (chain row t >= 1: the message of step t into step t-1; row 0 is not written) */
    QEM_T_W = 8,        /* [n, K] T: marginal weights */
    QEM_T_ROOTL = 9,    /* [n] or [series] f64: per-component log-sum-exp at the root;
                           chain under a parent: [series, Kb], the message of each series
                           into its parent instance */
    QEM_T_LOGPHAT = 10, /* [1] f64 (node -1) */
    QEM_T_STATUS = 11,  /* [4] u32 (node -1): flags, variance-floor hits, 2 reserved */
    QEM_T_PAIR_M = 12,  /* [Ka, Kb] f64 (node -1): sum over instances of two-parent messages */
    QEM_T_PAIR_W = 13,  /* [Ka, Kb] f64 (node -1): joint root weights */
    QEM_T_FSHIFT = 14   /* reserved (row shifts of a stored BF16-exp chain table, which is no
                           longer kept): QEM_E_INVALID */
} qem_tensor_kind;

typedef enum { QEM_DT_F64 = 0, QEM_DT_F32 = 1, QEM_DT_U32 = 2, QEM_DT_BF16 = 3 } qem_dtype;

typedef struct {
    size_t offset;      /* bytes from the workspace base */
    size_t bytes;
    int32_t dtype;      /* qem_dtype */
    int32_t ndim;
    int64_t shape[4];
} qem_tensor_info;

/* Location of a workspace tensor; node = -1 for the global tensors.
 * Returns QEM_E_INVALID when the node has no such tensor. */
qem_status qem_tensor(qem_ctx ctx, int32_t node, int32_t kind, qem_tensor_info* out);

/* Status flags (word 0 of QEM_T_STATUS), cleared by each iteration's sampling
 * call and set by the device:
 *   QEM_FLAG_NONFINITE_LOGPHAT  log P_MP is not finite (the EMA update is skipped);
 *   QEM_FLAG_VAR_FLOOR          an M-step variance (or another floored mean
 *                               parameter) hit its floor (count in word 1);
 *   QEM_FLAG_GAMMA_MEAN         a Gamma M-step had E z <= 0;
 *   QEM_FLAG_NEG_INF_ROW        a plate forward row had log-sum-exp -inf: for
 *                               some instance and parent sample, every child
 *                               sample has a factor or u-tilde of -inf (data of
 *                               probability zero under that parent sample).
 *                               The row's message is -inf and the reverse pass
 *                               gives that parent sample's branch weight 0.
 *                               Chain and two-parent factors here are finite
 *                               densities, so their rows never are all -inf. */
#define QEM_FLAG_NONFINITE_LOGPHAT 0x1u
#define QEM_FLAG_VAR_FLOOR         0x2u
#define QEM_FLAG_GAMMA_MEAN        0x4u
#define QEM_FLAG_NEG_INF_ROW       0x8u

/* The E-step and M-step calls.  Seeds and iteration numbers key a Philox4x32-10
 * stream (Salmon et al., SC'11) with key (seed lo, seed hi).  For element
 * e = (i*K + k)*dim + j of node v at iteration t: a Gaussian proposal takes
 * the cosine (e even) or sine (e odd) Box-Muller branch of the block at
 * counter (e >> 1, 0, t, v); a Gamma proposal runs Marsaglia-Tsang on
 * counters (e, 1 + 2a, t, v), (e, 2 + 2a, t, v) for attempt a and boosts a
 * shape below 1 with the uniform at (e, 0, t, v). */
/* iter <= 2^32 - 1 (a Philox counter word), else QEM_E_INVALID. */
qem_status qem_sample(qem_ctx ctx, uint64_t seed, uint64_t iter);
qem_status qem_logfactors(qem_ctx ctx);
qem_status qem_contract_fwd(qem_ctx ctx);
/* dlogphat: device pointer to one f64 scaling the weights (the upstream
 * gradient of log P_MP), or NULL for 1. */
qem_status qem_contract_bwd(qem_ctx ctx, const double* dlogphat);
qem_status qem_moments(qem_ctx ctx);
/* EMA with weight lam on the new moments, then Q from the EMA.  The EMA is
 * skipped (m_{t-1} kept) when this iteration's log P_MP was not finite.
 * lam = 0 only refreshes Q from QEM_T_MEMA. */
qem_status qem_mstep(qem_ctx ctx, double lam);
/* One iteration of Algorithm 1 after Q_t is set: sample, log-factors,
 * forward and reverse contraction, moments, EMA and M-step for Q_{t+1}.
 * QEM_E_INVALID when iter is 0 under the t^-p step size of qem_set_ema, or
 * above 2^32 - 1 (2^31 - 1 with the second sample, whose stream flips the
 * counter word's top bit). */
qem_status qem_step(qem_ctx ctx, uint64_t seed, uint64_t iter, double lam);

/* Options of the EMA in qem_step and qem_run (the stage call qem_mstep is not
 * affected).  p = 0: weight lam on the new moments (Eq. ema).  0 < p < 1: the
 * decreasing step t^-p of Theorem 1 at iteration t (lam is then ignored).
 * second_sample = 1: after the E-step a second, independent sample of the
 * same Q_t (Philox iteration word t XOR QEM_SECOND_SAMPLE_STREAM) is drawn and
 * contracted, and the moments enter the EMA scaled by P_MP(z) / P_MP(z_new),
 * the variant discussed after Theorem 1 (the unnormalised estimate divided
 * by the marginal likelihood of a distinct sample).  Iterations start at
 * t = 1 under the t^-p step (qem_step and qem_run reject t = 0).  The EMA is skipped when
 * either log P_MP is not finite.  After such a step, QEM_T_LOGPHAT, the
 * weights and the moments belong to the first sample; samples, factors,
 * u-tilde and messages to the second.  QEM_E_INVALID unless 0 <= p < 1 and
 * second_sample is 0 or 1.  A captured qem_run graph is rebuilt. */
#define QEM_SECOND_SAMPLE_STREAM 0x80000000u
qem_status qem_set_ema(qem_ctx ctx, double p, int32_t second_sample);

/* n_iter iterations of Algorithm 1 (each as qem_step) with iteration numbers
 * iter0, iter0+1, ...  One iteration, and eight in a row, are captured once
 * as HIP graphs (again when seed or lam change) and replayed: the eight-
 * iteration graph while at least eight remain, then the one-iteration graph.
 * The iteration number lives in a device counter that each iteration
 * advances.  Results equal n_iter calls of qem_step.  Kernel timing does not
 * see replayed kernels.  Every iteration number must pass qem_step's checks
 * (QEM_E_INVALID otherwise, before anything is launched). */
qem_status qem_run(qem_ctx ctx, uint64_t seed, uint64_t iter0, double lam, int32_t n_iter);

/* Marginal effective sample size of every instance of `node` from this
 * E-step's weights (QEM_T_W): ess[i] = 1 / sum_k w[i,k]^2 in FP64 (ess: a
 * device buffer of n doubles, caller-owned), and, when mean is not NULL, their
 * mean (a device double; fixed-order sum).  K for weights concentrated on one
 * sample, K for uniform weights.  Stream-ordered; QEM_E_INVALID for a bad
 * node or a null ess. */
qem_status qem_ess(qem_ctx ctx, int32_t node, double* ess, double* mean);

/* Synchronise the stream and read the status flags, floor-hit count and
 * log P_MP.  Returns QEM_E_NONFINITE when the flag is set. */
qem_status qem_read_status(qem_ctx ctx, uint32_t* flags, uint32_t* floor_hits, double* logphat);

/* Kernel timing (tracing).  While enabled, every kernel launch of the E-step
 * and M-step calls is bracketed by a pair of HIP events recorded on the
 * context's stream, and durations are accumulated per (node, phase);
 * node -1 holds the global kernels.  qem_timing (enable or disable)
 * synchronises the stream, drops the events still pending and clears the
 * accumulators; qem_timing_read synchronises the stream. */
typedef enum {
    QEM_PH_SAMPLE = 0, QEM_PH_UNARY = 1, QEM_PH_PAIRTABLE = 2, QEM_PH_PLATE_FWD = 3,
    QEM_PH_PLATE_BWD = 4, QEM_PH_CHAIN_FWD = 5, QEM_PH_CHAIN_BWD = 6, QEM_PH_TP_FWD = 7,
    QEM_PH_TP_BWD = 8, QEM_PH_CHILDSUM = 9, QEM_PH_ROOT = 10, QEM_PH_MOMENTS = 11,
    QEM_PH_MSTEP = 12, QEM_PH_COUNT = 13
} qem_phase;
qem_status qem_timing(qem_ctx ctx, int32_t enable);
qem_status qem_timing_read(qem_ctx ctx, int32_t node, int32_t phase, double* total_ms, int64_t* launches);

/* Stream-bandwidth calibration (a measurement aid, not part of the method):
 * one pass of a plain (mode 0) or nontemporal (1) write stream, or a plain
 * (2) or nontemporal (3) read stream, of 16-byte accesses over the device
 * buffer buf[bytes], each workgroup covering one contiguous 16 KB chunk (the
 * per-instance tile of the K = 64 plate kernels).  Reads sum the data and
 * store into sink (a device float) only on a NaN, so run them on a buffer a
 * write pass has filled.  bytes a positive multiple of 16384 (QEM_E_SHAPE
 * otherwise); asynchronous on `stream`.  The benchmark times these passes to
 * state the rates the chip sustains for such streams beside the HBM peak. */
qem_status qem_stream_probe(void* buf, size_t bytes, int32_t mode, float* sink, void* stream);

/* ------------------------------------------------------------------------
 * Amortised encoder of a group's Gaussian proposal factor (not in the paper).
 * It initialises Q for QEM: an MLP maps a group's data summary to the mean
 * and log variance of that group's proposal; it is trained on the posterior
 * moments QEM produces, with the KL objective of appendix B (maximum
 * likelihood of the proposal under the estimated posterior), and plain QEM is
 * its fallback.  Architecture 18 -> 64 -> 64 -> 2, exact GELU x*Phi(x),
 * BF16 weights (round to nearest even from FP32 master weights), FP32
 * accumulation.  Parameter layout (QEM_ENC_NPARAM floats):
 *   W1[64][18] b1[64] W2[64][64] b2[64] W3[2][64] b3[2]   (row-major).
 * All pointers are device pointers owned by the caller; calls are
 * asynchronous on `stream` (a hipStream_t; NULL = default stream).
 * ------------------------------------------------------------------------ */
#define QEM_ENC_IN 18
#define QEM_ENC_HID 64
#define QEM_ENC_NPARAM 5506

/* feat[n, 18] (FP32) = [1, mean_o y, mean_o cov (8), mean_o y*cov (8)] from
 * y[n, n_per] and cov[n, n_per, 8] (FP64).  QEM_E_SHAPE unless n_cov == 8. */
qem_status qem_enc_features(const double* y, const double* cov, int32_t n, int32_t n_per, int32_t n_cov,
                            float* feat, void* stream);
/* Input rows of the global head, a second network of the same architecture
 * and kernels that initialises the global latents beta[8] and log sigma:
 * rows[9, 18] (FP32) from one dataset's group features feat[n, 18] (groups of
 * n_per observations), pooled in FP64 with fixed-order reductions.  Feature 1
 * of every row is a plug-in estimate of its latent; the head predicts the
 * residual (qem_enc_apply_residual).
 * Pass 1: P = mean feature, V = variance of the group means of y,
 *   P_yx = P[10..17], u = P_yx / |P_yx|.  Stein's lemma gives, for Gaussian
 *   covariates, E[y x] = E[sigma'(eta)] beta with eta ~ N(0, |beta|^2 + sigma^2),
 *   so B = |beta| solves c(sqrt(B^2 + sigma^2)) B = |P_yx| with
 *   c(s) = E[sigma'(s Z)] (trapezoid rule on [-10, 10], step 0.05; bisection
 *   on [0, 50], 60 steps); beta^ = u B.
 * Pass 2: kappa = 4 c(B); per group the empirical logit
 *   e = log(yc / (1 - yc)), yc = (ybar n_per + 1/2) / (n_per + 1), a = e - kappa xbar . beta^,
 *   noise = 1 / (n_per yc (1 - yc)); sigma^2 = max((Var(a) - kappa mean noise) / kappa^2, 1e-4).
 *   B starts at sigma = 0; B and sigma alternate 3 times.
 *   row j < 8 (beta_j): [1, beta^_j, u_j, B, 5|P_yx|, 4 sqrt V, 0, 5 P[2+j], P[1], kappa, 0 ...]
 *   row 8 (log sigma):  [1, log(sigma^2)/2, 0, B, 5|P_yx|, 4 sqrt V, 1, 0, P[1], kappa, Var(a), mean noise, 0 ...]
 * QEM_E_SHAPE if n < 1 or n_per < 1. */
qem_status qem_enc_pool(const float* feat, int32_t n, int32_t n_per, float* rows, void* stream);
/* Group features with the dataset context of rows (from qem_enc_pool): for
 * group i with mean outcome ybar and the quantities of qem_enc_pool,
 *   out[i] = [1, ybar, xbar . beta^, mean(y x) . beta^, e, e / kappa - xbar . beta^,
 *             exp(rows[8, 1]), B, kappa, 1 / (n_per yc (1 - yc) kappa), 0 ...]
 * The group encoder reads these instead of the raw summaries, so its proposal
 * for b_i can depend on the dataset's global latents. */
qem_status qem_enc_features_ctx(const float* feat, const float* rows, int32_t n, int32_t n_per, float* out,
                                void* stream);
/* out[n, 2] = (mean, log var); act[n, 128] (optional) keeps the two
 * pre-activation layers for qem_enc_bwd. */
qem_status qem_enc_fwd(const uint16_t* w_bf16, const float* feat, int32_t n, float* out, float* act, void* stream);
/* Per-group KL(N(target mean, target var) || N(out mean, exp(out log var)))
 * into kl[n] (FP64), its gradient divided by n into dout[n, 2], and the mean
 * KL into *loss (FP64, fixed-order reduction) when loss is not NULL.
 * target[n, 2] = (mean, var), FP64. */
qem_status qem_enc_loss(const float* out, const double* target, int32_t n, float* dout, double* kl, double* loss,
                        void* stream);
/* Bytes of scratch qem_enc_bwd needs for n groups. */
size_t qem_enc_scratch_bytes(int32_t n);
/* grad[QEM_ENC_NPARAM] = sum over the n groups of d loss / d params
 * (overwritten; partial sums per 32-group chunk added in chunk order). */
qem_status qem_enc_bwd(const uint16_t* w_bf16, const float* feat, const float* act, const float* dout, int32_t n,
                       float* grad, void* scratch, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc): as
 * qem_enc_bwd, same kernels and result, with the partial gradients kept in a
 * device array the library owns instead of a caller's scratch buffer.  The
 * array holds QEM_ENC_NOALLOC_MAX_N groups (11.3 MB); every GPU the library
 * runs on keeps its own copy until the process ends.  No device memory is
 * allocated or freed by the call.  QEM_E_SHAPE if n < 1 or
 * n > QEM_ENC_NOALLOC_MAX_N; QEM_E_INVALID for a null pointer or a stream
 * that does not belong to the current device.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (different streams, or
 * host threads) race and must be ordered by the caller. */
#define QEM_ENC_NOALLOC_MAX_N 16384
qem_status qem_enc_bwd_noalloc(const uint16_t* w_bf16, const float* feat, const float* act, const float* dout,
                               int32_t n, float* grad, void* stream);
/* One Adam step (Kingma and Ba, 2015; step >= 1) on the FP32 master weights,
 * then the BF16 copy; m1, m2 are the moment buffers (zero before step 1). */
qem_status qem_enc_adam(float* master, uint16_t* w_bf16, const float* grad, float* m1, float* m2, int32_t step,
                        float lr, float beta1, float beta2, float eps, void* stream);
/* w_bf16 = round-to-nearest-even(master). */
qem_status qem_enc_to_bf16(const float* master, uint16_t* w_bf16, void* stream);
/* Training targets of the encoder from EMA mean parameters (the posterior
 * summaries plain QEM produces): mema[n][2] = (E z, E z^2) (FP64; a Gaussian
 * node's QEM_T_MEMA, n instances of a scalar latent or the dims of one vector
 * latent), target[n][2] = (E z - rows[i, 1], max(E z^2 - (E z)^2, var_floor)),
 * the rows term only when rows (qem_enc_pool's [n, 18] FP32 rows, whose
 * feature 1 is the plug-in estimate the global head's output is a residual
 * of) is not NULL.  QEM_E_SHAPE if n < 1. */
qem_status qem_enc_targets(const double* mema, int32_t n, double var_floor, const float* rows, double* target,
                           void* stream);
/* Write (mean, var = exp(log var)) of n rows into a proposal-parameter
 * tensor laid out [n, 2] (QEM_T_QPARAM of a Gaussian node: its n instances of
 * a scalar latent, or the d dimensions of one vector latent). */
qem_status qem_enc_apply(const float* out, int32_t n, double* qparam, void* stream);
/* As qem_enc_apply for the global head, whose mean output is a residual of the
 * plug-in feature of its input row: mean_i = rows[i, 1] + out[i, 0],
 * var_i = exp(out[i, 1]).  rows[n, 18] as written by qem_enc_pool. */
qem_status qem_enc_apply_residual(const float* out, const float* rows, int32_t n, double* qparam, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* QEM_H */
