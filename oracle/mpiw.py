"""MPIW E-step and QEM loop, written plainly in FP64 (oracle side).

What is computed (paper section 3.2, Eq. mp_iw, and Algorithm 1):

* K samples z_i^1..z_i^K for every latent instance i, drawn from the
  independent proposal Q (Q_MP reduces to Q when the proposal has no
  parents, which is the case for every model here).
* For an index tuple k in {1..K}^n:  r_k = P(x, z^k) / prod_i Q(z_i^{k_i})
  (Eq. rmp), and the marginal-likelihood estimate
  P_MP = K^-n sum_k r_k (Eq. Prmp).
* The moment estimate m_MP = K^-n sum_k (r_k / P_MP) m(z^k) (Eq. mmp); with
  m = (z, z^2) per latent this is sum_k w_i[k] (z_i^k, (z_i^k)^2), where
  w_i[k] is the share of the total weight of the tuples whose i-th index is k.
* EMA of the mean parameters m_t = (1 - lam) m_{t-1} + lam m_one_t
  (Eq. ema) and the M-step that sets the proposal from its mean parameters
  (Algorithm 1; Gaussian: mean m1 and variance m2 - m1^2).

Two ways to evaluate the sums are provided:

``brute_force_*``  enumerate every tuple k (tiny models only);
``contract``/``reverse``  variable elimination that exploits the model's
    conditional independence (the contraction the paper relies on, section
    3.2 and section 6): each latent is summed out children-first, giving
    log P_MP, then a parents-first pass gives the marginal weights.

Log factors.  Every term of log r_k depends on one latent instance, on an
instance and its parent, or (two-parent nodes) on an instance and a pair of
single-instance root nodes:
    unary  u_v[i,k]      = own observations + root prior - log Q - log K
    pair   F_v[i,kp,k]   = terms linking instance i of v to its factor parent
    triple T_v[i,ka,kb,k] for the two-parent case.
The -log K per latent instance accounts for the 1/K^n of Eq. Prmp.

Mean parameters.  Gaussian and moment-matched Gamma proposals use
m = (z, z^2); the exponential-family Gamma proposal ("gamma_ef") uses its
sufficient statistics m = (z, log z), whose mean parameters
(shape / rate, psi(shape) - log rate) map back to (shape, rate) by solving
log shape - psi(shape) = log m1 - m2 (section 4: parameters recovered from
the mean parameters of the exponential family).

Chains under a parent (a chain node with one prior parent, scalar): series g
of length T has parent instance p(g) (parent_index is constant within a
series); x_{g,0} ~ N(beta + init_b, init_var) and x_{g,t} ~ N(a x_{g,t-1}
+ (1 - a) beta + b, var) with beta = z_parent[p(g)]: an AR(1) around the
parent's level.  Eliminating the chain leaves a message over the parent's K
samples: the chain is eliminated once per parent sample.

Dirichlet latents ("dirichlet", d = C >= 2 components on the simplex; Beta
is C = 2): Q = Dir(alpha); a sample normalises C Gamma(alpha_c, 1) draws
(in log space); mean parameters (E z_c, E log z_c) = (alpha_c / alpha_0,
psi(alpha_c) - psi(alpha_0)), alpha_0 = sum_c alpha_c; the M-step solves
psi(alpha_c) - psi(alpha_0) = m2_c for all c (the exponential-family
moment match; section 4), which has a solution when sum_c exp(m2_c) < 1;
symmetric Dirichlet prior Dir(shape, ..., shape); categorical observations
y_ij in {0..C-1} ~ Categorical(z_i), entering through their counts.

Categorical latents ("categorical", d = C >= 2): a sample is the one-hot
vector of a category, Q(c) = p_c / sum_j p_j; mean parameters (E z_c, E z_c^2)
= (p_c, p_c); M-step p_c = m1_c clamped to [BERN_FLOOR, 1]; the category of
sample e is the first c with u * P_{C-1} <= P_c, P the running sums of p and
u the (0, 1] uniform of counter (e, 0).  Prior: uniform over the C
categories, or Categorical(pi) with pi a Dirichlet parent's sample (the
mixture weights); Gaussian-mixture observations y_ij ~ N(mu_c, var) with the
component means mu given.

Discrete latents ("bernoulli"): Q(z = 1) = p, mean parameters (E z, E z^2)
= (p, p), M-step p = m1 clamped to [BERN_FLOOR, 1 - BERN_FLOOR]; prior
Bernoulli(sigmoid(a z_parent + b)); detections y_r ~ Bernoulli(p_det z).

Readings where the paper is silent: N(mean, variance); Gamma(shape, rate);
a d-dimensional latent is one latent with K vector samples; LSE of an
all -inf row is -inf and the weights under it are zero.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
from scipy.optimize import brentq, root
from scipy.special import digamma, polygamma

from . import densities as dn
from . import philox

VAR_FLOOR = 1e-12
# exponential-family Gamma: floor of log m1 - m2, which is positive unless Q
# is a point mass (Jensen); hits are counted with the variance-floor hits
EF_GAP_FLOOR = 1e-12
# Bernoulli proposals keep p in [BERN_FLOOR, 1 - BERN_FLOOR]; clamps are counted with the floor hits
BERN_FLOOR = 1e-9
# Dirichlet M-step: mean parameters with 1 - sum_c exp(E log z_c) below this
# gap are moved back to it (a floor hit) before the solve.
DIR_GAP_FLOOR = 1e-12
TABLE_BYTES = 1 << 28   # chunk size for large factor tables


# --------------------------------------------------------------------------
# helpers

def lse(a, axis):
    """log sum exp along ``axis``; -inf where every entry is -inf."""
    a = np.asarray(a, dtype=np.float64)
    mx = np.max(a, axis=axis, keepdims=True)
    sh = np.where(np.isfinite(mx), mx, 0.0)
    with np.errstate(divide="ignore"):
        out = np.log(np.sum(np.exp(a - sh), axis=axis, keepdims=True)) + sh
    return np.squeeze(out, axis=axis)


def factor_parents(model, v: int):
    """Latent nodes that share a factor with node v: prior parents, then
    the coefficient node of a Bernoulli-logit observation."""
    ps = list(model.nodes[v].parents)
    for ob in model.obs:
        if ob.node == v and ob.kind == "bernoulli_logit" and ob.coef not in ps:
            ps.append(ob.coef)
    return tuple(ps)


def pair_roots(model):
    """The (a, b) roots of the two-parent nodes (at most one pair)."""
    pairs = {factor_parents(model, v) for v in range(len(model.nodes))
             if len(factor_parents(model, v)) == 2}
    assert len(pairs) <= 1, "at most one root pair is supported"
    return next(iter(pairs)) if pairs else None


def _chunks(n: int, row_bytes: int):
    """Slices of at most TABLE_BYTES / WORKERS bytes of table rows each (so
    the tables of the chunks in flight stay within TABLE_BYTES)."""
    step = max(1, TABLE_BYTES // max(row_bytes, 1) // max(WORKERS, 1))
    for s in range(0, n, step):
        yield slice(s, min(n, s + step))


# Threads that evaluate independent chunks of instances at once (numpy
# releases the interpreter lock inside its array operations).  Each chunk's
# result is the same whatever the number of threads; every sum across
# instances is still taken afterwards, in instance order.
WORKERS = 1


def _map_chunks(fn, slices):
    """[fn(sl) for sl in slices], on WORKERS threads when WORKERS > 1."""
    slices = list(slices)
    if WORKERS <= 1 or len(slices) <= 1:
        return [fn(sl) for sl in slices]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=WORKERS) as ex:
        return list(ex.map(fn, slices))


# --------------------------------------------------------------------------
# proposal: parameters, mean parameters, sampling (Algorithm 1)

def q_init(model) -> List[Dict[str, np.ndarray]]:
    """Initial proposal Q_0 (constants from the model description)."""
    qs = []
    for nd in model.nodes:
        a, b = nd.q0
        if nd.qfamily == "gauss":
            qs.append({"mean": np.full((nd.n, nd.dim), a), "var": np.full((nd.n, nd.dim), b)})
        elif nd.qfamily == "bernoulli":
            qs.append({"p": np.full((nd.n, 1), a)})
        elif nd.qfamily == "dirichlet":
            qs.append({"alpha": np.full((nd.n, nd.dim), a)})
        elif nd.qfamily == "categorical":
            qs.append({"p": np.full((nd.n, nd.dim), a)})
        else:
            qs.append({"shape": np.full((nd.n, 1), a), "rate": np.full((nd.n, 1), b)})
    return qs


def mean_params(model, qs) -> List[np.ndarray]:
    """Mean parameters of each proposal factor, [n, d, 2]: (E z, E z^2), or
    (E z, E log z) for the exponential-family Gamma."""
    out = []
    for nd, q in zip(model.nodes, qs):
        if nd.qfamily == "gauss":
            m1, m2 = q["mean"], q["mean"] ** 2 + q["var"]
        elif nd.qfamily == "gamma_ef":
            m1 = q["shape"] / q["rate"]
            m2 = digamma(q["shape"]) - np.log(q["rate"])
        elif nd.qfamily in ("bernoulli", "categorical"):
            m1, m2 = q["p"], q["p"]
        elif nd.qfamily == "dirichlet":
            a0 = q["alpha"].sum(-1, keepdims=True)
            m1 = q["alpha"] / a0
            m2 = digamma(q["alpha"]) - digamma(a0)
        else:
            m1 = q["shape"] / q["rate"]
            m2 = q["shape"] * (q["shape"] + 1.0) / q["rate"] ** 2
        out.append(np.stack([m1, m2], axis=-1))
    return out


def ef_gamma_shape(gap: float) -> float:
    """The shape a with log a - psi(a) = gap (> 0), by bracketing root search;
    the left side decreases from +inf to 0 as a grows."""
    f = lambda a: np.log(a) - digamma(a) - gap
    lo, hi = 1e-300, 1.0
    while f(hi) > 0.0:
        lo, hi = hi, hi * 2.0
    return float(brentq(f, lo, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500))


def dirichlet_alpha(L, mbar):
    """The concentration alpha with psi(alpha_c) - psi(sum alpha) = L_c for all c
    (requires sum_c exp(L_c) < 1).  Root search in log alpha with the exact
    Jacobian, from the precision that psi(x) ~ log x - 1/(2x) implies for the
    means ``mbar``; the residual is checked."""
    L = np.asarray(L, dtype=np.float64)
    m = np.clip(np.asarray(mbar, dtype=np.float64), 1e-300, None)
    m = m / m.sum()
    gap = np.sum(m * np.maximum(np.log(m) - L, 1e-300))
    s0 = max(np.sum(1.0 - m) / (2.0 * gap), 1e-6)

    def f(x):
        a = np.exp(x)
        return digamma(a) - digamma(a.sum()) - L

    def jac(x):
        a = np.exp(x)
        return (np.diag(polygamma(1, a)) - polygamma(1, a.sum())) * a[None, :]

    r = root(f, np.log(s0 * m), jac=jac, method="hybr", options={"xtol": 1e-15})
    a = np.exp(r.x)
    res = np.max(np.abs(f(r.x)))
    if not res <= 1e-10 * (1.0 + np.max(np.abs(L))):
        raise ValueError(f"Dirichlet M-step did not converge (residual {res:.3e})")
    return a


def set_params(model, ms):
    """M-step: proposal parameters from mean parameters.

    Gaussian: mean = m1, var = max(m2 - m1^2, floor).  Gamma (moment
    matching): v = max(m2 - m1^2, floor), shape = m1^2 / v, rate = m1 / v.
    Exponential-family Gamma: gap = max(log m1 - m2, floor), shape from
    log shape - psi(shape) = gap, rate = shape / m1.  Dirichlet: an instance
    with 1 - sum_c exp(m2_c) below DIR_GAP_FLOOR has m2 shifted down by a
    constant until the gap is the floor (one hit), then alpha solves
    psi(alpha_c) - psi(alpha_0) = m2_c.
    Returns (params, number of floor hits)."""
    qs, hits = [], 0
    for nd, m in zip(model.nodes, ms):
        m1, m2 = m[..., 0], m[..., 1]
        if nd.qfamily == "dirichlet":
            alpha = np.empty_like(m2)
            for i in range(m2.shape[0]):
                L = m2[i].copy()
                if 1.0 - np.exp(L).sum() < DIR_GAP_FLOOR:
                    hits += 1
                    L = L - (np.log(np.exp(L).sum()) - np.log1p(-DIR_GAP_FLOOR))
                alpha[i] = dirichlet_alpha(L, m1[i])
            qs.append({"alpha": alpha})
            continue
        if nd.qfamily == "bernoulli":
            hits += int(np.sum((m1 < BERN_FLOOR) | (m1 > 1.0 - BERN_FLOOR)))
            qs.append({"p": np.clip(m1, BERN_FLOOR, 1.0 - BERN_FLOOR)})
            continue
        if nd.qfamily == "categorical":
            hits += int(np.sum((m1 < BERN_FLOOR) | (m1 > 1.0)))
            qs.append({"p": np.clip(m1, BERN_FLOOR, 1.0)})
            continue
        if nd.qfamily == "gamma_ef":
            gap = np.log(m1) - m2
            hits += int(np.sum(gap < EF_GAP_FLOOR))
            gap = np.maximum(gap, EF_GAP_FLOOR)
            shape = np.vectorize(ef_gamma_shape)(gap)
            qs.append({"shape": shape, "rate": shape / m1})
            continue
        raw = m2 - m1 * m1
        hits += int(np.sum(raw < VAR_FLOOR))
        v = np.maximum(raw, VAR_FLOOR)
        if nd.qfamily == "gauss":
            qs.append({"mean": m1.copy(), "var": v})
        else:
            qs.append({"shape": m1 * m1 / v, "rate": m1 / v})
    return qs, hits


def sample(model, qs, K: int, it: int, seed: int, node_ids=None):
    """K samples per latent instance: z_v [n, K, d].

    Element e = (i*K + k)*d + j of a Gaussian node takes its normal from the
    Philox block at counter (e >> 1, 0, it, v) (Box-Muller pairs); a Gamma
    node's element uses counters (e, sub, it, v)."""
    zs = []
    for v, (nd, q) in enumerate(zip(model.nodes, qs)):
        if node_ids is not None and v not in node_ids:
            zs.append(None)
            continue
        e = np.arange(nd.n * K * nd.dim, dtype=np.uint64).reshape(nd.n, K, nd.dim)
        if nd.qfamily == "gauss":
            eps = philox.std_normal_paired(e, it, v, seed)
            zs.append(q["mean"][:, None, :] + np.sqrt(q["var"])[:, None, :] * eps)
        elif nd.qfamily == "bernoulli":
            u = philox.uniform_oc(e, np.uint64(0), it, v, seed)
            zs.append((u <= q["p"][:, None, :]).astype(np.float64))
        elif nd.qfamily == "dirichlet":
            zs.append(_dirichlet_draw(q["alpha"][:, None, :], e, it, v, seed))
        elif nd.qfamily == "categorical":
            zs.append(_categorical_draw(q["p"], np.arange(nd.n * K, dtype=np.uint64).reshape(nd.n, K), it, v, seed))
        else:
            g = philox.gamma_unit_rate(q["shape"][:, None, :], e, it, v, seed)
            zs.append(g / q["rate"][:, None, :])
    return zs


def _categorical_draw(p, e, it: int, v: int, seed: int):
    """One-hot categorical samples [n, K, C] for sample counters e [n, K]: the
    first c with u * P_{C-1} <= P_c (P the running sums of p_i, u the (0, 1]
    uniform of counter (e, 0)), else the last category."""
    P = np.cumsum(p, axis=-1)                                   # [n, C]
    u = philox.uniform_oc(e, np.uint64(0), it, v, seed)         # [n, K]
    C = p.shape[-1]
    below = (u[..., None] * P[:, None, -1:]) <= P[:, None, :]   # [n, K, C]
    cat = np.where(below.any(-1), below.argmax(-1), C - 1)
    return np.eye(C)[cat]


def category_of(z):
    """Category index of one-hot samples (last axis)."""
    return np.argmax(z, axis=-1)


def _dirichlet_draw(alpha, e, it: int, v: int, seed: int):
    """Dir(alpha) samples: component c of the sample with elements e normalises
    the Gamma(alpha_c, 1) draws of its C elements, z = softmax(log G); a
    component below FP64's smallest normal is raised to it (as Gamma samples
    are), so log z stays finite."""
    lg = philox.gamma_log_unit_rate(alpha, e, it, v, seed)
    g = np.exp(lg - lg.max(-1, keepdims=True))
    return np.maximum(g / g.sum(-1, keepdims=True), np.finfo(np.float64).tiny)


def sample_instances(model, qs, K: int, it: int, seed: int, v: int, inst):
    """The samples of instances ``inst`` of node v only (same counters as ``sample``)."""
    nd = model.nodes[v]
    q = qs[v]
    inst = np.asarray(inst, dtype=np.uint64)
    e = ((inst[:, None, None] * np.uint64(K) + np.arange(K, dtype=np.uint64)[None, :, None]) * np.uint64(nd.dim)
         + np.arange(nd.dim, dtype=np.uint64)[None, None, :])
    ii = inst.astype(np.int64)
    if nd.qfamily == "gauss":
        eps = philox.std_normal_paired(e, it, v, seed)
        return q["mean"][ii][:, None, :] + np.sqrt(q["var"][ii])[:, None, :] * eps
    if nd.qfamily == "bernoulli":
        u = philox.uniform_oc(e, np.uint64(0), it, v, seed)
        return (u <= q["p"][ii][:, None, :]).astype(np.float64)
    if nd.qfamily == "dirichlet":
        return _dirichlet_draw(q["alpha"][ii][:, None, :], e, it, v, seed)
    if nd.qfamily == "categorical":
        es = inst[:, None] * np.uint64(K) + np.arange(K, dtype=np.uint64)[None, :]
        return _categorical_draw(q["p"][ii], es, it, v, seed)
    g = philox.gamma_unit_rate(q["shape"][ii][:, None, :], e, it, v, seed)
    return g / q["rate"][ii][:, None, :]


# --------------------------------------------------------------------------
# log factors (Eq. rmp split by the latents each term touches)

def _log_q(nd, q, z):
    if nd.qfamily == "gauss":
        return dn.normal(z, q["mean"][:, None, :], q["var"][:, None, :]).sum(-1)
    if nd.qfamily == "bernoulli":
        p = q["p"][:, None, 0]
        with np.errstate(divide="ignore"):   # p = 0 or 1 gives -inf for the impossible value
            return np.where(z[..., 0] == 1.0, np.log(p), np.log1p(-p))
    if nd.qfamily == "dirichlet":
        return dn.dirichlet(z, q["alpha"][:, None, :])
    if nd.qfamily == "categorical":
        p = q["p"] / q["p"].sum(-1, keepdims=True)
        return np.log(np.take_along_axis(p, category_of(z), axis=1))
    return dn.gamma(z[..., 0], q["shape"][:, None, 0], q["rate"][:, None, 0])


def unary(model, qs, zs, K: int) -> List[np.ndarray]:
    """u_v[i, k]: terms touching only instance i of node v, minus log Q, minus log K."""
    us = []
    for v, nd in enumerate(model.nodes):
        z = zs[v]
        u = -_log_q(nd, qs[v], z) - np.log(K)
        if nd.chain_len > 1 and not nd.parents:
            T = nd.chain_len
            first = np.zeros((nd.n // T, T), dtype=bool)
            first[:, 0] = True
            first = first.reshape(-1)
            u = u + np.where(first[:, None], dn.normal(z[..., 0], nd.init_b, nd.init_var), 0.0)
        elif nd.prior == "normal" and not nd.parents:
            u = u + dn.normal(z, nd.b, nd.var).sum(-1)
        elif nd.prior == "gamma":
            u = u + dn.gamma(z[..., 0], nd.shape, nd.rate)
        elif nd.prior == "bernoulli_logit" and not nd.parents:
            u = u + dn.bernoulli_logit(z[..., 0], nd.b)
        elif nd.prior == "dirichlet":
            u = u + dn.dirichlet(z, nd.shape)
        elif nd.prior == "categorical" and not nd.parents:
            u = u - np.log(nd.dim)
        for ob in model.obs:
            if ob.node != v:
                continue
            if ob.kind == "gauss":
                # sum over observations j and dimensions d of log N(x_ijd; z_ikd, var)
                x = ob.x[:, None, :, :]           # [n, 1, J, d]
                u = u + dn.normal(x, z[:, :, None, :], ob.var).sum(axis=(2, 3))
            elif ob.kind == "poisson":
                u = u + dn.poisson(ob.x[:, None, :], z[..., 0][:, :, None]).sum(axis=2)
            elif ob.kind == "detection":
                u = u + dn.detection(ob.x[:, None, :], z[..., 0][:, :, None], ob.var).sum(axis=2)
            elif ob.kind == "categorical":
                u = u + dn.categorical_counts(category_counts(ob, nd.dim)[:, None, :], z)
            elif ob.kind == "gauss_mixture":
                lik = mixture_loglik(ob, nd.dim)                  # [n, C]
                u = u + np.take_along_axis(lik, category_of(z), axis=1)
        us.append(u)
    return us


def pair_table(model, zs, v: int, sl: slice) -> np.ndarray:
    """F_v[i, kp, k] for instances ``sl`` of a node with one factor parent."""
    nd = model.nodes[v]
    (p,) = factor_parents(model, v)
    pidx = nd.parent_index[sl] if nd.parent_index is not None else np.zeros(sl.stop - sl.start, np.int64)
    zc = zs[v][sl][:, None, :, :]                  # [n, 1, K, d]
    zp = zs[p][pidx][:, :, None, :]                # [n, Kp, 1, d]
    F = 0.0
    if p in nd.parents:
        if nd.prior == "normal":
            F = F + dn.normal(zc, nd.a * zp + nd.b, nd.var).sum(-1)
        elif nd.prior == "normal_logscale":
            F = F + dn.normal(zc[..., 0], 0.0, np.exp(2.0 * zp[..., 0]))
        elif nd.prior == "bernoulli_logit":
            F = F + dn.bernoulli_logit(zc[..., 0], nd.a * zp[..., 0] + nd.b)
        elif nd.prior == "categorical":
            # log pi^kp of the child's category: zp [i, kp, 1, C], category [i, 1, k]
            cat = category_of(zc[:, 0])                           # [i, k]
            F = F + np.log(np.take_along_axis(zp[:, :, 0, :], cat[:, None, :].repeat(zp.shape[1], 1), axis=2))
        else:
            raise ValueError(nd.prior)
    for ob in model.obs:
        if ob.node == v and ob.kind == "bernoulli_logit" and ob.coef == p:
            F = F + _bern_table(ob, zs[p], zs[v], sl)
    return np.broadcast_to(F, (sl.stop - sl.start, zs[p].shape[1], zs[v].shape[1])).copy()


def _bern_table(ob, zcoef, zv, sl):
    """sum_j log Bernoulli(y_ij | sigmoid(cov_ij . beta^kb + b_i^k)) as [n, Kb, K]."""
    s = np.einsum("njd,bd->nbj", ob.cov[sl], zcoef[0])          # [n, Kb, J]
    eta = s[:, :, None, :] + zv[sl][:, None, :, 0, None]         # [n, Kb, K, J]
    return dn.bernoulli_logit(ob.x[sl][:, None, None, :], eta).sum(-1)


def triple_table(model, zs, v: int, sl: slice) -> np.ndarray:
    """T_v[i, ka, kb, k] for a node whose two factor parents are roots."""
    nd = model.nodes[v]
    a, b = factor_parents(model, v)
    zv = zs[v][sl][..., 0]                                        # [n, K]
    Ka, Kb = zs[a].shape[1], zs[b].shape[1]
    za = zs[a][0, :, 0][None, :, None, None]
    zb = zs[b][0, :, 0][None, None, :, None]
    if nd.prior == "gamma_parents":
        Tb = dn.gamma(zv[:, None, None, :], za, zb)
    elif nd.prior == "normal_logscale":
        Tb = dn.normal(zv[:, None, None, :], 0.0, np.exp(2.0 * za))
        for ob in model.obs:
            if ob.node == v and ob.kind == "bernoulli_logit":
                assert ob.coef == b
                Tb = Tb + _bern_table(ob, zs[b], zs[v], sl)[:, None, :, :]
    else:
        raise ValueError(nd.prior)
    return np.broadcast_to(Tb, (zv.shape[0], Ka, Kb, zv.shape[1])).copy()


def chainp_tables(model, zs, v: int, series: slice):
    """Factors of a chain under a parent, per parent sample kb:
    init [g, Kb, K] = log N(x_{g,0}^k; beta^kb + init_b, init_var) and
    step [g, Kb, T-1, Kp, K] = log N(x_{g,t}^k; a x_{g,t-1}^kp + (1 - a) beta^kb + b, var)."""
    nd = model.nodes[v]
    (p,) = nd.parents
    T = nd.chain_len
    K = zs[v].shape[1]
    x = zs[v][..., 0].reshape(-1, T, K)[series]                     # [g, T, K]
    ps = nd.parent_index.reshape(-1, T)[series, 0]                   # [g]
    beta = zs[p][ps][..., 0]                                         # [g, Kb]
    init = dn.normal(x[:, None, 0, :], beta[:, :, None] + nd.init_b, nd.init_var)
    mean = nd.a * x[:, None, :-1, :, None] + (1.0 - nd.a) * beta[:, :, None, None, None] + nd.b
    step = dn.normal(x[:, None, 1:, None, :], mean, nd.var)
    return init, step


def chain_table(model, zs, v: int, series: slice) -> np.ndarray:
    """F[g, t-1, kp, k] = log N(z_{g,t}^k; a z_{g,t-1}^kp + b, var), t >= 1."""
    nd = model.nodes[v]
    T = nd.chain_len
    K = zs[v].shape[1]
    z = zs[v][..., 0].reshape(-1, T, K)[series]
    return dn.normal(z[:, 1:, None, :], nd.a * z[:, :-1, :, None] + nd.b, nd.var)


# --------------------------------------------------------------------------
# elimination (forward) and reverse pass

@dataclass
class FwdState:
    ut: List[np.ndarray]                      # u-tilde per node [n, K]
    msg: List[Optional[np.ndarray]]           # m_v: [n, Kp] | [n, Ka, Kb] | chain [G, T, K]
    root_L: Dict[int, np.ndarray] = field(default_factory=dict)   # per-instance root LSE
    chain_L: Dict[int, np.ndarray] = field(default_factory=dict)  # per-series LSE
    pair: Optional[tuple] = None
    M: Optional[np.ndarray] = None            # sum_i m_v[i, ka, kb] over two-parent nodes
    pair_L: float = 0.0
    logphat: float = 0.0


def contract(model, zs, us) -> FwdState:
    """Children-first elimination; returns log P_MP and the saved messages."""
    N = len(model.nodes)
    ut = [u.copy() for u in us]
    st = FwdState(ut=ut, msg=[None] * N)
    st.pair = pair_roots(model)
    for v in reversed(range(N)):
        nd = model.nodes[v]
        fp = factor_parents(model, v)
        K = ut[v].shape[1]
        if nd.chain_len > 1 and fp:
            # once per parent sample kb: u-tilde of the series given kb
            (p,) = fp
            T = nd.chain_len
            G = nd.n // T
            Kb = ut[p].shape[1]
            u3 = ut[v].reshape(G, T, K)
            ub = np.repeat(u3[:, None].copy(), Kb, axis=1)        # [G, Kb, T, K]
            m = np.full((G, Kb, T, K), np.nan)
            for sl in _chunks(G, Kb * T * K * K * 8):
                init, step = chainp_tables(model, zs, v, sl)
                ub[sl, :, 0] += init
                for t in range(T - 1, 0, -1):
                    mt = lse(step[:, :, t - 1] + ub[sl, :, t, None, :], axis=3)
                    m[sl, :, t] = mt
                    ub[sl, :, t - 1] += mt
            L = lse(ub[:, :, 0], axis=2)                        # [G, Kb]: the message to the parent
            st.msg[v] = (m, ub, L)
            ps = nd.parent_index.reshape(G, T)[:, 0]
            for g in range(G):                                    # sequential FP64 accumulation
                ut[p][ps[g]] += L[g]
        elif nd.chain_len > 1:
            T = nd.chain_len
            G = nd.n // T
            u3 = ut[v].reshape(G, T, K)           # view: updates land in ut[v]
            m = np.full((G, T, K), np.nan)
            for sl in _chunks(G, T * K * K * 8):
                F = chain_table(model, zs, v, sl)  # [g, T-1, K, K]
                for t in range(T - 1, 0, -1):
                    mt = lse(F[:, t - 1] + u3[sl, t, None, :], axis=2)
                    m[sl, t] = mt
                    u3[sl, t - 1] += mt
            st.msg[v] = m
            st.chain_L[v] = lse(u3[:, 0], axis=1)
        elif len(fp) == 0:
            if st.pair is not None and v in st.pair:
                continue
            st.root_L[v] = lse(ut[v], axis=1)
        elif len(fp) == 1:
            (p,) = fp
            Kp = ut[p].shape[1]
            m = np.empty((nd.n, Kp))
            sls = list(_chunks(nd.n, Kp * K * 8))
            parts = _map_chunks(lambda sl: lse(pair_table(model, zs, v, sl) + ut[v][sl, None, :], axis=2), sls)
            for sl, part in zip(sls, parts):
                m[sl] = part
            st.msg[v] = m
            pidx = nd.parent_index if nd.parent_index is not None else np.zeros(nd.n, np.int64)
            for i in range(nd.n):                 # sequential FP64 accumulation
                ut[p][pidx[i]] += m[i]
        else:
            a, b = fp
            Ka, Kb = ut[a].shape[1], ut[b].shape[1]
            m = np.empty((nd.n, Ka, Kb))
            sls = list(_chunks(nd.n, Ka * Kb * K * 8))
            parts = _map_chunks(lambda sl: lse(triple_table(model, zs, v, sl) + ut[v][sl, None, None, :], axis=3),
                                sls)
            for sl, part in zip(sls, parts):
                m[sl] = part
            st.msg[v] = m
            acc = np.zeros((Ka, Kb)) if st.M is None else st.M
            for i in range(nd.n):
                acc = acc + m[i]
            st.M = acc
    total = 0.0
    for L in st.root_L.values():
        total += float(np.sum(L))
    for L in st.chain_L.values():
        total += float(np.sum(L))
    if st.pair is not None:
        a, b = st.pair
        J = ut[a][0][:, None] + ut[b][0][None, :] + st.M
        st.pair_L = float(lse(J.reshape(-1), axis=0))
        total += st.pair_L
    st.logphat = total
    return st


def _safe_exp_rows(wpar, X):
    """sum over parent index of wpar * exp(X), treating zero-weight rows as 0."""
    with np.errstate(invalid="ignore", over="ignore"):
        E = np.where(wpar > 0.0, wpar * np.exp(np.where(wpar > 0.0, X, -np.inf)), 0.0)
    return E


def reverse(model, zs, st: FwdState, g: float = 1.0) -> List[np.ndarray]:
    """Parents-first pass: w_v[i, k] = P(k_{v,i} = k), scaled by ``g``.

    Equal to d(g * log P_MP)/d u_v[i, k] (the source-term identity)."""
    N = len(model.nodes)
    ut = st.ut
    w: List[Optional[np.ndarray]] = [None] * N
    W = None
    if st.pair is not None:
        a, b = st.pair
        J = ut[a][0][:, None] + ut[b][0][None, :] + st.M
        W = g * np.exp(J - st.pair_L)
        w[a] = W.sum(axis=1)[None, :]
        w[b] = W.sum(axis=0)[None, :]
    for v in range(N):
        nd = model.nodes[v]
        fp = factor_parents(model, v)
        K = ut[v].shape[1]
        if nd.chain_len > 1 and fp:
            (p,) = fp
            T = nd.chain_len
            G = nd.n // T
            m, ub, L = st.msg[v]
            Kb = ub.shape[1]
            ps = nd.parent_index.reshape(G, T)[:, 0]
            wv = np.zeros((G, T, K))
            for sl in _chunks(G, Kb * T * K * K * 8):
                _, step = chainp_tables(model, zs, v, sl)
                for kb in range(Kb):                              # weights given kb, summed in kb order
                    wk = np.zeros((sl.stop - sl.start, T, K))
                    wk[:, 0] = w[p][ps[sl], kb][:, None] * np.exp(ub[sl, kb, 0] - L[sl, kb][:, None])
                    for t in range(1, T):
                        X = step[:, kb, t - 1] + ub[sl, kb, t, None, :] - m[sl, kb, t][:, :, None]
                        wk[:, t] = _safe_exp_rows(wk[:, t - 1][:, :, None], X).sum(axis=1)
                    wv[sl] += wk
            w[v] = wv.reshape(nd.n, K)
        elif nd.chain_len > 1:
            T = nd.chain_len
            G = nd.n // T
            u3 = ut[v].reshape(G, T, K)
            m = st.msg[v]
            wv = np.zeros((G, T, K))
            wv[:, 0] = g * np.exp(u3[:, 0] - st.chain_L[v][:, None])
            for sl in _chunks(G, T * K * K * 8):
                F = chain_table(model, zs, v, sl)
                for t in range(1, T):
                    X = F[:, t - 1] + u3[sl, t, None, :] - m[sl, t][:, :, None]
                    wv[sl, t] = _safe_exp_rows(wv[sl, t - 1][:, :, None], X).sum(axis=1)
            w[v] = wv.reshape(nd.n, K)
        elif len(fp) == 0:
            if w[v] is None:
                w[v] = g * np.exp(ut[v] - st.root_L[v][:, None])
        elif len(fp) == 1:
            (p,) = fp
            pidx = nd.parent_index if nd.parent_index is not None else np.zeros(nd.n, np.int64)
            wv = np.empty((nd.n, K))

            def pair_rows(sl, v=v, p=p, pidx=pidx):
                X = pair_table(model, zs, v, sl) + ut[v][sl, None, :] - st.msg[v][sl][:, :, None]
                return _safe_exp_rows(w[p][pidx[sl]][:, :, None], X).sum(axis=1)
            sls = list(_chunks(nd.n, ut[p].shape[1] * K * 8))
            for sl, part in zip(sls, _map_chunks(pair_rows, sls)):
                wv[sl] = part
            w[v] = wv
        else:
            wv = np.empty((nd.n, K))

            def triple_rows(sl, v=v):
                X = triple_table(model, zs, v, sl) + ut[v][sl, None, None, :] - st.msg[v][sl][..., None]
                return _safe_exp_rows(W[None, :, :, None], X).sum(axis=(1, 2))
            sls = list(_chunks(nd.n, W.size * K * 8))
            for sl, part in zip(sls, _map_chunks(triple_rows, sls)):
                wv[sl] = part
            w[v] = wv
    return w


def mixture_loglik(ob, C: int) -> np.ndarray:
    """lik[i, c] = sum_j log N(y_ij; mu_c, var): the Gaussian-mixture
    observations of instance i if its category is c (mu = ob.cov)."""
    mu = np.asarray(ob.cov, dtype=np.float64).reshape(C)
    return dn.normal(ob.x[:, :, None], mu[None, None, :], ob.var).sum(1)


def category_counts(ob, C: int) -> np.ndarray:
    """Per-instance counts [n, C] of categorical observations x [n, n_per]
    (entries outside 0..C-1 are not counted)."""
    x = np.asarray(ob.x, dtype=np.float64)
    return np.stack([(x == c).sum(-1) for c in range(C)], axis=-1).astype(np.float64)


def moments(zs, ws, model=None) -> List[np.ndarray]:
    """m_one_v[i, j] = sum_k w_v[i, k] (z, z^2) (Eq. mmp with m = T(z));
    sum_k w (z, log z) for exponential-family Gamma and Dirichlet nodes of
    `model`."""
    out = []
    for v, (z, w) in enumerate(zip(zs, ws)):
        ef = model is not None and model.nodes[v].qfamily in ("gamma_ef", "dirichlet")
        out.append(np.stack([np.einsum("nk,nkd->nd", w, z),
                             np.einsum("nk,nkd->nd", w, np.log(z) if ef else z * z)], axis=-1))
    return out


def ema(m_prev, m_one, lam: float):
    """Eq. ema: m_t = (1 - lam) m_{t-1} + lam m_one_t."""
    return [(1.0 - lam) * a + lam * b for a, b in zip(m_prev, m_one)]


def ess(ws):
    """Marginal effective sample size per latent instance, 1 / sum_k w^2."""
    return [1.0 / np.sum(w * w, axis=1) for w in ws]


# --------------------------------------------------------------------------
# the E-step and the QEM loop (Algorithm 1)

def estep(model, qs, zs, K: int):
    us = unary(model, qs, zs, K)
    st = contract(model, zs, us)
    ws = reverse(model, zs, st)
    return st, ws, moments(zs, ws, model)


SECOND_SAMPLE_STREAM = 0x80000000   # Philox iteration word of the second sample: t XOR this


def ema_step(lam: float, p: float, t: int) -> float:
    """Weight of the new estimate at iteration t >= 1: lam (Eq. ema), or, for
    0 < p < 1, the decreasing step t^-p of Theorem 1 (whose weight on the
    previous estimate is 1 - t^-p)."""
    return float(t) ** (-p) if p > 0.0 else lam


def logphat_forward(model, qs, zs, K: int) -> float:
    """log P_MP of one sample (Eq. Prmp), forward elimination only."""
    return contract(model, zs, unary(model, qs, zs, K)).logphat


def qem(model, K: int, iters: int, lam: float, seed: int, m0=None, record=None, p: float = 0.0,
        second_sample: bool = False):
    """Algorithm 1.  Returns (final mean parameters, log P_MP per iteration).

    p > 0 replaces lam by the schedule of Theorem 1 (ema_step).  With
    second_sample the moment estimate of sample z is rescaled by
    P_MP(z) / P_MP(z_new), z_new a second, independent draw from the same Q_t
    (Philox iteration word t XOR SECOND_SAMPLE_STREAM): the unnormalised
    estimate K^-n sum_k r_k m(z^k) = P_MP(z) sum_k w_k m(z^k) divided by
    P_MP(z_new) instead of P_MP(z) (the variant discussed after Theorem 1).
    An iteration whose log P_MP (either one) is not finite keeps m_{t-1}."""
    q0 = q_init(model)
    m = mean_params(model, q0) if m0 is None else [x.copy() for x in m0]
    hist = []
    for t in range(1, iters + 1):
        # the first sample is drawn from Q_0 itself (its parameters, not their
        # round trip through the mean parameters: a Gamma or Dirichlet shape of
        # exactly 1 must not come back as 1 - 1e-16, which changes the draw)
        qs = q0 if (t == 1 and m0 is None) else set_params(model, m)[0]
        zs = sample(model, qs, K, t, seed)
        st, ws, m_one = estep(model, qs, zs, K)
        hist.append(st.logphat)
        ok = np.isfinite(st.logphat)
        if second_sample:
            lp_new = logphat_forward(model, qs, sample(model, qs, K, t ^ SECOND_SAMPLE_STREAM, seed), K)
            ok = ok and np.isfinite(lp_new)
            if ok:
                rho = np.exp(st.logphat - lp_new)
                m_one = [rho * x for x in m_one]
        if ok:
            m = ema(m, m_one, ema_step(lam, p, t))
        if record is not None:
            record.append(dict(t=t, logphat=st.logphat, m=[x.copy() for x in m]))
    return m, np.array(hist)


# --------------------------------------------------------------------------
# brute-force enumeration over all K^n index tuples (tiny models only)

def _instances(model):
    out = []
    for v, nd in enumerate(model.nodes):
        for i in range(nd.n):
            out.append((v, i))
    return out


def brute_force_tables(model, zs, us):
    """Eq. mp_iw by enumeration, building log r_k from the factor tables.

    Returns (log P_MP, weights per node)."""
    inst = _instances(model)
    n = len(inst)
    K = us[0].shape[1]
    pos = {vi: a for a, vi in enumerate(inst)}
    logr = np.zeros([K] * n)

    def add(table, axes):
        shape = [1] * n
        for ax in axes:
            shape[ax] = K
        order = np.argsort(axes)
        t = np.transpose(table, order).reshape([K if a in axes else 1 for a in range(n)])
        return t

    for v, nd in enumerate(model.nodes):
        fp = factor_parents(model, v)
        for i in range(nd.n):
            logr = logr + add(us[v][i], [pos[(v, i)]])
            if nd.chain_len > 1 and fp:
                (p,) = fp
                T = nd.chain_len
                g, t = divmod(i, T)
                pi = int(nd.parent_index[i])
                init, step = chainp_tables(model, zs, v, slice(g, g + 1))
                if t == 0:
                    logr = logr + add(init[0], [pos[(p, pi)], pos[(v, i)]])
                else:
                    logr = logr + add(step[0, :, t - 1], [pos[(p, pi)], pos[(v, i - 1)], pos[(v, i)]])
            elif nd.chain_len > 1 and i % nd.chain_len != 0:
                T = nd.chain_len
                g, t = divmod(i, T)
                F = chain_table(model, zs, v, slice(g, g + 1))[0, t - 1]
                logr = logr + add(F, [pos[(v, i - 1)], pos[(v, i)]])
            elif len(fp) == 1:
                p = fp[0]
                pi = int(nd.parent_index[i]) if nd.parent_index is not None else 0
                F = pair_table(model, zs, v, slice(i, i + 1))[0]
                logr = logr + add(F, [pos[(p, pi)], pos[(v, i)]])
            elif len(fp) == 2:
                a, b = fp
                Tb = triple_table(model, zs, v, slice(i, i + 1))[0]
                logr = logr + add(Tb, [pos[(a, 0)], pos[(b, 0)], pos[(v, i)]])
    L = lse(logr.reshape(-1), axis=0)
    R = np.exp(logr - L)
    ws = [np.zeros((nd.n, K)) for nd in model.nodes]
    for a, (v, i) in enumerate(inst):
        ws[v][i] = R.sum(axis=tuple(x for x in range(n) if x != a))
    return float(L), ws


def log_joint_direct(model, zsel):
    """log P(x, z) for C joint configurations, by walking the generative model.

    ``zsel[v]`` is [C, n, d].  Independent of the factor-table split."""
    C = zsel[0].shape[0]
    lp = np.zeros(C)
    for v, nd in enumerate(model.nodes):
        z = zsel[v]
        if nd.chain_len > 1:
            T = nd.chain_len
            zz = z[..., 0].reshape(C, -1, T)
            if nd.parents:
                # AR(1) around the parent's level beta of each series
                beta = zsel[nd.parents[0]][:, nd.parent_index.reshape(-1, T)[:, 0], 0]   # [C, G]
                lp += dn.normal(zz[:, :, 0], beta + nd.init_b, nd.init_var).sum(1)
                lp += dn.normal(zz[:, :, 1:], nd.a * zz[:, :, :-1] + (1.0 - nd.a) * beta[:, :, None] + nd.b,
                                nd.var).sum((1, 2))
            else:
                lp += dn.normal(zz[:, :, 0], nd.init_b, nd.init_var).sum(1)
                lp += dn.normal(zz[:, :, 1:], nd.a * zz[:, :, :-1] + nd.b, nd.var).sum((1, 2))
        elif nd.prior == "normal":
            if nd.parents:
                zp = zsel[nd.parents[0]][:, nd.parent_index, :]
                lp += dn.normal(z, nd.a * zp + nd.b, nd.var).sum((1, 2))
            else:
                lp += dn.normal(z, nd.b, nd.var).sum((1, 2))
        elif nd.prior == "gamma":
            lp += dn.gamma(z, nd.shape, nd.rate).sum((1, 2))
        elif nd.prior == "gamma_parents":
            sa = zsel[nd.parents[0]][:, 0:1, 0]
            rb = zsel[nd.parents[1]][:, 0:1, 0]
            lp += dn.gamma(z[..., 0], sa, rb).sum(1)
        elif nd.prior == "normal_logscale":
            ls = zsel[nd.parents[0]][:, 0:1, 0]
            lp += dn.normal(z[..., 0], 0.0, np.exp(2.0 * ls)).sum(1)
        elif nd.prior == "dirichlet":
            lp += dn.dirichlet(z, nd.shape).sum(1)
        elif nd.prior == "categorical":
            # the category's probability: pi of the parent instance, or 1 / C
            cat = np.argmax(z, axis=-1)                           # [C_conf, n]
            if nd.parents:
                pi = zsel[nd.parents[0]][:, nd.parent_index, :]   # [C_conf, n, C]
                lp += np.log(np.take_along_axis(pi, cat[..., None], axis=2)[..., 0]).sum(1)
            else:
                lp += -np.log(nd.dim) * z.shape[1]
        elif nd.prior == "bernoulli_logit":
            # P(z = 1) = 1 / (1 + exp(-eta)), P(z = 0) = 1 - P(z = 1)
            if nd.parents:
                eta = nd.a * zsel[nd.parents[0]][:, nd.parent_index, 0] + nd.b
            else:
                eta = np.full(z.shape[:2], nd.b)
            p1 = 1.0 / (1.0 + np.exp(-eta))
            lp += np.log(np.where(z[..., 0] == 1.0, p1, 1.0 - p1)).sum(1)
    for ob in model.obs:
        z = zsel[ob.node]
        if ob.kind == "gauss":
            lp += dn.normal(ob.x[None], z[:, :, None, :], ob.var).sum((1, 2, 3))
        elif ob.kind == "poisson":
            lp += dn.poisson(ob.x[None], z[:, :, 0:1]).sum((1, 2))
        elif ob.kind == "bernoulli_logit":
            beta = zsel[ob.coef][:, 0, :]                         # [C, D]
            eta = np.einsum("njd,cd->cnj", ob.cov, beta) + z[:, :, 0:1]
            lp += dn.bernoulli_logit(ob.x[None], eta).sum((1, 2))
        elif ob.kind == "detection":
            # each visit detects with probability p z
            pz = ob.var * z[:, :, 0:1]
            with np.errstate(divide="ignore"):
                lp += np.log(np.prod(np.where(ob.x[None] == 1.0, pz, 1.0 - pz), axis=2)).sum(1)
        elif ob.kind == "gauss_mixture":
            mu = np.asarray(ob.cov, dtype=np.float64).reshape(-1)[np.argmax(z, axis=-1)]   # [C_conf, n]
            lp += dn.normal(ob.x[None], mu[:, :, None], ob.var).sum((1, 2))
        elif ob.kind == "categorical":
            # the probability of each observed category, draw by draw
            idx = ob.x.astype(np.int64)                           # [n, J]
            lp += np.log(np.take_along_axis(z, np.broadcast_to(idx[None], (C,) + idx.shape), axis=2)).sum((1, 2))
    return lp


def log_q_direct(model, qs, zsel):
    C = zsel[0].shape[0]
    lq = np.zeros(C)
    for nd, q, z in zip(model.nodes, qs, zsel):
        if nd.qfamily == "gauss":
            lq += dn.normal(z, q["mean"][None], q["var"][None]).sum((1, 2))
        elif nd.qfamily == "bernoulli":
            lq += np.log(np.where(z[..., 0] == 1.0, q["p"][None, :, 0], 1.0 - q["p"][None, :, 0])).sum(1)
        elif nd.qfamily == "dirichlet":
            lq += dn.dirichlet(z, q["alpha"][None]).sum(1)
        elif nd.qfamily == "categorical":
            p = q["p"] / q["p"].sum(-1, keepdims=True)            # [n, C]
            lq += np.log((z * p[None]).sum(-1)).sum(1)
        else:
            lq += dn.gamma(z[..., 0], q["shape"][None, :, 0], q["rate"][None, :, 0]).sum(1)
    return lq


def brute_force_direct(model, qs, zs, chunk: int = 1 << 16):
    """Eq. mp_iw by enumerating every tuple and evaluating r_k from the
    joint density and the proposal density directly.

    Returns (log P_MP, weights per node, moments per node)."""
    inst = _instances(model)
    n = len(inst)
    K = zs[0].shape[1]
    total = K ** n
    logr_all = np.empty(total)
    for s in range(0, total, chunk):
        idx = np.arange(s, min(total, s + chunk))
        digits = np.stack([(idx // K ** (n - 1 - a)) % K for a in range(n)], axis=1)
        zsel = [np.empty((len(idx), nd.n, nd.dim)) for nd in model.nodes]
        for a, (v, i) in enumerate(inst):
            zsel[v][:, i, :] = zs[v][i][digits[:, a]]
        logr_all[s:s + len(idx)] = log_joint_direct(model, zsel) - log_q_direct(model, qs, zsel)
    L = lse(logr_all, axis=0)
    logphat = float(L - n * np.log(K))
    R = np.exp(logr_all - L).reshape([K] * n)
    ws = [np.zeros((nd.n, K)) for nd in model.nodes]
    for a, (v, i) in enumerate(inst):
        ws[v][i] = R.sum(axis=tuple(x for x in range(n) if x != a))
    return logphat, ws, moments(zs, ws)
