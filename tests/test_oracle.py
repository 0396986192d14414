"""Pins for the CPU oracle: it is checked against things other than itself.

* Philox4x32-10 against the published known-answer vectors.
* Sampler output distributions against scipy's CDFs (KS tests).
* Elimination (contract/reverse) against brute-force enumeration of all K^n
  tuples, with r_k evaluated directly from the generative model (Eq. mp_iw).
* Special cases: K = 1 (a single importance weight, Eq. rglobal with K = 1);
  a proposal equal to the exact conjugate posterior (every r_k equals P(x));
  sum_k w = 1; d log P_MP / d u = w (source-term identity, finite differences).
* Chains against the textbook HMM forward-backward recursion.
* Gaussian models against closed-form posteriors (Gaussian conditioning,
  Kalman filter / RTS smoother) as K grows, and E[P_MP] = P(x).
* Reparameterisation invariance (paper appendix E).
"""
import numpy as np
import pytest
from scipy import stats
from scipy.special import digamma, gammaln

import qem_synth as S
from oracle import mpiw as M
from oracle import philox

GOLDEN = __file__.replace("test_oracle.py", "golden/")


def _estep(model, K, seed=11, it=1, qs=None):
    qs = M.q_init(model) if qs is None else qs
    zs = M.sample(model, qs, K, it, seed)
    us = M.unary(model, qs, zs, K)
    st = M.contract(model, zs, us)
    ws = M.reverse(model, zs, st)
    return qs, zs, us, st, ws


def _tiny_occupancy():
    """A global occupancy logit and three sites, one of them detected."""
    m = S.occupancy(5, n_sites=3, n_visits=3, K=3)
    m.obs[0].x[:] = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    return m


TINY = [
    lambda: S.mixture(7, n_groups=3, C=3, n_obs=2, K=3),
    lambda: S.dirichlet_categorical(6, n_groups=2, C=3, n_obs=5, shape=0.8, K=4),
    lambda: S.ar_regions(3, n_regions=2, T=3, K=3),
    _tiny_occupancy,
    lambda: S.tiny_tree(0, K=3),
    lambda: S.normal_normal(1, n_groups=3, n_obs=2, K=3),
    lambda: S.chain(2, n_series=2, T=3, K=3),
    lambda: S.gamma_poisson(3, n_groups=2, n_obs=5, K=3),
    lambda: S.logistic(4, n_groups=2, n_obs=4, D=2, K=3),
]


# ---------------------------------------------------------------- Philox / samplers

def test_philox_known_answers():
    for line in open(GOLDEN + "philox4x32_10_kat.txt"):
        if line.startswith("#") or not line.strip():
            continue
        cols = line.split()
        f = [int(cols[0])] + [int(x, 16) for x in cols[1:]]
        assert f[0] == 10
        out = philox.philox4x32_10(*[np.array([c], np.uint64) for c in f[1:5]], f[5], f[6])
        assert [int(o[0]) for o in out] == f[7:11]


def test_normal_sampler_distribution():
    e = np.arange(200000, dtype=np.uint64)
    x = philox.std_normal(e, 0, 5, 2, 1234)
    assert stats.kstest(x, "norm").pvalue > 1e-3
    # different counters give different, uncorrelated streams
    y = philox.std_normal(e, 0, 6, 2, 1234)
    assert abs(np.corrcoef(x, y)[0, 1]) < 0.01


def test_paired_normal_sampler():
    """Both Box-Muller branches are N(0, 1), the two members of a pair are
    uncorrelated, and together they recover the radius: x_2p^2 + x_2p+1^2 =
    -2 log u1 of their shared block; the even member equals the cosine-branch
    normal of the same block."""
    e = np.arange(200000, dtype=np.uint64)
    x = philox.std_normal_paired(e, 5, 2, 1234)
    even, odd = x[0::2], x[1::2]
    assert stats.kstest(even, "norm").pvalue > 1e-3
    assert stats.kstest(odd, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(even, odd)[0, 1]) < 0.01
    p = np.arange(100000, dtype=np.uint64)
    np.testing.assert_array_equal(even, philox.std_normal(p, 0, 5, 2, 1234))
    k0, k1 = 1234, 0
    r0, r1, _, _ = philox.philox4x32_10(p, 0, 5, 2, k0, k1)
    u1 = (((r0.astype(np.uint64) << np.uint64(32)) | r1.astype(np.uint64)) >> np.uint64(11)).astype(np.float64)
    u1 = (u1 + 1.0) * 2.0 ** -53
    np.testing.assert_allclose(even ** 2 + odd ** 2, -2.0 * np.log(u1), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("shape", [0.3, 1.0, 2.5, 40.0])
def test_gamma_sampler_distribution(shape):
    e = np.arange(100000, dtype=np.uint64)
    g = philox.gamma_unit_rate(shape, e, 3, 1, 99)
    assert stats.kstest(g, stats.gamma(shape).cdf).pvalue > 1e-3


def test_samples_are_counter_based():
    m = S.nested_gaussian(0, n_schools=3, n_classes=2, n_students=2, dim=3, K=5)
    qs = M.q_init(m)
    a = M.sample(m, qs, 5, 7, 42)
    b = M.sample(m, qs, 5, 7, 42)
    c = M.sample(m, qs, 5, 8, 42)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y)
        assert not np.allclose(x, z)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("mk", TINY)
def test_elimination_equals_brute_force(mk):
    model = mk()
    qs, zs, us, st, ws = _estep(model, model.K)
    L, wb, mb = M.brute_force_direct(model, qs, zs)
    assert abs(st.logphat - L) <= 1e-12 * max(1.0, abs(L))
    for a, b in zip(ws, wb):
        np.testing.assert_allclose(a, b, atol=1e-13)
    for a, b in zip(M.moments(zs, ws), mb):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("mk", TINY)
def test_factor_tables_equal_direct_joint(mk):
    model = mk()
    qs, zs, us, st, ws = _estep(model, model.K, seed=5)
    L1, w1 = M.brute_force_tables(model, zs, us)
    L2, w2, _ = M.brute_force_direct(model, qs, zs)
    assert abs(L1 - L2) <= 1e-12 * max(1.0, abs(L2))


def test_normal_normal_K8_brute_force():
    """The 2-level normal-normal model (8 groups) at K = 8: all 8^9 tuples."""
    model = S.normal_normal(0)
    qs, zs, us, st, ws = _estep(model, 8, seed=17)
    L, wb = M.brute_force_tables(model, zs, us)
    assert abs(st.logphat - L) <= 1e-11 * abs(L)
    for a, b in zip(ws, wb):
        np.testing.assert_allclose(a, b, atol=1e-12)


# ---------------------------------------------------------------- special cases

def test_K1_is_single_importance_weight():
    model = S.normal_normal(2)
    qs, zs, us, st, ws = _estep(model, 1, seed=3)
    mu, z = zs[0][0, 0, 0], zs[1][:, 0, 0]
    x = model.obs[0].x[:, :, 0]
    logp = (stats.norm(0, 1).logpdf(mu) + stats.norm(mu, 1).logpdf(z).sum()
            + stats.norm(z[:, None], 0.5).logpdf(x).sum())
    logq = stats.norm(0, 1).logpdf(mu) + stats.norm(0, 1).logpdf(z).sum()
    assert abs(st.logphat - (logp - logq)) < 1e-12 * abs(logp)
    for w in ws:
        np.testing.assert_allclose(w, 1.0, atol=1e-15)
    m = M.moments(zs, ws)
    np.testing.assert_allclose(m[1][:, 0, 0], z, atol=1e-15)
    np.testing.assert_allclose(m[1][:, 0, 1], z * z, atol=1e-14)


def test_K1_gamma_poisson_shape_rate_roles():
    """K = 1 on the Gamma-Poisson hierarchy: log P_MP = log P(y, z) - log Q(z)
    with every density taken from scipy in its own parameterisation, so the
    roles of the two parents (alpha the shape, beta the rate of lambda_i) are
    pinned: Gamma(shape a, rate b) is scipy's gamma(a, scale=1/b)."""
    model = S.gamma_poisson(5, n_groups=6, n_obs=9)
    qs, zs, us, st, ws = _estep(model, 1, seed=13)
    al, be, lam = zs[0][0, 0, 0], zs[1][0, 0, 0], zs[2][:, 0, 0]
    y = model.obs[0].x
    # the two parents have distinct values, so exchanging their roles is seen
    assert abs(al - be) > 0.05
    logp = (stats.gamma(2.0, scale=1.0).logpdf(al) + stats.gamma(2.0, scale=1.0).logpdf(be)
            + stats.gamma(al, scale=1.0 / be).logpdf(lam).sum()
            + stats.poisson(lam[:, None]).logpmf(y).sum())
    logq = (stats.gamma(2.0, scale=1.0).logpdf(al) + stats.gamma(2.0, scale=1.0).logpdf(be)
            + stats.gamma(2.0, scale=1.0).logpdf(lam).sum())
    assert abs(st.logphat - (logp - logq)) < 1e-12 * abs(logp)
    # the same sample under the swapped reading gives a different value
    swapped = logp - stats.gamma(al, scale=1.0 / be).logpdf(lam).sum() + stats.gamma(be, scale=1.0 / al).logpdf(lam).sum()
    assert abs(swapped - logp) > 1e-3
    for w in ws:
        np.testing.assert_allclose(w, 1.0, atol=1e-15)
    m = M.moments(zs, ws, model)
    np.testing.assert_allclose(m[2][:, 0, 0], lam, rtol=1e-15)


def test_K1_logistic_scale_convention():
    """K = 1 on the mixed-effects logistic model: b_i ~ N(0, sigma^2) with
    sigma = exp(log sigma) (scipy's norm(0, scale=sigma)), and
    y_ij ~ Bernoulli(sigmoid(cov_ij . beta + b_i)) (scipy's bernoulli)."""
    from scipy.special import expit
    model = S.logistic(6, n_groups=5, n_obs=7, D=3)
    qs, zs, us, st, ws = _estep(model, 1, seed=19)
    beta, ls, b = zs[0][0, 0, :], zs[1][0, 0, 0], zs[2][:, 0, 0]
    # a log-scale away from 0, so sigma and sigma^2 differ
    assert abs(ls) > 0.05
    ob = model.obs[0]
    eta = ob.cov @ beta + b[:, None]
    logp = (stats.norm(0.0, 1.0).logpdf(beta).sum() + stats.norm(0.0, 1.0).logpdf(ls)
            + stats.norm(0.0, np.exp(ls)).logpdf(b).sum()
            + stats.bernoulli(expit(eta)).logpmf(ob.x).sum())
    logq = (stats.norm(0.0, 1.0).logpdf(beta).sum() + stats.norm(0.0, 1.0).logpdf(ls)
            + stats.norm(0.0, 1.0).logpdf(b).sum())
    assert abs(st.logphat - (logp - logq)) < 1e-12 * abs(logp)
    wrong = logp - stats.norm(0.0, np.exp(ls)).logpdf(b).sum() + stats.norm(0.0, np.exp(0.5 * ls)).logpdf(b).sum()
    assert abs(wrong - logp) > 1e-3
    for w in ws:
        np.testing.assert_allclose(w, 1.0, atol=1e-15)


def test_synthetic_generators_follow_the_stated_parameterisations():
    """The generators draw lambda_i ~ Gamma(shape alpha, rate beta) and
    b_i ~ N(0, exp(log sigma)^2): sample moments of a large draw agree."""
    gp = S.gamma_poisson(2, n_groups=200000, n_obs=1)
    al, be = gp.truth[0][0, 0], gp.truth[1][0, 0]
    lam = gp.truth[2][:, 0]
    assert abs(lam.mean() - al / be) < 4 * np.sqrt(al) / be / np.sqrt(lam.size)
    assert abs(lam.var() / (al / be ** 2) - 1.0) < 0.03
    lg = S.logistic(3, n_groups=200000, n_obs=1, D=2)
    ls = lg.truth[1][0, 0]
    b = lg.truth[2][:, 0]
    assert abs(b.std() / np.exp(ls) - 1.0) < 0.01


def _gp_roots(seed, n, J, a0, b0):
    """Independent lambda_i ~ Gamma(a0, b0), y_ij ~ Poisson(lambda_i)."""
    src = S.gamma_poisson(seed, n_groups=n, n_obs=J)
    node = S.Node("lambda", n, 1, "gamma", "gamma", shape=a0, rate=b0, q0=(2.0, 1.0))
    return S.Model("gp_roots", [node], [S.Obs(0, "poisson", src.obs[0].x)], K=64)


def test_exact_posterior_proposal_gamma_poisson():
    """With Q equal to the conjugate posterior Gamma(a0 + sum y, b0 + J),
    every r_k equals P(y), so log P_MP is the closed-form evidence for any K."""
    a0, b0, J = 2.0, 1.5, 20
    model = _gp_roots(7, 5, J, a0, b0)
    y = model.obs[0].x
    sy = y.sum(1)
    qs = [{"shape": (a0 + sy)[:, None], "rate": np.full((5, 1), b0 + J)}]
    _, zs, us, st, ws = _estep(model, 16, qs=qs)
    logev = (a0 * np.log(b0) - gammaln(a0) + gammaln(a0 + sy) - (a0 + sy) * np.log(b0 + J)
             - gammaln(y + 1).sum(1))
    assert abs(st.logphat - logev.sum()) < 1e-11 * abs(logev.sum())
    np.testing.assert_allclose(ws[0], 1.0 / 16, atol=1e-13)


def test_exact_posterior_proposal_gaussian():
    """Single Gaussian latent with Gaussian observations and Q = exact posterior."""
    src = S.normal_normal(4, n_groups=3, n_obs=6)
    node = S.Node("theta", 3, 1, "gauss", "normal", b=0.3, var=2.0)
    model = S.Model("nn_roots", [node], [S.Obs(0, "gauss", src.obs[0].x, var=0.25)], K=8)
    x = src.obs[0].x[:, :, 0]
    prec = 1 / 2.0 + 6 / 0.25
    mean = (0.3 / 2.0 + x.sum(1) / 0.25) / prec
    qs = [{"mean": mean[:, None], "var": np.full((3, 1), 1 / prec)}]
    _, zs, us, st, ws = _estep(model, 8, qs=qs)
    logev = sum(stats.multivariate_normal(np.full(6, 0.3), 2.0 + 0.25 * np.eye(6)).logpdf(x[i])
                for i in range(3))
    assert abs(st.logphat - logev) < 1e-11 * abs(logev)


@pytest.mark.parametrize("mk", TINY + [lambda: S.nested_gaussian(0, 4, 3, 2, 2, K=6)])
def test_weights_sum_to_one(mk):
    model = mk()
    _, _, _, _, ws = _estep(model, model.K, seed=21)
    for w in ws:
        np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-12)
        assert (w >= 0).all()


@pytest.mark.parametrize("mk", TINY)
def test_finite_difference_adjoint(mk):
    """d log P_MP / d u_v[i,k] = w_v[i,k] (source-term identity)."""
    model = mk()
    qs, zs, us, st, ws = _estep(model, model.K, seed=8)
    h = 1e-6
    rng = np.random.default_rng(0)
    for v in range(len(us)):
        for _ in range(3):
            i = rng.integers(us[v].shape[0])
            k = rng.integers(us[v].shape[1])
            up = [u.copy() for u in us]
            dn_ = [u.copy() for u in us]
            up[v][i, k] += h
            dn_[v][i, k] -= h
            fd = (M.contract(model, zs, up).logphat - M.contract(model, zs, dn_).logphat) / (2 * h)
            assert abs(fd - ws[v][i, k]) < 1e-6


# ---------------------------------------------------------------- chains

def test_chain_matches_hmm_forward_backward():
    """Textbook scaled forward-backward with K states per step on the same
    factor tables: forward alpha from t = 0, backward beta from t = T-1."""
    model = S.chain(5, n_series=3, T=7, K=5)
    qs, zs, us, st, ws = _estep(model, 5, seed=13)
    T, K = 7, 5
    F = M.chain_table(model, zs, 0, slice(0, 3))
    U = us[0].reshape(3, T, K)
    W = ws[0].reshape(3, T, K)
    total = 0.0
    for g in range(3):
        E = np.exp(F[g])                         # [T-1, K, K]
        e = np.exp(U[g])
        alpha = np.zeros((T, K))
        c = np.zeros(T)
        a = e[0]
        c[0] = a.sum()
        alpha[0] = a / c[0]
        for t in range(1, T):
            a = (alpha[t - 1] @ E[t - 1]) * e[t]
            c[t] = a.sum()
            alpha[t] = a / c[t]
        beta = np.ones((T, K))
        for t in range(T - 2, -1, -1):
            beta[t] = E[t] @ (e[t + 1] * beta[t + 1]) / c[t + 1]
        post = alpha * beta
        np.testing.assert_allclose(W[g], post, atol=1e-12)
        total += np.log(c).sum()
    assert abs(st.logphat - total) < 1e-11 * abs(total)


# ---------------------------------------------------------------- Gaussian closed forms

def _normal_normal_posterior(model):
    """Exact Gaussian posterior over (mu, z_1..z_n) by Gaussian conditioning."""
    n = model.nodes[1].n
    x = model.obs[0].x[:, :, 0]
    J = x.shape[1]
    # prior: mu ~ N(0,1), z_i = mu + e_i, e_i ~ N(0,1)
    A = np.zeros((n + 1, n + 1))
    A[:, 0] = 1.0
    A[1:, 1:] = np.eye(n)
    S0 = A @ A.T
    # observations: x_ij = z_i + noise(0.25)
    H = np.zeros((n * J, n + 1))
    for i in range(n):
        H[i * J:(i + 1) * J, i + 1] = 1.0
    R = 0.25 * np.eye(n * J)
    Sx = H @ S0 @ H.T + R
    G = S0 @ H.T @ np.linalg.inv(Sx)
    mean = G @ x.reshape(-1)
    cov = S0 - G @ H @ S0
    logev = stats.multivariate_normal(np.zeros(n * J), Sx).logpdf(x.reshape(-1))
    return mean, np.diag(cov), logev


def test_unbiased_marginal_likelihood():
    """E[P_MP] = P(x) (paper section 3.2), Monte Carlo over sample seeds."""
    model = S.normal_normal(6, n_groups=2, n_obs=2, K=8)
    _, _, logev = _normal_normal_posterior(model)
    r = []
    for s in range(1500):
        _, _, _, st, _ = _estep(model, 8, seed=1000 + s)
        r.append(np.exp(st.logphat - logev))
    r = np.array(r)
    se = r.std() / np.sqrt(len(r))
    assert abs(r.mean() - 1.0) < 4 * se + 1e-3


def test_qem_approaches_closed_form_posterior():
    """QEM's fixed point approaches the exact posterior moments as K grows
    (paper appendix C); the error shrinks from K = 8 to K = 256."""
    model = S.normal_normal(0)
    mean, var, _ = _normal_normal_posterior(model)
    errs = []
    for K in (8, 256):
        m, hist = M.qem(model, K, 30, 0.3, seed=77)
        m1 = np.concatenate([m[0][:, 0, 0], m[1][:, 0, 0]])
        v = np.concatenate([m[0][:, 0, 1], m[1][:, 0, 1]]) - m1 ** 2
        errs.append((np.abs(m1 - mean).max(), np.abs(v / var - 1).max()))
    assert errs[1][0] < 0.05 and errs[1][1] < 0.25
    assert errs[1][0] < errs[0][0]


def test_theorem1_schedule_unbiased_and_vanishing_variance():
    """Theorem 1: with unbiased, finite-variance new estimates and the step
    t^-p (0 < p < 1), the EMA's bias and variance go to zero; a constant step
    keeps a variance of about lam / (2 - lam).  4000 independent replicates of
    an estimator m_hat ~ N(mu, 1) from m_0 = 0."""
    rng = np.random.default_rng(11)
    mu, reps = 2.0, 4000
    for p, lam in ((0.6, None), (0.0, 0.3)):
        m = [np.zeros(reps)]
        var_at = {}
        for t in range(1, 3001):
            m = M.ema(m, [mu + rng.normal(size=reps)], M.ema_step(lam if lam else 0.0, p, t))
            if t in (100, 3000):
                var_at[t] = (m[0].mean() - mu, m[0].var())
        if p > 0:
            assert abs(var_at[3000][0]) < 0.01 and var_at[3000][1] < 0.01
            assert var_at[3000][1] < 0.5 * var_at[100][1]
        else:
            assert abs(var_at[3000][1] - lam / (2 - lam)) < 0.02


def test_second_sample_numerator_is_unbiased():
    """The rescaled estimate keeps K^-n sum_k r_k m(z^k) = P_MP(z) sum_k w_k m(z^k),
    whose expectation is P(x) E_post[m] for any K (section 3.2); Monte Carlo
    over sample seeds on the conjugate normal-normal model, m = (mu, mu^2)."""
    model = S.normal_normal(6, n_groups=2, n_obs=2, K=4)
    mean, var, logev = _normal_normal_posterior(model)
    acc = []
    for s_ in range(3000):
        qs, zs, us, st, ws = _estep(model, 4, seed=2000 + s_)
        m_one = M.moments(zs, ws)[0][0, 0]
        acc.append(np.exp(st.logphat - logev) * m_one)
    acc = np.array(acc)
    se = acc.std(0) / np.sqrt(len(acc))
    target = np.array([mean[0], mean[0] ** 2 + var[0]])
    assert np.all(np.abs(acc.mean(0) - target) < 4 * se + 1e-3), (acc.mean(0), target, se)


def test_second_sample_qem_uses_an_independent_draw():
    """With second_sample the first iteration rescales m_one by
    P_MP(z) / P_MP(z_new), z_new drawn from the second Philox stream."""
    model = S.normal_normal(3)
    K, lam, seed = 8, 0.5, 4
    m1, _ = M.qem(model, K, 1, lam, seed, second_sample=True)
    m0 = M.mean_params(model, M.q_init(model))
    qs, _ = M.set_params(model, m0)
    zs = M.sample(model, qs, K, 1, seed)
    st, ws, m_one = M.estep(model, qs, zs, K)
    z2 = M.sample(model, qs, K, 1 ^ M.SECOND_SAMPLE_STREAM, seed)
    assert not np.allclose(z2[1], zs[1])
    rho = np.exp(st.logphat - M.logphat_forward(model, qs, z2, K))
    ref = M.ema(m0, [rho * x for x in m_one], lam)
    for a, b in zip(m1, ref):
        np.testing.assert_allclose(a, b, rtol=1e-14)


def _kalman_rts(x, a, q, r, m0, p0):
    T = len(x)
    mf, pf = np.zeros(T), np.zeros(T)
    mp, pp = m0, p0
    for t in range(T):
        if t > 0:
            mp, pp = a * mf[t - 1], a * a * pf[t - 1] + q
        k = pp / (pp + r)
        mf[t], pf[t] = mp + k * (x[t] - mp), (1 - k) * pp
    ms, ps = mf.copy(), pf.copy()
    for t in range(T - 2, -1, -1):
        pred = a * a * pf[t] + q
        c = a * pf[t] / pred
        ms[t] = mf[t] + c * (ms[t + 1] - a * mf[t])
        ps[t] = pf[t] + c * c * (ps[t + 1] - pred)
    return ms, ps


def test_chain_qem_approaches_kalman_smoother():
    model = S.chain(9, n_series=2, T=8, K=256)
    m, _ = M.qem(model, 256, 25, 0.3, seed=5)
    x = model.obs[0].x.reshape(2, 8)
    m1 = m[0][:, 0, 0].reshape(2, 8)
    v = (m[0][:, 0, 1] - m[0][:, 0, 0] ** 2).reshape(2, 8)
    for g in range(2):
        ms, ps = _kalman_rts(x[g], 0.9, 0.09, 0.25, 0.0, 1.0)
        assert np.abs(m1[g] - ms).max() < 0.05
        assert np.abs(v[g] / ps - 1).max() < 0.3


def test_gamma_poisson_conditional():
    """lambda | y ~ Gamma(a0 + sum y, b0 + J): QEM moments approach it."""
    a0, b0, J = 2.0, 1.0, 64
    model = _gp_roots(11, 6, J, a0, b0)
    sy = model.obs[0].x.sum(1)
    m, _ = M.qem(model, 1024, 40, 0.3, seed=3)
    post_mean = (a0 + sy) / (b0 + J)
    post_var = (a0 + sy) / (b0 + J) ** 2
    np.testing.assert_allclose(m[0][:, 0, 0], post_mean, rtol=0.02)
    np.testing.assert_allclose(m[0][:, 0, 1] - m[0][:, 0, 0] ** 2, post_var, rtol=0.15)


def test_gamma_poisson_conditional_ef():
    """The same conjugate case with the exponential-family M-step: the fixed
    point of QEM is the exact posterior Gamma(a0 + sum y, b0 + J) itself, so
    the fitted shape and rate approach it (not only its mean and variance)."""
    a0, b0, J = 2.0, 1.0, 64
    model = _gp_roots(11, 6, J, a0, b0)
    model.nodes[0].qfamily = "gamma_ef"
    sy = model.obs[0].x.sum(1)
    m, _ = M.qem(model, 1024, 40, 0.3, seed=3)
    q, hits = M.set_params(model, m)
    assert hits == 0
    np.testing.assert_allclose(q[0]["shape"][:, 0], a0 + sy, rtol=0.15)
    np.testing.assert_allclose(q[0]["rate"][:, 0], b0 + J, rtol=0.15)
    np.testing.assert_allclose(m[0][:, 0, 0], (a0 + sy) / (b0 + J), rtol=0.02)
    # E log lambda of the posterior: psi(a) - log b, with psi from scipy
    np.testing.assert_allclose(m[0][:, 0, 1], digamma(a0 + sy) - np.log(b0 + J), atol=0.02)


# ---------------------------------------------------------------- appendix E

@pytest.mark.parametrize("alpha", [1e-2, 1e-3, 1e-4])
def test_reparameterisation_invariance(alpha):
    """Scale mu to mu~ = mu / alpha with its prior and proposal scaled and the
    same standard-normal draws: log P_MP is unchanged and the moments of mu~
    scale by (1/alpha, 1/alpha^2)."""
    base = S.normal_normal(3)
    scaled = S.normal_normal(3)
    scaled.nodes[0] = S.Node("mu_s", 1, 1, "gauss", "normal", b=0.0, var=1.0 / alpha ** 2)
    scaled.nodes[1].a = alpha
    q0 = M.q_init(base)
    q1 = M.q_init(scaled)
    q1[0] = {"mean": q0[0]["mean"] / alpha, "var": q0[0]["var"] / alpha ** 2}
    _, z0, _, st0, w0 = _estep(base, 8, qs=q0)
    _, z1, _, st1, w1 = _estep(scaled, 8, qs=q1)
    assert abs(st0.logphat - st1.logphat) < 1e-12 * abs(st0.logphat) * 1e3
    m0 = M.moments(z0, w0)
    m1 = M.moments(z1, w1)
    np.testing.assert_allclose(m1[0][..., 0] * alpha, m0[0][..., 0], rtol=1e-9)
    np.testing.assert_allclose(m1[0][..., 1] * alpha ** 2, m0[0][..., 1], rtol=1e-9)
    np.testing.assert_allclose(m1[1], m0[1], rtol=1e-9)


# ---------------------------------------------------------------- M-step

def test_mstep_round_trip():
    m = S.gamma_poisson(0, n_groups=3)
    qs = [{"shape": np.array([[2.5]]), "rate": np.array([[0.7]])},
          {"shape": np.array([[1.2]]), "rate": np.array([[3.0]])},
          {"shape": np.array([[4.0], [0.5], [9.0]]), "rate": np.array([[1.0], [2.0], [0.1]])}]
    back, hits = M.set_params(m, M.mean_params(m, qs))
    assert hits == 0
    for a, b in zip(qs, back):
        np.testing.assert_allclose(a["shape"], b["shape"], rtol=1e-12)
        np.testing.assert_allclose(a["rate"], b["rate"], rtol=1e-12)


def test_ema_keeps_valid_second_moment():
    m_prev = [np.array([[[1.0, 1.5]]])]
    m_one = [np.array([[[3.0, 9.0 + 1e-3]]])]
    out = M.ema(m_prev, m_one, 0.3)[0]
    assert out[0, 0, 1] - out[0, 0, 0] ** 2 > 0
    np.testing.assert_allclose(out, 0.7 * m_prev[0] + 0.3 * m_one[0])


def test_sample_instances_matches_full_sample():
    m = S.chain(1, n_series=4, T=5)
    qs = M.q_init(m)
    full = M.sample(m, qs, 6, 3, 9)[0]
    part = M.sample_instances(m, qs, 6, 3, 9, 0, [7, 12])
    np.testing.assert_array_equal(part, full[[7, 12]])


def test_bf16exp_fold_without_rounding_is_exact():
    """The transfer-matrix fold of the BF16-exp mode with its rounding switched
    off equals the FP64 elimination (messages, log-sum-exp, weights)."""
    from oracle import chain_bf16 as CB
    model = S.chain(3, n_series=2, T=6, K=7)
    qs, zs, us, st, ws = _estep(model, 7, seed=19)
    F = M.chain_table(model, zs, 0, slice(0, 2))
    U = us[0].reshape(2, 6, 7)
    W = ws[0].reshape(2, 6, 7)
    for g in range(2):
        A, c = CB.factors(F[g], rnd=CB.ident)
        m, utt, L = CB.fold(A, c, U[g], rnd=CB.ident, acc=CB.ident)
        assert abs(L - st.chain_L[0][g]) < 1e-11 * abs(L)
        np.testing.assert_allclose(m[1:], st.msg[0][g, 1:], rtol=1e-12, atol=1e-10)
        np.testing.assert_allclose(CB.weights(F[g], m, utt, L), W[g], atol=1e-12)


def test_bf16_rounding_of_fold_is_small():
    """With BF16 rounding on, the fold stays within a few BF16 ulps per step."""
    from oracle import chain_bf16 as CB
    model = S.chain(4, n_series=1, T=10, K=64)
    qs, zs, us, st, ws = _estep(model, 64, seed=2)
    F = M.chain_table(model, zs, 0, slice(0, 1))[0]
    A, c = CB.factors(F)
    m, utt, L = CB.fold(A, c, us[0].reshape(10, 64))
    assert abs(L - st.chain_L[0][0]) < 1e-3 * abs(L)


def _ef_model(n=1):
    m = S.gamma_poisson(0, n_groups=n, qfamily="gamma_ef")
    return m


def test_ef_gamma_exponential_case():
    """Shape 1 (the exponential distribution): E log z = -gamma_E - log rate
    with the Euler-Mascheroni constant, so the M-step must return shape 1."""
    euler_gamma = 0.57721566490153286061
    m = _ef_model()
    rate = np.array([[0.3]])
    ms = [np.stack([1.0 / rate, -euler_gamma - np.log(rate)], axis=-1)] * 2 + \
         [np.stack([1.0 / rate, -euler_gamma - np.log(rate)], axis=-1)]
    q, hits = M.set_params(m, ms)
    assert hits == 0
    for qq in q:
        np.testing.assert_allclose(qq["shape"], 1.0, rtol=1e-12)
        np.testing.assert_allclose(qq["rate"], rate, rtol=1e-12)


def test_ef_gamma_round_trip_wide_range():
    m = _ef_model(n=40)
    rng = np.random.default_rng(5)
    shape = np.exp(rng.uniform(np.log(0.02), np.log(2000.0), size=(40, 1)))
    rate = np.exp(rng.uniform(np.log(0.01), np.log(100.0), size=(40, 1)))
    qs = [{"shape": shape[:1], "rate": rate[:1]}, {"shape": shape[1:2], "rate": rate[1:2]},
          {"shape": shape, "rate": rate}]
    back, hits = M.set_params(m, M.mean_params(m, qs))
    assert hits == 0
    for a, b in zip(qs, back):
        np.testing.assert_allclose(b["shape"], a["shape"], rtol=1e-9)
        np.testing.assert_allclose(b["rate"], a["rate"], rtol=1e-9)


@pytest.mark.parametrize("shape,rate", [(0.4, 2.0), (2.0, 0.5), (30.0, 3.0)])
def test_ef_gamma_recovers_sampled_distribution(shape, rate):
    """The M-step applied to sample averages of (z, log z) of 2e6 draws from
    numpy's Gamma sampler recovers its parameters within 5 standard errors
    of the maximum-likelihood estimate (var(shape) = 1 / (N (psi'(a) - 1/a)))."""
    from scipy.special import polygamma
    N = 2_000_000
    z = np.random.default_rng(11).gamma(shape, 1.0 / rate, size=N)
    m = _ef_model()
    ms = [np.array([[[z.mean(), np.log(z).mean()]]])] * 3
    q, _ = M.set_params(m, ms)
    se = np.sqrt(1.0 / (N * (polygamma(1, shape) - 1.0 / shape)))
    assert abs(q[0]["shape"][0, 0] - shape) < 5 * se
    assert abs(q[0]["shape"][0, 0] / q[0]["rate"][0, 0] - shape / rate) < 5 * np.sqrt(shape / N) / rate


def test_ef_gamma_degenerate_gap_is_floored():
    m = _ef_model()
    ms = [np.array([[[2.0, np.log(2.0)]]])] * 3   # a point mass: log m1 - m2 = 0
    q, hits = M.set_params(m, ms)
    assert hits == 3
    assert np.all(np.isfinite(q[0]["shape"])) and q[0]["shape"][0, 0] > 1e10


def test_ef_moments_use_log_z():
    """The second statistic of an exponential-family Gamma node is log z:
    for a Q equal to the exact posterior every tuple has the same weight,
    so the moments are the plain sample averages of (z, log z)."""
    a0, b0, J = 2.0, 1.5, 20
    model = _gp_roots(7, 5, J, a0, b0)
    model.nodes[0].qfamily = "gamma_ef"
    sy = model.obs[0].x.sum(1)
    qs = [{"shape": (a0 + sy)[:, None], "rate": np.full((5, 1), b0 + J)}]
    _, zs, us, st, ws = _estep(model, 16, qs=qs)
    mo = M.moments(zs, ws, model)[0]
    np.testing.assert_allclose(mo[:, 0, 0], zs[0][:, :, 0].mean(1), rtol=1e-12)
    np.testing.assert_allclose(mo[:, 0, 1], np.log(zs[0][:, :, 0]).mean(1), rtol=1e-12)


# ---------------------------------------------------------------- discrete latents

def _occ_const(n=40, R=4, p_det=0.5, psi=0.4, seed=2):
    """Sites with a known occupancy probability psi (constant prior), so the
    posterior of each site has a closed form."""
    m = S.occupancy(seed, n_sites=n, n_visits=R, p_det=p_det)
    node = S.Node("z", n, 1, "bernoulli", "bernoulli_logit", b=float(np.log(psi / (1 - psi))), q0=(0.5, 1.0))
    return S.Model("occ_const", [node], [S.Obs(0, "detection", m.obs[0].x, var=p_det)], K=8)


def _occ_posterior(y, p_det, psi):
    S_ = y.sum(1)
    R = y.shape[1]
    l1 = psi * p_det ** S_ * (1 - p_det) ** (R - S_)
    l0 = (1 - psi) * (S_ == 0)
    return l1 / (l1 + l0), np.log(l1 + l0)


def test_bernoulli_sampler_frequency():
    m = _occ_const(n=500)
    qs = [{"p": np.full((500, 1), 0.3)}]
    z = M.sample(m, qs, 2000, 4, 9)[0]
    assert set(np.unique(z)) <= {0.0, 1.0}
    assert abs(z.mean() - 0.3) < 5 * np.sqrt(0.21 / z.size)


def test_occupancy_exact_posterior_proposal():
    """With Q(z_i = 1) equal to the exact posterior every r_k equals P(y), so
    log P_MP is the closed-form evidence for any K and the moments are the
    posterior occupancy probabilities."""
    m = _occ_const()
    y = m.obs[0].x
    assert (y.sum(1) > 0).any() and (y.sum(1) == 0).any()
    post, logev = _occ_posterior(y, 0.5, 0.4)
    qs = [{"p": post[:, None]}]
    _, zs, us, st, ws = _estep(m, 8, qs=qs)
    assert abs(st.logphat - logev.sum()) < 1e-10 * abs(logev.sum())
    mo = M.moments(zs, ws, m)[0]
    np.testing.assert_allclose(mo[:, 0, 0], zs[0][:, :, 0].mean(1), atol=1e-14)


def test_occupancy_qem_converges_to_the_posterior():
    m = _occ_const(seed=4)
    y = m.obs[0].x
    post, _ = _occ_posterior(y, 0.5, 0.4)
    mm, _ = M.qem(m, 512, 30, 0.3, seed=3)
    q, _ = M.set_params(m, mm)
    det = y.sum(1) > 0
    # a detected site is occupied: each iteration's moment is exactly 1, so
    # the EMA approaches 1 as 1 - 0.5 (1 - lam)^t
    np.testing.assert_allclose(q[0]["p"][det, 0], 1.0 - 0.5 * 0.7 ** 30, rtol=1e-12)
    # undetected sites: posterior 0.04; the EMA of K = 512 importance
    # estimates has a standard error of about 0.004 per site
    np.testing.assert_allclose(q[0]["p"][~det, 0], post[~det], atol=0.02)
    np.testing.assert_allclose(q[0]["p"][~det, 0].mean(), post[~det].mean(), rtol=0.05)


def test_bernoulli_mstep_clamps_and_counts():
    m = _occ_const(n=3)
    q, hits = M.set_params(m, [np.array([[[0.0, 0.0]], [[0.5, 0.5]], [[1.0, 1.0]]])])
    assert hits == 2
    np.testing.assert_allclose(q[0]["p"][:, 0], [M.BERN_FLOOR, 0.5, 1.0 - M.BERN_FLOOR])


# ---------------------------------------------------------------- chains under a parent

def _gaussian_posterior(model):
    """Exact posterior means and variances of every latent of a linear-Gaussian
    model, by assembling the joint precision of (latents) given the data."""
    sizes = [nd.n for nd in model.nodes]
    off = np.cumsum([0] + sizes)
    n = off[-1]
    Lam = np.zeros((n, n))
    h = np.zeros(n)

    def add_gauss(rows, coefs, const, var):
        # a factor N(sum_j coefs_j z_rows_j ; const, var) in the exponent -(c.z - const)^2 / (2 var)
        c = np.zeros(n)
        for r, k in zip(rows, coefs):
            c[r] += k
        Lam[:] += np.outer(c, c) / var
        h[:] += c * const / var

    for v, nd in enumerate(model.nodes):
        for i in range(nd.n):
            me = off[v] + i
            if nd.chain_len > 1:
                T = nd.chain_len
                g, t = divmod(i, T)
                pb = off[nd.parents[0]] + int(nd.parent_index[i])
                if t == 0:
                    add_gauss([me, pb], [1.0, -1.0], nd.init_b, nd.init_var)
                else:
                    add_gauss([me, me - 1, pb], [1.0, -nd.a, -(1.0 - nd.a)], nd.b, nd.var)
            elif nd.parents:
                pp = off[nd.parents[0]] + (int(nd.parent_index[i]) if nd.parent_index is not None else 0)
                add_gauss([me, pp], [1.0, -nd.a], nd.b, nd.var)
            else:
                add_gauss([me], [1.0], nd.b, nd.var)
    for ob in model.obs:
        for i in range(model.nodes[ob.node].n):
            for x in ob.x[i, :, 0]:
                add_gauss([off[ob.node] + i], [1.0], x, ob.var)
    cov = np.linalg.inv(Lam)
    mean = cov @ h
    return [(mean[off[v]:off[v + 1]], np.diag(cov)[off[v]:off[v + 1]]) for v in range(len(sizes))]


def test_chain_under_parent_converges_to_exact_posterior():
    """With large K, QEM's means and variances of mu, the region levels and
    the chains approach the exact Gaussian posterior."""
    model = S.ar_regions(7, n_regions=2, T=5)
    post = _gaussian_posterior(model)
    m, _ = M.qem(model, 64, 40, 0.3, seed=5)
    for v in range(3):
        mean, var = post[v]
        np.testing.assert_allclose(m[v][:, 0, 0], mean, atol=0.1)
        np.testing.assert_allclose(m[v][:, 0, 1] - m[v][:, 0, 0] ** 2, var, rtol=0.35, atol=0.01)


def test_chain_under_parent_message_is_the_series_likelihood():
    """The message a series sends to its parent sample kb is the log of the
    K-sample estimate of p(y_series | beta^kb): with a single region, a
    parent with one sample (K_parent = K, all samples equal) must give the
    same value for every kb."""
    model = S.ar_regions(2, n_regions=1, T=4, K=5)
    qs = M.q_init(model)
    zs = M.sample(model, qs, 5, 1, 3)
    zs[1][:] = zs[1][0, 0]      # every parent sample the same value
    us = M.unary(model, qs, zs, 5)
    st = M.contract(model, zs, us)
    L = st.msg[2][2]            # [G, Kb]
    np.testing.assert_allclose(L[0], L[0, 0], rtol=1e-14)


# ---------------------------------------------------------------- Dirichlet latents

def _dir_node_model(n, C):
    return S.Model("dir", [S.Node("p", n, C, "dirichlet", "dirichlet", shape=1.0, q0=(1.0, 1.0))], [], None)


def test_dirichlet_beta_case_is_scipy_beta():
    """C = 2: Dir((a, b)) at (z, 1 - z) is the Beta(a, b) density."""
    from oracle import densities as dn
    rng = np.random.default_rng(0)
    z = rng.uniform(0.001, 0.999, size=50)
    a, b = rng.uniform(0.1, 20.0, size=50), rng.uniform(0.1, 20.0, size=50)
    got = dn.dirichlet(np.stack([z, 1.0 - z], -1), np.stack([a, b], -1))
    np.testing.assert_allclose(got, stats.beta.logpdf(z, a, b), rtol=1e-12, atol=1e-12)
    got3 = dn.dirichlet(np.array([0.2, 0.3, 0.5]), np.array([1.5, 2.0, 0.7]))
    assert abs(got3 - stats.dirichlet.logpdf([0.2, 0.3, 0.5], [1.5, 2.0, 0.7])) < 1e-12


@pytest.mark.parametrize("C", [2, 3, 6])
def test_dirichlet_round_trip_wide_range(C):
    """Mean parameters (alpha_c / alpha_0, psi(alpha_c) - psi(alpha_0)) of
    concentrations from 0.05 to 500, back through the M-step solve."""
    rng = np.random.default_rng(C)
    a = np.exp(rng.uniform(np.log(0.05), np.log(500.0), size=(40, C)))
    m = _dir_node_model(40, C)
    mp = M.mean_params(m, [{"alpha": a}])
    np.testing.assert_allclose(mp[0][..., 1], digamma(a) - digamma(a.sum(-1, keepdims=True)), rtol=1e-15)
    qs, hits = M.set_params(m, mp)
    assert hits == 0
    np.testing.assert_allclose(qs[0]["alpha"], a, rtol=1e-9)


@pytest.mark.parametrize("alpha", [(0.3, 2.0, 7.0), (0.05, 0.05), (40.0, 15.0, 5.0, 1.0)])
def test_dirichlet_sampler_moments(alpha):
    """Draws lie on the simplex; their sample means of z and log z match
    alpha / alpha_0 and psi(alpha) - psi(alpha_0) within 5 standard errors;
    the first component's marginal is Beta(alpha_1, alpha_0 - alpha_1) (KS)
    where rounding at 1 is negligible."""
    alpha = np.asarray(alpha)
    C, K = alpha.size, 40000
    m = _dir_node_model(1, C)
    z = M.sample(m, [{"alpha": alpha[None]}], K, 3, 77)[0][0]          # [K, C]
    assert np.all(z > 0.0) and np.max(np.abs(z.sum(-1) - 1.0)) < 1e-14
    a0 = alpha.sum()
    for vals, mean in ((z, alpha / a0), (np.log(z), digamma(alpha) - digamma(a0))):
        se = vals.std(0) / np.sqrt(K)
        assert np.all(np.abs(vals.mean(0) - mean) < 5 * se + 1e-12), (vals.mean(0), mean)
    if alpha.min() >= 0.2:
        # (with alpha = 0.05 a few percent of the mass lies within 1e-16 of 1
        # and rounds to it, so the KS distance there measures rounding)
        ks = stats.kstest(z[:, 0], stats.beta(alpha[0], a0 - alpha[0]).cdf)
        assert ks.pvalue > 1e-3


def test_dirichlet_exact_posterior_makes_every_ratio_equal():
    """With Q_i = Dir(shape + counts_i), the exact posterior, every
    P(x, z) / Q(z) equals P(y_i) = B(shape + counts) / B(shape) (the
    probability of the observed sequence), so u is log P(y_i) - log K for
    every sample and the weights are uniform."""
    m = S.dirichlet_categorical(2, n_groups=5, C=4, n_obs=9, shape=0.6)
    K = 12
    cnt = M.category_counts(m.obs[0], 4)
    post = [{"alpha": 0.6 + cnt}]
    zs = M.sample(m, post, K, 1, 4)
    us = M.unary(m, post, zs, K)
    logpy = gammaln(4 * 0.6) - gammaln(4 * 0.6 + 9) + (gammaln(0.6 + cnt) - gammaln(0.6)).sum(-1)
    np.testing.assert_allclose(us[0], np.broadcast_to(logpy[:, None] - np.log(K), us[0].shape), rtol=0, atol=1e-12)
    st = M.contract(m, zs, us)
    ws = M.reverse(m, zs, st)
    np.testing.assert_allclose(ws[0], 1.0 / K, atol=1e-14)
    assert abs(st.logphat - logpy.sum()) < 1e-11


def test_dirichlet_moments_use_log_z():
    m = S.dirichlet_categorical(3, n_groups=3, C=3, n_obs=4)
    qs, zs, us, st, ws = _estep(m, 8)
    mo = M.moments(zs, ws, m)[0]
    np.testing.assert_allclose(mo[..., 0], np.einsum("nk,nkc->nc", ws[0], zs[0]), rtol=1e-14)
    np.testing.assert_allclose(mo[..., 1], np.einsum("nk,nkc->nc", ws[0], np.log(zs[0])), rtol=1e-14)


def test_dirichlet_degenerate_mean_parameters_are_floored():
    """sum_c exp(E log z_c) >= 1 has no Dirichlet; the M-step moves it to the
    floor gap (a hit) and still returns a concentration that solves it."""
    m = _dir_node_model(2, 3)
    L = np.log(np.array([[0.3, 0.3, 0.4], [0.2, 0.5, 0.31]]))   # sums 1.0 and 1.01
    mp = [np.stack([np.exp(L), L], -1)]
    qs, hits = M.set_params(m, mp)
    assert hits == 2
    a = qs[0]["alpha"]
    got = digamma(a) - digamma(a.sum(-1, keepdims=True))
    assert np.all(np.abs(np.exp(got).sum(-1) - (1.0 - M.DIR_GAP_FLOOR)) < 1e-9)


def test_dirichlet_qem_approaches_the_exact_posterior():
    """With many samples, the QEM fixed point is close to Dir(shape + counts)."""
    m = S.dirichlet_categorical(4, n_groups=3, C=3, n_obs=12, shape=1.0)
    cnt = M.category_counts(m.obs[0], 3)
    ms, _ = M.qem(m, 4096, 25, 0.5, seed=8)
    qs, _ = M.set_params(m, ms)
    np.testing.assert_allclose(qs[0]["alpha"], 1.0 + cnt, rtol=0.15)


# ---------------------------------------------------------------- Categorical latents

def _flat_mixture(seed, n=6, C=4, J=5):
    """Categorical memberships with a uniform prior and Gaussian-mixture data."""
    m = S.mixture(seed, n_groups=n, C=C, n_obs=J)
    nodes = [S.Node("z", n, C, "categorical", "categorical", q0=(1.0 / C, 1.0))]
    return S.Model("flat_mixture", nodes, [S.Obs(0, "gauss_mixture", m.obs[0].x, var=m.obs[0].var, cov=m.obs[0].cov)],
                   None, K=8)


def test_categorical_sampler_frequencies():
    """One-hot draws whose category frequencies match p / sum(p) (unnormalised
    p) within 5 binomial standard errors."""
    C, K = 4, 60000
    m = S.Model("c", [S.Node("z", 1, C, "categorical", "categorical", q0=(0.25, 1.0))], [], None)
    p = np.array([[0.7, 1.4, 2.1, 2.8]])
    z = M.sample(m, [{"p": p}], K, 2, 31)[0][0]
    assert np.all((z == 0.0) | (z == 1.0)) and np.all(z.sum(-1) == 1.0)
    f, pr = z.mean(0), p[0] / p[0].sum()
    assert np.all(np.abs(f - pr) < 5 * np.sqrt(pr * (1 - pr) / K))


def test_categorical_exact_posterior_makes_every_ratio_equal():
    """With Q_i(c) the exact posterior, prop. to exp(sum_j log N(y_ij; mu_c, var)) / C,
    every ratio P(y, z) / Q(z) equals P(y_i) = sum_c exp(lik_ic) / C."""
    from scipy.special import logsumexp
    m = _flat_mixture(3)
    K = 16
    y, mu, var = m.obs[0].x, m.obs[0].cov, m.obs[0].var
    lik = stats.norm.logpdf(y[:, :, None], mu[None, None, :], np.sqrt(var)).sum(1)     # [n, C]
    post = np.exp(lik - logsumexp(lik, axis=1, keepdims=True))
    qs = [{"p": post}]
    zs = M.sample(m, qs, K, 1, 4)
    us = M.unary(m, qs, zs, K)
    logpy = logsumexp(lik, axis=1) - np.log(4)
    np.testing.assert_allclose(us[0], np.broadcast_to(logpy[:, None] - np.log(K), us[0].shape), atol=1e-10)
    st = M.contract(m, zs, us)
    assert abs(st.logphat - logpy.sum()) < 1e-9


def test_categorical_log_q_is_normalised_and_mstep_clamps():
    m = _flat_mixture(4, n=3, C=5)
    p = np.array([[1.0, 2.0, 3.0, 4.0, 5.0]] * 3)
    lq = np.array([[M._log_q(m.nodes[0], {"p": p[:1]}, np.eye(5)[None, c:c + 1])[0, 0] for c in range(5)]])
    assert abs(np.exp(lq).sum() - 1.0) < 1e-15
    m1 = np.array([[0.5, 0.5, 0.0, 0.0, 0.0], [0.2, 0.2, 0.2, 0.2, 0.2], [1.0, 0.0, 0.0, 0.0, 0.0]])
    qs, hits = M.set_params(m, [np.stack([m1, m1], -1)])
    assert hits == 3 + 0 + 4
    assert np.all(qs[0]["p"] >= M.BERN_FLOOR)


@pytest.mark.parametrize("make,K", [(lambda: S.logistic(2, n_groups=23, n_obs=6, D=3), 5),
                                    (lambda: S.gamma_poisson(1, n_groups=19, n_obs=4), 6),
                                    (lambda: S.nested_gaussian(1, n_schools=5, n_classes=7, n_students=2, dim=2), 7)])
def test_threaded_chunks_give_the_same_bits(make, K, monkeypatch):
    """Chunks of instances evaluated on several threads give exactly the
    single-threaded results (each chunk's arithmetic is the same; the sums
    across instances are taken afterwards in instance order)."""
    model = make()
    qs = M.q_init(model)
    zs = M.sample(model, qs, K, 1, 3)
    us = M.unary(model, qs, zs, K)
    monkeypatch.setattr(M, "TABLE_BYTES", 4096)     # many small chunks
    monkeypatch.setattr(M, "WORKERS", 1)
    st1 = M.contract(model, zs, [u.copy() for u in us])
    w1 = M.reverse(model, zs, st1)
    monkeypatch.setattr(M, "WORKERS", 4)
    st4 = M.contract(model, zs, [u.copy() for u in us])
    w4 = M.reverse(model, zs, st4)
    assert st1.logphat == st4.logphat
    for a, b in zip(w1, w4):
        assert np.array_equal(a, b)
    for a, b in zip(st1.ut, st4.ut):
        assert np.array_equal(a, b)
