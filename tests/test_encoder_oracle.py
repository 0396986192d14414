"""Pins for the encoder oracle: backprop against central finite differences,
GELU and its derivative against numeric differentiation, the KL loss against
numeric integration, and BF16 rounding against its definition."""
import numpy as np
from scipy import integrate, stats

from oracle import encoder as E


def _params(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, E.NPARAM)


def test_param_count():
    assert E.NPARAM == 18 * 64 + 64 + 64 * 64 + 64 + 2 * 64 + 2 == 5506


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = _params()
    x = rng.normal(size=(7, E.IN))
    target = np.stack([rng.normal(size=7), rng.uniform(0.1, 2.0, size=7)], 1)
    out, cache = E.forward(p, x)
    loss, d = E.kl_loss(out, target)
    g = E.backward(p, cache, d)
    h = 1e-6
    for idx in rng.choice(E.NPARAM, 60, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[idx] += h
        pm[idx] -= h
        fd = (E.kl_loss(E.forward(pp, x)[0], target)[0] - E.kl_loss(E.forward(pm, x)[0], target)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7 + 1e-6 * abs(fd), idx


def test_gelu_derivative():
    a = np.linspace(-6, 6, 101)
    h = 1e-6
    np.testing.assert_allclose(E.gelu_grad(a), (E.gelu(a + h) - E.gelu(a - h)) / (2 * h), atol=1e-8)
    np.testing.assert_allclose(E.gelu(a), a * stats.norm.cdf(a), atol=1e-14)


def test_kl_against_integration():
    for mt, vt, mu, s in [(0.3, 0.5, -0.2, 0.1), (2.0, 0.05, 1.5, -1.0)]:
        p = stats.norm(mt, np.sqrt(vt))
        q = stats.norm(mu, np.exp(0.5 * s))
        kl_num = integrate.quad(lambda z: p.pdf(z) * (p.logpdf(z) - q.logpdf(z)), -30, 30, limit=200)[0]
        kl, _ = E.kl_loss(np.array([[mu, s]]), np.array([[mt, vt]]))
        assert abs(kl - kl_num) < 1e-8


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -3.140625, 1e-3], dtype=np.float32)
    r = E.bf16_round(x)
    assert r[0] == 1.0
    assert r[2] == 1.0                       # below half an ulp (2^-7 at 1) rounds down
    assert r[4] == -3.140625                 # exactly representable
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> 1 (even mantissa)
    assert r[1] == 1.0
    # 1 + 3*2^-9 rounds up to 1 + 2^-7
    assert r[3] == 1.0 + 2 ** -7
    # bf16 values keep 8 significant bits
    m, e = np.frexp(r[5])
    assert abs(m * 2 ** 8 - round(m * 2 ** 8)) < 1e-12


# ------------------------------------------------ the global head's pooled inputs

def test_mean_sigmoid_slope_against_integration():
    """c(s) = E[sigma'(s Z)] by the trapezoid rule equals adaptive quadrature;
    c(0) = 1/4 and s c(s) -> 1/sqrt(2 pi) for large s (sigma' integrates to 1)."""
    from scipy import special
    for s in (0.0, 0.3, 1.0, 2.8, 7.0):
        ref = integrate.quad(lambda z: stats.norm.pdf(z) * special.expit(s * z) * (1 - special.expit(s * z)),
                             -40, 40, limit=200)[0]
        assert abs(E.mean_sigmoid_slope(s) - ref) < 1e-10, s
    assert abs(E.mean_sigmoid_slope(0.0) - 0.25) < 1e-12
    assert abs(40.0 * E.mean_sigmoid_slope(40.0) - 1.0 / np.sqrt(2 * np.pi)) < 2e-3


def test_stein_identity_behind_the_beta_plug_in():
    """For x ~ N(0, I) and eta = x'beta + b, E[sigma(eta) x] = E[sigma'(eta)] beta
    (Monte Carlo, 4M draws, bound of 5 standard errors), and solve_beta_norm
    inverts |E[y x]| exactly."""
    rng = np.random.default_rng(3)
    beta = np.array([0.8, -1.1, 0.3])
    sig = 0.7
    n = 4_000_000
    x = rng.normal(size=(n, 3))
    eta = x @ beta + sig * rng.normal(size=n)
    px = (1.0 / (1.0 + np.exp(-eta)))[:, None] * x
    se = px.std(0) / np.sqrt(n)
    c = E.mean_sigmoid_slope(np.sqrt(beta @ beta + sig * sig))
    assert np.all(np.abs(px.mean(0) - c * beta) < 5 * se)
    nyx = c * np.sqrt(beta @ beta)
    assert abs(E.solve_beta_norm(nyx, sig * sig) - np.sqrt(beta @ beta)) < 1e-9


def test_pooled_plug_ins_recover_the_generating_globals():
    """On the mixed-effects logistic hierarchy (8192 groups x 50 observations)
    the plug-ins of pool_rows land near the latents that generated the data:
    the direction of beta to a cosine above 0.995, |beta| within 8%, log sigma
    within 0.15 (the head learns the remaining residual)."""
    import qem_synth as S
    for seed in (0, 3):
        m = S.logistic(seed)
        ob = m.obs[0]
        rows = E.pool_rows(E.features(ob.x, ob.cov), ob.x.shape[1])
        b_true = np.asarray(m.truth[0]).ravel()
        ls_true = float(np.asarray(m.truth[1]).ravel()[0])
        b = rows[:8, 1]
        cos = b @ b_true / np.sqrt((b @ b) * (b_true @ b_true))
        assert cos > 0.995, (seed, cos)
        assert abs(np.sqrt(b @ b) / np.sqrt(b_true @ b_true) - 1.0) < 0.08, seed
        assert abs(rows[8, 1] - ls_true) < 0.15, (seed, rows[8, 1], ls_true)
        # the rows are consistent with their own definition
        assert np.allclose(rows[:8, 2], b / np.sqrt(b @ b)) and np.all(rows[:, 0] == 1.0)
        assert rows[8, 6] == 1.0 and np.all(rows[:8, 6] == 0.0)


def test_context_features_follow_their_definition():
    rng = np.random.default_rng(5)
    y = (rng.uniform(size=(40, 50)) < 0.4).astype(float)
    cov = rng.normal(size=(40, 50, 8))
    f = E.features(y, cov)
    rows = E.pool_rows(f, 50)
    g = E.features_ctx(f, rows, 50)
    beta, kappa = rows[:8, 1], rows[0, 9]
    i = 7
    ybar = y[i].mean()
    yc = (ybar * 50 + 0.5) / 51
    e = np.log(yc / (1 - yc))
    o = cov[i].mean(0) @ beta
    np.testing.assert_allclose(g[i, :10], [1, ybar, o, (y[i][:, None] * cov[i]).mean(0) @ beta, e, e / kappa - o,
                                           np.exp(rows[8, 1]), rows[0, 3], kappa, 1 / (50 * yc * (1 - yc) * kappa)],
                               rtol=1e-12)
    assert np.all(g[:, 10:] == 0)
