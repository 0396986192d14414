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
