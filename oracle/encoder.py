"""FP64 reference of the amortised encoder (oracle side, test infrastructure).

The encoder is not part of the paper: it maps a group's data summary to the
parameters of that group's Gaussian proposal factor, and is trained on the
posterior moments QEM itself produces.  Architecture: 18 -> 64 -> 64 -> 2 with
exact GELU (x * Phi(x)); outputs (mean, log variance).  Loss: the mean over
groups of KL(N(mean_t, var_t) || N(mu, exp(s))), i.e. maximum likelihood of the
proposal under the QEM posterior, the objective L_post of appendix B.

Parameter vector layout (5506 entries):
    W1[64, 18], b1[64], W2[64, 64], b2[64], W3[2, 64], b3[2]   (row-major)
Weights are used as BF16 values (round to nearest even from FP32).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

IN, HID, OUT = 18, 64, 2
SHAPES = [(HID, IN), (HID,), (HID, HID), (HID,), (OUT, HID), (OUT,)]
NPARAM = int(sum(np.prod(s) for s in SHAPES))


def unpack(p):
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(np.asarray(p[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def bf16_round(x):
    """FP32 -> BF16 (round to nearest, ties to even), returned as float64 values."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def features(y, cov):
    """[1, mean_j y, mean_j x_j (D), mean_j y_j x_j (D)] per group."""
    y = np.asarray(y, dtype=np.float64)
    cov = np.asarray(cov, dtype=np.float64)
    n = y.shape[0]
    return np.concatenate([np.ones((n, 1)), y.mean(1, keepdims=True), cov.mean(1),
                           (y[:, :, None] * cov).mean(1)], axis=1)


def _elogit(ybar, J):
    """Empirical logit of a group mean of J Bernoulli outcomes (with the usual +1/2 counts)."""
    yc = (ybar * J + 0.5) / (J + 1.0)
    return np.log(yc / (1.0 - yc)), yc


POOL_FIXED_POINT = 3   # alternations of the |beta| and sigma plug-ins
QUAD_H, QUAD_N = 0.05, 401   # trapezoid nodes z = -10 + h i, i < 401
BISECT_STEPS, B_MAX = 60, 50.0


def mean_sigmoid_slope(s):
    """c(s) = E[sigma'(s Z)], Z ~ N(0, 1), by the trapezoid rule on [-10, 10]
    (the integrand is smooth and negligible beyond the ends)."""
    z = -10.0 + QUAD_H * np.arange(QUAD_N)
    w = np.full(QUAD_N, QUAD_H)
    w[0] = w[-1] = 0.5 * QUAD_H
    t = np.exp(-np.abs(s * z))
    return float((w * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi) * t / (1.0 + t) ** 2).sum())


def solve_beta_norm(nyx, s2):
    """B with c(sqrt(B^2 + s2)) B = nyx by bisection on [0, B_MAX]."""
    lo, hi = 0.0, B_MAX
    for _ in range(BISECT_STEPS):
        mid = 0.5 * (lo + hi)
        if mean_sigmoid_slope(np.sqrt(mid * mid + s2)) * mid < nyx:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def pool_rows(feat, J: int):
    """Input rows of the global head from one dataset's group features [n, 18]
    (J observations per group).

    Pass 1 pools the features: P = mean feature, V = variance of the group
    means of y.  With Gaussian covariates, Stein's lemma gives exactly
    E[y x] = E[sigma'(eta)] beta with eta = x'beta + b ~ N(0, |beta|^2 + sigma^2),
    so P_yx = P[10..17] points along beta (u = P_yx / |P_yx|) and
    B = |beta| solves c(sqrt(B^2 + sigma^2)) B = |P_yx|, c(s) = E[sigma'(s Z)].
    Pass 2 pools the groups' empirical logits e_i against their offsets
    o_i = xbar_i . beta^ (beta^ = u B): within a group the linear predictor
    varies with variance about B^2, which attenuates the logit of the group
    mean by kappa = 4 c(B); a_i = e_i - kappa o_i ~ kappa b_i + noise, the
    noise of the empirical logit being about kappa / (J yc (1 - yc)) (delta
    method, outcomes with varying probabilities), so
        sigma^2 = max((Var(a) - kappa mean noise) / kappa^2, 1e-4),  noise_i = 1 / (J yc_i (1 - yc_i)).
    B starts at sigma = 0 and the two are alternated POOL_FIXED_POINT times.
    Feature 1 of each row is its plug-in estimate (the head predicts the
    residual):
        beta_j:    [1, beta^_j,    u_j, B, 5 |P_yx|, 4 sqrt V, 0, 5 P_xj, P_y, kappa, 0,      0,          0 ...]
        log sigma: [1, log sigma^, 0,   B, 5 |P_yx|, 4 sqrt V, 1, 0,      P_y, kappa, Var(a), mean noise, 0 ...]"""
    f = np.asarray(feat, dtype=np.float64)
    n = f.shape[0]
    P = f.sum(0) / n
    V = max((f[:, 1] * f[:, 1]).sum() / n - P[1] * P[1], 0.0)
    sdy = np.sqrt(V)
    yx = P[10:18]
    nyx = np.sqrt((yx * yx).sum())
    u = yx / nyx if nyx > 0 else np.zeros(8)
    e, yc = _elogit(f[:, 1], J)
    noise = 1.0 / (J * yc * (1.0 - yc))
    mnoise = noise.sum() / n
    s2 = 0.0
    for _ in range(POOL_FIXED_POINT):
        B = solve_beta_norm(nyx, s2)
        beta = u * B
        kappa = 4.0 * mean_sigmoid_slope(B)
        a = e - kappa * (f[:, 2:10] @ beta)
        var_a = max((a * a).sum() / n - (a.sum() / n) ** 2, 0.0)
        s2 = max((var_a - kappa * mnoise) / (kappa * kappa), 1e-4)
    rows = np.zeros((9, IN))
    for j in range(8):
        rows[j, :10] = [1.0, beta[j], u[j], B, 5.0 * nyx, 4.0 * sdy, 0.0, 5.0 * P[2 + j], P[1], kappa]
    rows[8, :12] = [1.0, 0.5 * np.log(s2), 0.0, B, 5.0 * nyx, 4.0 * sdy, 1.0, 0.0, P[1], kappa, var_a, mnoise]
    return rows


def features_ctx(feat, rows, J: int):
    """Group features with the dataset context of the global head's plug-ins
    (rows from pool_rows): for group i with mean outcome ybar_i,
        [1, ybar_i, o_i = xbar_i . beta^, m_i = mean(y x)_i . beta^, e_i (empirical logit),
         b~_i = e_i / kappa - o_i, sigma^, B, kappa, 1 / (J yc_i (1 - yc_i) kappa), 0 ...]
    (the last entry is the noise variance of b~_i)."""
    f = np.asarray(feat, dtype=np.float64)
    r = np.asarray(rows, dtype=np.float64)
    beta, lsig, B, kappa = r[:8, 1], r[8, 1], r[0, 3], r[0, 9]
    e, yc = _elogit(f[:, 1], J)
    o = f[:, 2:10] @ beta
    m = f[:, 10:18] @ beta
    g = np.zeros((f.shape[0], IN))
    g[:, 0] = 1.0
    g[:, 1] = f[:, 1]
    g[:, 2] = o
    g[:, 3] = m
    g[:, 4] = e
    g[:, 5] = e / kappa - o
    g[:, 6] = np.exp(lsig)
    g[:, 7] = B
    g[:, 8] = kappa
    g[:, 9] = 1.0 / (J * yc * (1.0 - yc) * kappa)
    return g


def gelu(a):
    return 0.5 * a * (1.0 + erf(a / np.sqrt(2.0)))


def gelu_grad(a):
    phi = np.exp(-0.5 * a * a) / np.sqrt(2.0 * np.pi)
    return 0.5 * (1.0 + erf(a / np.sqrt(2.0))) + a * phi


def forward(p, x):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    a1 = x @ W1.T + b1
    h1 = gelu(a1)
    a2 = h1 @ W2.T + b2
    h2 = gelu(a2)
    out = h2 @ W3.T + b3
    return out, (x, a1, h1, a2, h2)


def kl_loss(out, target):
    """Mean KL(N(m_t, v_t) || N(mu, exp(s))) and its gradient w.r.t. out."""
    mu, s = out[:, 0], out[:, 1]
    mt, vt = target[:, 0], target[:, 1]
    es = np.exp(-s)
    kl = 0.5 * (s - np.log(vt)) + 0.5 * (vt + (mt - mu) ** 2) * es - 0.5
    n = out.shape[0]
    d = np.stack([-(mt - mu) * es, 0.5 - 0.5 * (vt + (mt - mu) ** 2) * es], axis=1) / n
    return float(kl.mean()), d


def backward(p, cache, dout):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x, a1, h1, a2, h2 = cache
    gW3 = dout.T @ h2
    gb3 = dout.sum(0)
    dz2 = (dout @ W3) * gelu_grad(a2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * gelu_grad(a1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    return np.concatenate([g.reshape(-1) for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam(master, grad, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) on FP32 master weights."""
    m1 = b1 * m1 + (1 - b1) * grad
    m2 = b2 * m2 + (1 - b2) * grad * grad
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    master = master - lr * mh / (np.sqrt(vh) + eps)
    return master, m1, m2
