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
