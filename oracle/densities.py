"""Log-densities used by the model and the proposal (oracle side, FP64).

Conventions: Normal(mean, variance); Gamma(shape, rate); Poisson(rate);
Bernoulli with a logit, where log p(y | eta) = y*eta - softplus(eta) and
softplus(eta) = max(eta, 0) + log1p(exp(-|eta|)); Dirichlet(alpha) on the
simplex of the last axis; categorical draws summarised by their counts.
"""
from __future__ import annotations

import numpy as np
from scipy.special import gammaln

LOG_2PI = float(np.log(2.0 * np.pi))


def normal(x, mean, var):
    x = np.asarray(x, dtype=np.float64)
    return -0.5 * (LOG_2PI + np.log(var)) - 0.5 * (x - mean) ** 2 / var


def gamma(x, shape, rate):
    x = np.asarray(x, dtype=np.float64)
    return shape * np.log(rate) - gammaln(shape) + (shape - 1.0) * np.log(x) - rate * x


def poisson(y, rate):
    y = np.asarray(y, dtype=np.float64)
    return y * np.log(rate) - rate - gammaln(y + 1.0)


def softplus(eta):
    eta = np.asarray(eta, dtype=np.float64)
    return np.maximum(eta, 0.0) + np.log1p(np.exp(-np.abs(eta)))


def bernoulli_logit(y, eta):
    return np.asarray(y, dtype=np.float64) * eta - softplus(eta)


def detection(y, z, p):
    """log P(y | z) for a detection y in {0, 1} ~ Bernoulli(p z), z in {0, 1}:
    y log(p z) + (1 - y) log(1 - p z), with 0 log 0 = 0."""
    y = np.asarray(y, dtype=np.float64)
    pz = p * np.asarray(z, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.where(y == 1.0, np.log(pz), np.log1p(-pz))


def dirichlet(z, alpha):
    """log Dir(z; alpha) over the last axis: lgamma(sum alpha) - sum lgamma(alpha)
    + sum (alpha - 1) log z."""
    z = np.asarray(z, dtype=np.float64)
    alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), z.shape)
    return gammaln(alpha.sum(-1)) - gammaln(alpha).sum(-1) + ((alpha - 1.0) * np.log(z)).sum(-1)


def categorical_counts(counts, z):
    """log of the probability of a sequence of categorical draws with per-category
    counts n_c under category probabilities z: sum_c n_c log z_c (last axis)."""
    return (np.asarray(counts, dtype=np.float64) * np.log(np.asarray(z, dtype=np.float64))).sum(-1)
