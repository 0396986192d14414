"""BF16-exp chain contraction, emulated in numpy (oracle side, test infrastructure).

The chain contraction (section 3.2's elimination applied to a series) written
as products of transfer matrices in the exponential domain: a carried matrix
R[k, kend] over the samples of the current step and of the last step, kept as
entries in [0, 1] with per-column log-scales, multiplied step by step by the
row-shifted factor matrices exp(F_t - c_t).  With ``rnd`` = BF16 rounding and
``acc`` = FP32 rounding this reproduces the rounding points of the BF16-exp
mode (BF16 operands, FP32 products and bookkeeping); with both set to the
identity it is exact and must agree with the FP64 elimination in mpiw.py.

Messages m_t[kp] (into step t-1) and the per-series log-sum-exp L come from
the fold; the marginal weights from the forward recursion over the exact
factors F with those messages, renormalised per step (the messages are those
of the rounded products, so the weights of one step sum to one only after
renormalising).
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to BF16 (nearest, ties to even) from FP32; float32 result."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def f32(x):
    return np.asarray(x, dtype=np.float32)


def ident(x):
    return np.asarray(x, dtype=np.float64)


def factors(F, rnd=bf16):
    """F [T-1, K, K] -> (A = rnd(exp(F - c)), c = row max of F)."""
    c = F.max(axis=-1)
    return rnd(np.exp(F - c[..., None])), c


def fold(A, c, ut, rnd=bf16, acc=f32):
    """One series: A [T-1, K, K], c [T-1, K], ut [T, K] (u plus child messages).

    Returns (messages m [T, K] with m[t] the message into step t-1 for t >= 1,
    u-tilde [T, K], L)."""
    T, K = ut.shape
    R = np.eye(K)
    r = np.array(ut[T - 1], dtype=np.float64)
    m = np.full((T, K), np.nan)
    utt = np.array(ut, dtype=np.float64)
    for t in range(T - 1, 0, -1):
        P = np.asarray(acc(np.asarray(A[t - 1], np.float64) @ np.asarray(R, np.float64)), np.float64)
        rmax = r.max()
        s = (P * np.exp(r - rmax)[None, :]).sum(1)
        with np.errstate(divide="ignore"):
            m[t] = c[t - 1] + rmax + np.log(s)
        gvec = ut[t - 1] + c[t - 1]
        utt[t - 1] = ut[t - 1] + m[t]
        if t == 1:
            break
        mu = gvec.max()
        x = P * np.exp(gvec - mu)[:, None]
        colmax = x.max(0)
        with np.errstate(divide="ignore", invalid="ignore"):
            R = np.where(colmax > 0, rnd(x / np.where(colmax > 0, colmax, 1.0)), 0.0)
            r = np.where(colmax > 0, r + mu + np.log(np.where(colmax > 0, colmax, 1.0)), -np.inf)
    top = utt[0].max()
    L = float(top + np.log(np.exp(utt[0] - top).sum()))
    return m, utt, L


def weights(F, m, utt, L):
    """Marginal weights of every step: w_0 = exp(ut~_0 - L), then
    w_t[k] proportional to sum_kp w_{t-1}[kp] exp(F_t[kp,k] + ut~_t[k] - m_t[kp])
    with the exact factors F [T-1, K, K], renormalised to sum to one."""
    T, K = utt.shape
    w = np.zeros((T, K))
    w[0] = np.exp(utt[0] - L)
    for t in range(1, T):
        X = np.asarray(F[t - 1], np.float64) - m[t][:, None] + utt[t][None, :]
        wt = (w[t - 1][:, None] * np.exp(X)).sum(0)
        w[t] = wt / wt.sum()
    return w
