"""Philox4x32-10 and the proposal samplers built on it (oracle side).

Philox4x32 follows Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
as easy as 1, 2, 3" (SC'11): a 4x32-bit counter and a 2x32-bit key; each of
the 10 rounds multiplies counter words 0 and 2 by two fixed odd constants,
and mixes the high halves with the other counter words and the round key;
the key is advanced by the two Weyl constants between rounds.

Counter layout used by the E-step sampler, for element e of a node's sample
tensor [n, K, d] (flat index (i*K + k)*d + j), at QEM iteration t, node id v:
    counter = (e, sub, t, v),  key = (seed & 0xffffffff, seed >> 32)
``sub`` selects the draw: 0 for the Gamma shape boost uniform; 1 + 2a and
2 + 2a for the normal and the uniform of Marsaglia-Tsang attempt a.  The
Gaussian proposal draws its normals in pairs: elements 2p and 2p + 1 share
the block at counter (p, 0, t, v).

Uniforms take 53 bits from two 32-bit words ((w0 << 32 | w1) >> 11).
Normals use the Box-Muller transform on the two uniforms (u1, u2) of one
Philox block: r = sqrt(-2 log u1), theta = 2 pi u2, giving r cos(theta) and
r sin(theta); the Gaussian proposal uses both (even element: cosine, odd
element: sine), the Gamma sampler the cosine branch of its own block.  Gamma variates use Marsaglia and Tsang (2000),
"A simple method for generating gamma variables", with the shape < 1 boost
Gamma(a) = Gamma(a + 1) * U^(1/a).
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF
MT_MAX_ATTEMPTS = 32

_u64 = np.uint64


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Return the four 32-bit output words for counters (c0..c3) and key (k0, k1)."""
    c = [np.asarray(x, dtype=np.uint64) & _u64(MASK32) for x in (c0, c1, c2, c3)]
    c = list(np.broadcast_arrays(*c))
    k0 &= MASK32
    k1 &= MASK32
    for r in range(10):
        p0 = _u64(M0) * c[0]
        p1 = _u64(M1) * c[2]
        hi0, lo0 = p0 >> _u64(32), p0 & _u64(MASK32)
        hi1, lo1 = p1 >> _u64(32), p1 & _u64(MASK32)
        c = [hi1 ^ c[1] ^ _u64(k0), lo1, hi0 ^ c[3] ^ _u64(k1), lo0]
        k0 = (k0 + W0) & MASK32
        k1 = (k1 + W1) & MASK32
    return tuple(x.astype(np.uint32) for x in c)


def _bits53(w_hi, w_lo):
    return ((w_hi.astype(np.uint64) << _u64(32)) | w_lo.astype(np.uint64)) >> _u64(11)


def _u_open_closed(w_hi, w_lo):
    """Uniform on (0, 1]."""
    return (_bits53(w_hi, w_lo).astype(np.float64) + 1.0) * 2.0 ** -53


def _u_closed_open(w_hi, w_lo):
    """Uniform on [0, 1)."""
    return _bits53(w_hi, w_lo).astype(np.float64) * 2.0 ** -53


def _key(seed: int):
    return seed & MASK32, (seed >> 32) & MASK32


def std_normal(e, sub, it: int, node: int, seed: int):
    """Standard normal for elements ``e`` (Box-Muller, cosine branch)."""
    k0, k1 = _key(seed)
    r0, r1, r2, r3 = philox4x32_10(e, sub, it, node, k0, k1)
    u1 = _u_open_closed(r0, r1)
    u2 = _u_closed_open(r2, r3)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def std_normal_paired(e, it: int, node: int, seed: int):
    """Standard normal for elements ``e`` of a Gaussian proposal: the block at
    counter (e >> 1, 0, it, node) gives the pair (r cos theta, r sin theta);
    even elements take the cosine, odd ones the sine."""
    e = np.asarray(e, dtype=np.uint64)
    k0, k1 = _key(seed)
    r0, r1, r2, r3 = philox4x32_10(e >> _u64(1), 0, it, node, k0, k1)
    u1 = _u_open_closed(r0, r1)
    u2 = _u_closed_open(r2, r3)
    r = np.sqrt(-2.0 * np.log(u1))
    theta = 2.0 * np.pi * u2
    return r * np.where((e & _u64(1)) == _u64(1), np.sin(theta), np.cos(theta))


def uniform_oc(e, sub, it: int, node: int, seed: int):
    """Uniform on (0, 1] from words 0 and 1 of the block."""
    k0, k1 = _key(seed)
    r0, r1, _, _ = philox4x32_10(e, sub, it, node, k0, k1)
    return _u_open_closed(r0, r1)


def gamma_unit_rate(shape, e, it: int, node: int, seed: int):
    """Gamma(shape, 1) by Marsaglia-Tsang; ``shape`` broadcast against ``e``.

    Attempts are drawn from their own counters, so each element's result does
    not depend on any other element.  If all attempts are rejected (probability
    below 1e-40 for any shape) the mode-like value d is returned.
    """
    e = np.asarray(e, dtype=np.uint64)
    shape = np.broadcast_to(np.asarray(shape, dtype=np.float64), e.shape)
    boost = shape < 1.0
    a = np.where(boost, shape + 1.0, shape)
    d = a - 1.0 / 3.0
    c = 1.0 / np.sqrt(9.0 * d)
    out = d.copy()
    done = np.zeros(e.shape, dtype=bool)
    for att in range(MT_MAX_ATTEMPTS):
        x = std_normal(e, 1 + 2 * att, it, node, seed)
        t = 1.0 + c * x
        v = t * t * t
        u = uniform_oc(e, 2 + 2 * att, it, node, seed)
        pos = v > 0.0
        logv = np.log(np.where(pos, v, 1.0))
        ok = pos & (np.log(u) < 0.5 * x * x + d - d * v + d * logv)
        take = ok & ~done
        out = np.where(take, d * v, out)
        done |= ok
        if done.all():
            break
    ub = uniform_oc(e, 0, it, node, seed)
    with np.errstate(divide="ignore"):
        out = np.where(boost, out * ub ** (1.0 / shape), out)
    return out


def gamma_log_unit_rate(shape, e, it: int, node: int, seed: int):
    """log of the Gamma(shape, 1) draw of ``gamma_unit_rate`` (same counters and
    steps), formed in log space: log(d v) for the accepted attempt (log d if
    none), plus log(u) / shape for shapes below 1, so draws too small for FP64
    keep a finite logarithm."""
    e = np.asarray(e, dtype=np.uint64)
    shape = np.broadcast_to(np.asarray(shape, dtype=np.float64), e.shape)
    boost = shape < 1.0
    a = np.where(boost, shape + 1.0, shape)
    d = a - 1.0 / 3.0
    c = 1.0 / np.sqrt(9.0 * d)
    out = np.log(d)
    done = np.zeros(e.shape, dtype=bool)
    for att in range(MT_MAX_ATTEMPTS):
        x = std_normal(e, 1 + 2 * att, it, node, seed)
        t = 1.0 + c * x
        v = t * t * t
        u = uniform_oc(e, 2 + 2 * att, it, node, seed)
        pos = v > 0.0
        logv = np.log(np.where(pos, v, 1.0))
        ok = pos & (np.log(u) < 0.5 * x * x + d - d * v + d * logv)
        take = ok & ~done
        out = np.where(take, np.log(d) + logv, out)
        done |= ok
        if done.all():
            break
    ub = uniform_oc(e, 0, it, node, seed)
    return np.where(boost, out + np.log(ub) / shape, out)
