"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded model, sample seed and iteration.

Both sides draw their own samples from the same Philox counters; the oracle
never reads a value produced by the HIP path.
"""
from __future__ import annotations

import sys

import numpy as np

from oracle import mpiw as M

# Tolerances, rel = |a - b| / max(|b|, 1):
#  log P_MP: 1e-10 (FP64), 1e-4 (FP32).
#  weights: absolute 1e-12 (FP64); FP32 rounds every factor entry (|F| up to
#    ~1e2, relative 6e-8) and the exponent F + ut - m, so weights carry
#    absolute errors up to a few 1e-6; 2e-5 leaves a margin.
#  moments: true relative error of each statistic (mom_rel_err): the first
#    moment against max(|E z|, sd), sd the posterior standard deviation
#    sqrt(E z^2 - (E z)^2), so a mean near zero is judged on the posterior's
#    own scale; E z^2 against |E z^2| (at least sd^2 > 0).  FP64 1e-10; FP32
#    1e-3: an FP32 weight error of a few 1e-6 per sample, summed over K
#    samples of spread ~sd around the mean, moves the mean by ~1e-5 sd.
TOL = {
    "fp64": dict(logphat=1e-10, w=1e-12, mom=1e-10, z=1e-13),
    "fp32": dict(logphat=1e-4, w=2e-5, mom=1e-3, z=3e-7),
}


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    """max |a - b| / max(|b|, 1); equal entries (the same infinity included) count 0."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if not a.size:
        return 0.0
    with np.errstate(invalid="ignore"):
        d = np.where(a == b, 0.0, np.abs(a - b) / np.maximum(np.abs(b), 1.0))
    return float(np.max(d))


# families whose second mean parameter is E log z (compared on the old scale)
LOG_STAT_FAMILIES = ("gamma_ef", "dirichlet")
# families whose sample is an indicator (z^2 = z): both statistics are a
# probability p whose posterior spread is the indicator's sd sqrt(p (1 - p))
INDICATOR_FAMILIES = ("bernoulli", "categorical")


def mom_rel_err(a, b, qfamily="gauss"):
    """Largest relative error of moments [n, d, 2] = (E z, E z^2) per
    instance and dimension: |da1| / max(|b1|, sd), |da2| / max(|b2|, sd^2),
    sd^2 = max(b2 - b1^2, 0) (a point mass, sd = 0, falls back to |b|).  For
    the E log z families the second statistic is judged against max(|b2|, 1).
    For indicator samples (Bernoulli, one-hot categorical) both statistics
    are the probability p and are judged against max(p, sqrt(p (1 - p))): a
    category of posterior probability 1e-37 sits at the edge of FP32's normal
    range, where its weight keeps only a few bits, but its error is nothing
    on the scale of the indicator's spread."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if not a.size:
        return 0.0
    a1, a2, b1, b2 = a[..., 0], a[..., 1], b[..., 0], b[..., 1]
    if qfamily in LOG_STAT_FAMILIES:
        return max(rel_err(a1, b1), rel_err(a2, b2))
    tiny = np.finfo(np.float64).tiny
    if qfamily in INDICATOR_FAMILIES:
        s = np.maximum(np.abs(b1), np.sqrt(np.clip(b1 * (1.0 - b1), 0.0, None)))
        with np.errstate(invalid="ignore"):
            e1 = np.where(a1 == b1, 0.0, np.abs(a1 - b1) / np.maximum(s, tiny))
            e2 = np.where(a2 == b2, 0.0, np.abs(a2 - b2) / np.maximum(s, tiny))
        return float(max(e1.max(), e2.max()))
    var = np.maximum(b2 - b1 * b1, 0.0)
    s1 = np.maximum(np.abs(b1), np.sqrt(var))
    s2 = np.maximum(np.abs(b2), var)
    with np.errstate(invalid="ignore"):
        e1 = np.where(a1 == b1, 0.0, np.abs(a1 - b1) / np.maximum(s1, tiny))
        e2 = np.where(a2 == b2, 0.0, np.abs(a2 - b2) / np.maximum(s2, tiny))
    return float(max(e1.max(), e2.max()))


def gpu_run(model, K, prec, seed, it, steps=("sample", "logfactors", "fwd", "bwd", "moments")):
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    say(f"[gpu] {model.name} K={K} prec={prec} seed={seed} it={it}")
    q = QEM(model, K, prec)
    if "sample" in steps:
        q.sample(seed, it)
    if "logfactors" in steps:
        q.logfactors()
    if "fwd" in steps:
        q.contract_fwd()
    if "bwd" in steps:
        q.contract_bwd()
    if "moments" in steps:
        q.moments()
    torch.cuda.synchronize()
    N = len(model.nodes)
    out = {
        "z": [q.tensor(v, _lib.T_Z).double().cpu().numpy() for v in range(N)],
        "u": [q.tensor(v, _lib.T_U).double().cpu().numpy() for v in range(N)],
        "ut": [q.tensor(v, _lib.T_UT).cpu().numpy() for v in range(N)],
        "w": [q.tensor(v, _lib.T_W).double().cpu().numpy() for v in range(N)],
        "mone": [q.tensor(v, _lib.T_MONE).cpu().numpy() for v in range(N)],
        "logphat": q.logphat(),
        "status": q.read_status(),
        "ctx": q,
    }
    return out


def oracle_run(model, K, seed, it, qs=None, workers=None):
    """The oracle's E-step at Q_0 (or the given proposal); `workers` host
    threads evaluate independent chunks of instances."""
    prev = M.WORKERS
    if workers is not None:
        M.WORKERS = workers
    try:
        qs = M.q_init(model) if qs is None else qs
        zs = M.sample(model, qs, K, it, seed)
        us = M.unary(model, qs, zs, K)
        st = M.contract(model, zs, us)
        ws = M.reverse(model, zs, st)
    finally:
        M.WORKERS = prev
    return dict(qs=qs, z=zs, u=us, st=st, w=ws, mone=M.moments(zs, ws, model), logphat=st.logphat,
                families=[nd.qfamily for nd in model.nodes])


def compare_estep(g, o, prec, check_u=True, model=None):
    tol = TOL[prec]
    for v, (a, b) in enumerate(zip(g["z"], o["z"])):
        e = rel_err(a, b)
        assert e <= tol["z"], f"samples of node {v}: rel err {e:.3e}"
    if check_u:
        for v, (a, b) in enumerate(zip(g["u"], o["u"])):
            e = rel_err(a, b)
            assert e <= 10 * tol["logphat"], f"unary factors of node {v}: rel err {e:.3e}"
    e = rel_err(g["logphat"], o["logphat"])
    assert e <= tol["logphat"], f"log P_MP {g['logphat']!r} vs {o['logphat']!r}: rel err {e:.3e}"
    for v, (a, b) in enumerate(zip(g["w"], o["w"])):
        e = float(np.max(np.abs(a - b)))
        assert e <= tol["w"], f"weights of node {v}: abs err {e:.3e}"
    for v, (a, b) in enumerate(zip(g["mone"], o["mone"])):
        fam = model.nodes[v].qfamily if model is not None else o.get("families", [None] * (v + 1))[v] or "gauss"
        e = mom_rel_err(a, b, fam)
        assert e <= tol["mom"], f"moments of node {v}: rel err {e:.3e}"
