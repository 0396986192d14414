"""Chains in BF16-exp mode (BF16 exp-shifted factors formed in the fold
kernel, MFMA transfer-matrix fold with FP32 accumulation and bookkeeping; the
reverse pass on the FP32 factors with the fold's messages, renormalised per
step) against the emulated-BF16 oracle, and the precision report of BF16-exp,
FP32 and FP64 against the FP64 oracle.
"""
import numpy as np
import pytest

import qem_synth as S
from oracle import chain_bf16 as CB
from oracle import mpiw as M

from _parity import gpu_run, mom_rel_err, rel_err, say

pytestmark = pytest.mark.gpu


def _series_reference(model, K, seed, it, g, zs=None):
    """FP64 oracle and emulated-BF16 oracle for series g (own samples)."""
    T = model.nodes[0].chain_len
    qs = M.q_init(model)
    z = M.sample_instances(model, qs, K, it, seed, 0, np.arange(g * T, g * T + T))
    sub = S.chain(0, n_series=1, T=T)
    sub.obs[0] = S.Obs(0, "gauss", model.obs[0].x.reshape(-1, T, 1, 1)[g].reshape(-1, 1, 1), var=model.obs[0].var)
    us = M.unary(sub, M.q_init(sub), [z], K)
    st = M.contract(sub, [z], us)
    ws = M.reverse(sub, [z], st)
    mom = M.moments([z], ws)[0]
    F = M.chain_table(sub, [z], 0, slice(0, 1))[0]
    A, c = CB.factors(F)
    m, utt, L = CB.fold(A, c, us[0].reshape(T, K))
    wb = CB.weights(F, m, utt, L)
    return dict(z=z[..., 0], L64=st.logphat, w64=ws[0], mom64=mom, Lb=L, wb=wb, mb=m)


def test_bexp_chain_small_vs_emulated_oracle():
    model = S.chain(2, n_series=6, T=9)
    K = 64
    g = gpu_run(model, K, "bf16exp", seed=7, it=2)
    from paper_2503_08264_amd import _lib
    Lg = g["ctx"].tensor(0, _lib.T_ROOTL).cpu().numpy()
    msg = g["ctx"].tensor(0, _lib.T_MSG).cpu().numpy()
    w = g["w"][0].reshape(6, 9, K)
    np.testing.assert_allclose(w.sum(-1), 1.0, atol=1e-5)
    errs = []
    for s in range(6):
        ref = _series_reference(model, K, 7, 2, s)
        errs.append((rel_err(Lg[s], ref["Lb"]), float(np.max(np.abs(msg[s, 1:] - ref["mb"][1:]))),
                     float(np.max(np.abs(w[s] - ref["wb"])))))
        assert rel_err(Lg[s], ref["Lb"]) < 2e-5, (s, Lg[s], ref["Lb"])
        np.testing.assert_allclose(msg[s, 1:], ref["mb"][1:], atol=2e-3)
        assert np.max(np.abs(w[s] - ref["wb"])) < 2e-3
        # against the exact FP64 oracle
        assert rel_err(Lg[s], ref["L64"]) < 1e-3
    e = np.max(np.array(errs), 0)
    say(f"[bf16exp vs emulated oracle] log P_MP rel {e[0]:.2e}, messages abs {e[1]:.2e}, weights abs {e[2]:.2e}")
    flags, _, _ = g["status"]
    assert flags == 0


def test_chain_precision_report_full_size():
    """1024 series x T = 64, K = 256: log P_MP per series, weights and moments
    of 64 series spread over the batch (every 16th, plus the last) in
    BF16-exp, FP32 and FP64 against the FP64 oracle.

    Bounds: FP64 and FP32 at the parity tolerances; BF16-exp: log P_MP of a
    series to 2e-4 relative, weights to 5e-4, moments to 1e-3 relative (the
    moment tolerance for this mode).  Moments are judged by their true
    relative error on the posterior's scale (mom_rel_err): E z against
    max(|E z|, sd), E z^2 against E z^2."""
    from paper_2503_08264_amd import _lib
    model = S.chain(0)
    K, seed, it, T = 256, 5, 2, 64
    picks = tuple(range(0, 1024, 16)) + (1023,)
    refs = {s: _series_reference(model, K, seed, it, s) for s in picks}
    rows = []
    bounds = {"fp64": (1e-10, 1e-12, 1e-10), "fp32": (1e-4, 2e-5, 1e-3), "bf16exp": (2e-4, 5e-4, 1e-3)}
    for prec in ("bf16exp", "fp32", "fp64"):
        g = gpu_run(model, K, prec, seed=seed, it=it)
        q = g["ctx"]
        Lg = q.tensor(0, _lib.T_ROOTL).cpu().numpy()
        w = g["w"][0].reshape(1024, T, K)
        mom = g["mone"][0].reshape(1024, T, 2)
        eL = max(rel_err(Lg[s], refs[s]["L64"]) for s in picks)
        ew = max(float(np.max(np.abs(w[s] - refs[s]["w64"]))) for s in picks)
        em = max(mom_rel_err(mom[s].reshape(T, 1, 2), refs[s]["mom64"].reshape(T, 1, 2)) for s in picks)
        rows.append((prec, eL, ew, em))
        q.close()
        del g
    say(f"[precision report] chain 1024 x 64, K=256, vs FP64 oracle ({len(picks)} series: every 16th and the last)")
    say("| mode | log P_MP rel err | weights max abs err | moments max rel err |")
    for prec, eL, ew, em in rows:
        say(f"| {prec} | {eL:.3e} | {ew:.3e} | {em:.3e} |")
    for prec, eL, ew, em in rows:
        bL, bw, bm = bounds[prec]
        assert eL <= bL and ew <= bw and em <= bm, (prec, eL, ew, em)
