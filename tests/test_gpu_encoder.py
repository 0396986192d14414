"""The encoder's hand-written kernels against the FP64 oracle, its training,
and what the learned initialisation gains over plain QEM.

The oracle receives the same host-generated master weights (and rounds them
to BF16 itself), computes its own features from the raw data and its own
forward pass, loss and backprop; nothing flows from the HIP path into it.
"""
import numpy as np
import pytest

import qem_synth as S
from oracle import encoder as E

from _parity import say

pytestmark = pytest.mark.gpu


def _enc_with(master_np):
    import torch
    from paper_2503_08264_amd.encoder import Encoder
    enc = Encoder(seed=0)
    enc.master.copy_(torch.as_tensor(master_np.astype(np.float32)))
    enc.lib.qem_enc_to_bf16(enc.master.data_ptr(), enc.w.data_ptr(), enc._s())
    return enc


def test_encoder_kernels_match_oracle():
    import torch
    say("[gpu] encoder kernels vs oracle")
    rng = np.random.default_rng(0)
    master = rng.normal(0, 0.25, E.NPARAM).astype(np.float32)
    enc = _enc_with(master)
    model = S.logistic(7, n_groups=300)
    ob = model.obs[0]
    feat = enc.features(ob.x, ob.cov)
    target = np.stack([rng.normal(size=300), rng.uniform(0.05, 2.0, size=300)], 1)
    tgt = torch.as_tensor(target, device="cuda")
    out, _ = enc.forward(feat)
    loss, grad = enc.loss_grad(feat, tgt)
    torch.cuda.synchronize()

    f_o = E.features(ob.x, ob.cov)
    np.testing.assert_allclose(feat.cpu().numpy(), f_o, rtol=1e-6, atol=1e-6)
    p = E.bf16_round(master)
    out_o, cache = E.forward(p, f_o)
    np.testing.assert_allclose(out.cpu().numpy(), out_o, rtol=1e-4, atol=1e-4)
    loss_o, d_o = E.kl_loss(out_o, target)
    assert abs(loss.item() - loss_o) < 1e-4 * max(1.0, abs(loss_o))
    g_o = E.backward(p, cache, d_o)
    g = grad.cpu().numpy()
    assert np.max(np.abs(g - g_o)) < 1e-3 * np.max(np.abs(g_o))


def test_encoder_adam_step_matches_oracle():
    import torch
    rng = np.random.default_rng(1)
    master = rng.normal(0, 0.25, E.NPARAM).astype(np.float32)
    enc = _enc_with(master)
    g1 = rng.normal(size=E.NPARAM).astype(np.float32)
    g2 = rng.normal(size=E.NPARAM).astype(np.float32)
    m_o, a, b = master.astype(np.float64), np.zeros(E.NPARAM), np.zeros(E.NPARAM)
    for step, g in ((1, g1), (2, g2)):
        enc.adam(torch.as_tensor(g, device="cuda"), lr=1e-2)
        m_o, a, b = E.adam(m_o, g.astype(np.float64), a, b, step, 1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(enc.master.cpu().numpy(), m_o, rtol=1e-5, atol=1e-6)
    w = enc.w.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    np.testing.assert_array_equal(w.view(np.float32), E.bf16_round(enc.master.cpu().numpy()).astype(np.float32))


def test_pool_context_and_residual_kernels_match_oracle():
    """The global head's pooled rows, the group encoder's context features and
    the residual apply against the oracle's definitions (the oracle pools its
    own FP64 summaries; the kernels pool the FP32 ones)."""
    import torch
    from paper_2503_08264_amd.encoder import Encoder
    say("[gpu] pooled rows / context features vs oracle")
    enc = Encoder(seed=0)
    model = S.logistic(7, n_groups=600)
    ob = model.obs[0]
    J = ob.x.shape[1]
    feat = enc.features(ob.x, ob.cov)
    rows = enc.pool(feat, J)
    ctx = enc.features_ctx(feat, rows, J)
    torch.cuda.synchronize()
    f_o = E.features(ob.x, ob.cov)
    rows_o = E.pool_rows(f_o, J)
    np.testing.assert_allclose(rows.cpu().numpy(), rows_o, rtol=2e-4, atol=2e-5)
    ctx_o = E.features_ctx(f_o, rows.cpu().numpy().astype(np.float64), J)
    np.testing.assert_allclose(ctx.cpu().numpy(), ctx_o, rtol=2e-5, atol=2e-5)
    out = torch.as_tensor(np.random.default_rng(2).normal(size=(9, 2)).astype(np.float32), device="cuda")
    qp = torch.empty((9, 2), dtype=torch.float64, device="cuda")
    enc.lib.qem_enc_apply_residual(out.data_ptr(), rows.data_ptr(), 9, qp.data_ptr(), enc._s())
    torch.cuda.synchronize()
    o, r = out.cpu().numpy().astype(np.float64), rows.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(qp.cpu().numpy(), np.stack([r[:, 1] + o[:, 0], np.exp(o[:, 1])], 1), rtol=1e-12)


def test_learned_init_gain_over_prior():
    """What the trained networks gain over the prior initialisation, judged
    by plain QEM.  Trained on the QEM posteriors of 16 training datasets and
    evaluated on a held-out one:
      - the group encoder's Q_0(b_i) is much closer (KL) to the held-out
        dataset's own QEM posterior than the prior N(0,1);
      - the global head's means of beta and log sigma are within a few
        posterior standard deviations, where the prior's mean is hundreds off;
      - the learned Q_0 has the higher log P_MP and marginal ESS at t = 0;
      - learned-init QEM reaches the band 1 nat below plain QEM's converged
        log P_MP (L*, checked flat over plain QEM's last 20 of 100 iterations)
        in under half of plain QEM's wall-clock time.  The 0.1-nat band sits
        inside the iteration-to-iteration fluctuation of the converged EMA at
        these R and training sizes, so it is reported here and judged by the
        multi-seed protocol of encoder.py (adaptive R to a 0.03-nat standard
        error, 64 training datasets)."""
    import torch
    from paper_2503_08264_amd import encoder as ENC
    say("[gpu] learned init vs plain")
    n, K, lam = 8192, 64, 0.3

    def make(s):
        return S.logistic(s, n_groups=n)

    enc = ENC.Encoder(seed=2)
    head = ENC.Encoder(seed=3)
    feat, target, grows, gtargets = ENC.training_set(make, range(100, 116), K, 120, lam, enc)
    hist = enc.train(feat, target, steps=800, log_every=100)
    ghist = head.train(grows, gtargets, steps=2500, log_every=500)
    assert hist[-1][1] < 0.05 * hist[0][1]
    held = make(0)
    q = ENC.plain_qem(held, K, 120, lam, seed=10_500)
    tgt = ENC.posterior_targets(q, 2)
    gt = ENC.global_targets(q).cpu().numpy()
    _, rows, ctx = ENC.dataset_inputs(enc, *q.obs_dev[0])
    kl_enc = enc.loss_grad(ctx, tgt)[0].item()
    prior_out = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    kl = torch.empty(n, dtype=torch.float64, device="cuda")
    dout = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    enc.lib.qem_enc_loss(prior_out.data_ptr(), tgt.data_ptr(), n, dout.data_ptr(), kl.data_ptr(),
                         loss.data_ptr(), enc._s())
    kl_prior = loss.item()
    out, _ = head.forward(rows)
    o, r = out.cpu().numpy().astype(np.float64), rows.cpu().numpy().astype(np.float64)
    z_head = (r[:, 1] + o[:, 0] - gt[:, 0]) / np.sqrt(gt[:, 1])
    z_prior = (0.0 - gt[:, 0]) / np.sqrt(gt[:, 1])
    say(f"[gpu] held-out KL of the group encoder {kl_enc:.3f} vs prior {kl_prior:.3f}; global head mean offsets "
        f"(posterior sds) {np.round(z_head, 1).tolist()} vs prior mean {np.round(z_prior, 0).tolist()}, "
        f"sd ratio {np.round(np.sqrt(np.exp(o[:, 1]) / gt[:, 1]), 2).tolist()}")
    q.close()
    assert kl_enc < 0.3 * kl_prior
    assert np.median(np.abs(z_head)) < 0.05 * np.median(np.abs(z_prior))
    res = ENC.evaluate(make, 0, enc, K, 100, lam, R=4, head=head)
    keys = ("L_star", "plain_iter", "learned_iter", "speedup", "plain_iter_1nat", "learned_iter_1nat",
            "speedup_1nat", "learned_choice", "init_scores", "learned_init_s", "plain_s_per_iter")
    say(f"[gpu] learned-init result: { {k: res[k] for k in keys} }")
    (lp_l, ess_l), (lp_p, ess_p) = res["init_scores"]["learned"], res["init_scores"]["prior"]
    assert res["learned_choice"] == "learned"
    assert lp_l > lp_p and ess_l > ess_p
    assert res["learned_iter_1nat"] is not None and res["plain_iter_1nat"] is not None
    # L* is plain QEM's converged score: its last 10 iterations within half a
    # nat of the 10 before them
    assert abs(res["plain_tail_drift"]) < 0.5, res["plain_tail_drift"]
    assert res["speedup_1nat"] > 2.0


def test_encoder_targets_kernel():
    """qem_enc_targets on synthetic mean parameters: (E z - plug-in,
    max(E z^2 - (E z)^2, floor)), against the definition in FP64 (the
    variance within the rounding of its one subtraction)."""
    import torch
    from paper_2503_08264_amd import _lib
    lib = _lib.load()
    rng = np.random.default_rng(4)
    n = 1000
    m1 = rng.normal(size=n)
    var = np.exp(rng.normal(-3, 2, size=n))
    var[:7] = 0.0                                  # point masses: the floor applies
    m = np.stack([m1, m1 * m1 + var], 1)
    rows = rng.normal(size=(n, 18)).astype(np.float32)
    md = torch.as_tensor(m, device="cuda")
    rd = torch.as_tensor(rows, device="cuda")
    out = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    for with_rows in (False, True):
        st = lib.qem_enc_targets(md.data_ptr(), n, 1e-8, rd.data_ptr() if with_rows else None, out.data_ptr(), None)
        assert st == 0
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        ref_mean = m1 - rows[:, 1].astype(np.float64) if with_rows else m1
        np.testing.assert_array_equal(o[:, 0], ref_mean)
        # E z^2 - (E z)^2 may be formed with one fused multiply-add: within
        # two roundings of E z^2
        ref_var = np.maximum(m[:, 1] - m1 * m1, 1e-8)
        assert np.all(np.abs(o[:, 1] - ref_var) <= 4.5e-16 * np.abs(m[:, 1])), np.max(np.abs(o[:, 1] - ref_var))
    assert lib.qem_enc_targets(md.data_ptr(), 0, 1e-8, None, out.data_ptr(), None) == _lib.QEM_E_SHAPE
