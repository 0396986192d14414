"""Dirichlet latents (QEM_Q_DIRICHLET; Beta as C = 2) with categorical
observations against the oracle: samples (the Gamma draws normalised in log
space), unary factors, log P_MP, weights and the (E z, E log z) moments of
the E-step; the initial mean parameters and the M-step solve over a wide
range of concentrations; the floored degenerate case; Algorithm 1 through
qem_step and the captured graph; and the full 4096-group workload."""
import numpy as np
import pytest
from scipy.special import digamma

import qem_synth as S
from oracle import mpiw as M

from _parity import compare_estep, gpu_run, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

SMALL = {
    "beta_k13": (lambda: S.dirichlet_categorical(1, n_groups=7, C=2, n_obs=9, shape=0.8), 13),
    "c3_k16": (lambda: S.dirichlet_categorical(2, n_groups=9, C=3, n_obs=12, shape=1.0), 16),
    "c5_k64": (lambda: S.dirichlet_categorical(3, n_groups=5, C=5, n_obs=20, shape=0.4), 64),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(SMALL))
def test_dirichlet_estep_parity(name, prec):
    make, K = SMALL[name]
    model = make()
    g = gpu_run(model, K, prec, seed=55, it=2)
    o = oracle_run(model, K, seed=55, it=2)
    compare_estep(g, o, prec)
    assert g["status"][0] == 0
    # every sample on the simplex
    z = g["z"][0]
    assert np.max(np.abs(z.sum(-1) - 1.0)) < (1e-14 if prec == "fp64" else 2e-6)


def _q(model, K, prec="fp64"):
    from paper_2503_08264_amd.api import QEM
    return QEM(model, K, prec)


def test_dirichlet_init_and_mstep_over_a_wide_range():
    """Device digamma in the initial mean parameters, and the device solve in
    the M-step, over concentrations from 0.05 to 500 with C = 2, 3 and 6:
    mean parameters against scipy's digamma; the M-step on them returns the
    concentrations."""
    import torch
    from paper_2503_08264_amd import _lib
    rng = np.random.default_rng(5)
    for C in (2, 3, 6):
        n = 48
        model = S.dirichlet_categorical(4, n_groups=n, C=C, n_obs=3)
        say(f"[gpu] Dirichlet init and M-step, C={C}")
        q = _q(model, 8)
        alpha = np.exp(rng.uniform(np.log(0.05), np.log(500.0), size=(n, C)))
        qp = q.tensor(0, _lib.T_QPARAM)
        qp.copy_(torch.tensor(np.stack([alpha, np.ones_like(alpha)], -1), dtype=torch.float64, device="cuda"))
        q.init_from_q(0)
        torch.cuda.synchronize()
        mema = q.tensor(0, _lib.T_MEMA).cpu().numpy()
        a0 = alpha.sum(-1, keepdims=True)
        assert rel_err(mema[..., 0], alpha / a0) < 1e-14
        assert rel_err(mema[..., 1], digamma(alpha) - digamma(a0)) < 1e-13
        q.mstep(0.0)
        torch.cuda.synchronize()
        back = q.tensor(0, _lib.T_QPARAM).cpu().numpy()
        assert rel_err(back[..., 0], alpha) < 1e-9, (C, rel_err(back[..., 0], alpha))
        assert np.all(back[..., 1] == 1.0)
        flags, hits, _ = q.read_status()
        assert hits == 0 and flags == 0


def test_dirichlet_degenerate_mean_parameters_are_floored():
    """sum_c exp(E log z_c) >= 1 has no Dirichlet: the M-step counts a floor
    hit per instance and solves the floored parameters: psi(alpha_c) -
    psi(alpha_0) equals them to FP64 rounding.  At the floor gap (1e-12) the
    concentrations are ~1e11 and set by the gap alone, which FP64 knows to
    ~1e-4 relative, so the oracle's root agrees to that."""
    import torch
    from paper_2503_08264_amd import _lib
    model = S.dirichlet_categorical(5, n_groups=2, C=3, n_obs=3)
    q = _q(model, 8)
    L = np.log(np.array([[0.3, 0.3, 0.4], [0.2, 0.5, 0.31]]))
    mp = np.stack([np.exp(L), L], -1)
    q.tensor(0, _lib.T_MEMA).copy_(torch.tensor(mp, dtype=torch.float64, device="cuda"))
    q.mstep(0.0)
    torch.cuda.synchronize()
    flags, hits, _ = q.read_status()
    assert hits == 2 and (flags & 0x4) == 0
    ref, rh = M.set_params(model, [mp])
    assert rh == 2
    a = q.tensor(0, _lib.T_QPARAM).cpu().numpy()[..., 0]
    Lf = L - (np.log(np.exp(L).sum(-1, keepdims=True)) - np.log1p(-M.DIR_GAP_FLOOR))
    assert np.max(np.abs(digamma(a) - digamma(a.sum(-1, keepdims=True)) - Lf)) < 1e-12
    assert rel_err(a, ref[0]["alpha"]) < 1e-2


def test_dirichlet_stage_mstep_matches_oracle():
    import torch
    from paper_2503_08264_amd import _lib
    model, K = SMALL["c3_k16"][0](), 16
    seed, it, lam = 91, 1, 0.35
    say("[gpu] Dirichlet EMA + M-step vs oracle")
    q = _q(model, K)
    q.estep(seed, it)
    q.mstep(lam)
    torch.cuda.synchronize()
    qs0 = M.q_init(model)
    zs = M.sample(model, qs0, K, it, seed)
    _, _, m_one = M.estep(model, qs0, zs, K)
    m = M.ema(M.mean_params(model, qs0), m_one, lam)
    qs, _ = M.set_params(model, m)
    assert rel_err(q.tensor(0, _lib.T_MEMA).cpu().numpy(), m[0]) < 1e-12
    assert rel_err(q.tensor(0, _lib.T_QPARAM).cpu().numpy()[..., 0], qs[0]["alpha"]) < 1e-9


@pytest.mark.parametrize("name", ["beta_k13", "c5_k64"])
def test_dirichlet_qem_loop_and_graph_vs_oracle(name):
    """Six iterations of Algorithm 1 through qem_step and through qem_run."""
    from paper_2503_08264_amd import _lib
    make, K = SMALL[name]
    model = make()
    say(f"[gpu] Dirichlet QEM loop and graph vs oracle: {name} fp64")
    m_ref, hist_ref = M.qem(model, K, 6, 0.3, seed=12)
    q = _q(model, K)
    hist = q.run(6, 0.3, seed=12, record=True)
    assert rel_err(hist, hist_ref) < 1e-10, (hist, hist_ref)
    assert rel_err(q.tensor(0, _lib.T_MEMA).cpu().numpy(), m_ref[0]) < 1e-9
    r = _q(model, K)
    r.run_graph(12, 1, 0.3, 6)
    assert rel_err(r.logphat(), hist_ref[-1]) < 1e-10
    assert rel_err(r.tensor(0, _lib.T_MEMA).cpu().numpy(), m_ref[0]) < 1e-9


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_dirichlet_full_size(prec):
    """4096 groups, C = 4, 20 draws each, K = 64: every element of the E-step
    against the oracle (the groups are independent and the oracle's E-step
    is linear in the number of groups)."""
    model = S.dirichlet_categorical(0)
    say(f"[gpu] Dirichlet full size 4096 x C=4, K=64, {prec}")
    g = gpu_run(model, 64, prec, seed=3, it=1)
    o = oracle_run(model, 64, seed=3, it=1)
    compare_estep(g, o, prec)
    np.testing.assert_allclose(g["w"][0].sum(-1), 1.0, atol=1e-5 if prec == "fp32" else 1e-12)
