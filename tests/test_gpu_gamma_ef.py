"""The exponential-family Gamma proposal (QEM_Q_GAMMA_EF) against the oracle:
moments of (z, log z), the initial mean parameters (E z, E log z), the
M-step that solves log shape - psi(shape) = log m1 - m2, and Algorithm 1 on
the Gamma-Poisson hierarchy with every latent in that family."""
import numpy as np
import pytest
from scipy.special import digamma

import qem_synth as S
from oracle import mpiw as M

from _parity import compare_estep, gpu_run, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu


def _model(n=9, J=7, seed=4):
    return S.gamma_poisson(seed, n_groups=n, n_obs=J, qfamily="gamma_ef")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ef_estep_parity(prec):
    model = _model()
    say(f"[gpu] exponential-family Gamma E-step parity, {prec}")
    g = gpu_run(model, 12, prec, seed=1234, it=2)
    o = oracle_run(model, 12, seed=1234, it=2)
    compare_estep(g, o, prec)
    assert g["status"][0] == 0


def test_ef_init_and_mstep_over_a_wide_range():
    """Device digamma in the initial mean parameters, and the device shape
    solve in the M-step, over shapes from 0.02 to 2000: mean parameters
    against scipy's digamma, and the M-step on exact mean parameters gives
    the shapes back."""
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    n = 64
    model = _model(n=n, J=3)
    say("[gpu] exponential-family Gamma init and M-step, shapes 0.02..2000")
    q = QEM(model, 8, "fp64")
    rng = np.random.default_rng(3)
    shape = np.exp(rng.uniform(np.log(0.02), np.log(2000.0), size=n))
    rate = np.exp(rng.uniform(np.log(0.01), np.log(100.0), size=n))
    qp = q.tensor(2, _lib.T_QPARAM)
    qp.copy_(torch.tensor(np.stack([shape, rate], -1)[:, None, :], dtype=torch.float64, device="cuda"))
    q.init_from_q(2)
    torch.cuda.synchronize()
    mema = q.tensor(2, _lib.T_MEMA).cpu().numpy()[:, 0, :]
    ref = np.stack([shape / rate, digamma(shape) - np.log(rate)], -1)
    assert np.max(np.abs(mema - ref) / np.maximum(np.abs(ref), 1.0)) < 1e-14
    # lam = 0 keeps m_{t-1}; the M-step then maps it back to (shape, rate)
    q.mstep(0.0)
    torch.cuda.synchronize()
    back = q.tensor(2, _lib.T_QPARAM).cpu().numpy()[:, 0, :]
    assert rel_err(back[:, 0], shape) < 1e-11, rel_err(back[:, 0], shape)
    assert rel_err(back[:, 1], rate) < 1e-11
    flags, hits, _ = q.read_status()
    assert hits == 0


def test_ef_stage_mstep_matches_oracle():
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model = _model()
    K, seed, it, lam = 16, 77, 1, 0.35
    say("[gpu] exponential-family Gamma EMA + M-step vs oracle")
    q = QEM(model, K, "fp64")
    q.estep(seed, it)
    q.mstep(lam)
    torch.cuda.synchronize()
    qs0 = M.q_init(model)
    zs = M.sample(model, qs0, K, it, seed)
    _, _, m_one = M.estep(model, qs0, zs, K)
    m = M.ema(M.mean_params(model, qs0), m_one, lam)
    qs, hits = M.set_params(model, m)
    for v in range(3):
        got = q.tensor(v, _lib.T_QPARAM).cpu().numpy()
        assert rel_err(got[..., 0], qs[v]["shape"]) < 1e-10, v
        assert rel_err(got[..., 1], qs[v]["rate"]) < 1e-10, v
        assert rel_err(q.tensor(v, _lib.T_MEMA).cpu().numpy(), m[v]) < 1e-12, v


def test_ef_qem_loop_vs_oracle_fp64():
    """Six iterations of Algorithm 1 through qem_step and through qem_run."""
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model = _model()
    K = 12
    say("[gpu] exponential-family Gamma QEM loop vs oracle, fp64")
    m_ref, hist_ref = M.qem(model, K, 6, 0.3, seed=21)
    q = QEM(model, K, "fp64")
    hist = q.run(6, 0.3, seed=21, record=True)
    assert rel_err(hist, hist_ref) < 1e-10, (hist, hist_ref)
    for v in range(3):
        assert rel_err(q.tensor(v, _lib.T_MEMA).cpu().numpy(), m_ref[v]) < 1e-9, v
    r = QEM(model, K, "fp64")
    r.run_graph(21, 1, 0.3, 6)
    assert rel_err(r.logphat(), hist_ref[-1]) < 1e-10
    for v in range(3):
        assert rel_err(r.tensor(v, _lib.T_MEMA).cpu().numpy(), m_ref[v]) < 1e-9, v


def _gamma_root_model():
    """A single-instance exponential-family Gamma root r ~ Gamma(2, 1) with a
    plate of Gaussian children c_i ~ N(r, 0.5) observed with noise: the fused
    iteration finishes the root (moments of (z, log z) and its M-step) in the
    root finisher."""
    rng = np.random.default_rng(17)
    r = rng.gamma(2.0, 1.0)
    c = r + np.sqrt(0.5) * rng.normal(size=(6, 1))
    x = c[:, None, :] + rng.normal(size=(6, 4, 1))
    nodes = [S.Node("r", 1, 1, "gamma_ef", "gamma", shape=2.0, rate=1.0, q0=(2.0, 1.0)),
             S.Node("c", 6, 1, "gauss", "normal", parents=(0,), parent_index=np.zeros(6, np.int32),
                    a=1.0, b=0.0, var=0.5, q0=(1.0, 1.0))]
    return S.Model("gamma_root", nodes, [S.Obs(1, "gauss", x, var=1.0)], K=16)


def test_ef_root_finisher_vs_oracle():
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model = _gamma_root_model()
    K = 16
    say("[gpu] exponential-family Gamma root through the root finisher, fp64")
    m_ref, hist_ref = M.qem(model, K, 5, 0.3, seed=8)
    q = QEM(model, K, "fp64")
    hist = q.run(5, 0.3, seed=8, record=True)
    assert rel_err(hist, hist_ref) < 1e-10, (hist, hist_ref)
    for v in range(2):
        assert rel_err(q.tensor(v, _lib.T_MEMA).cpu().numpy(), m_ref[v]) < 1e-9, v
