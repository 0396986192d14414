"""Categorical latents (QEM_Q_CATEGORICAL, one-hot over C categories) against
the oracle: a Gaussian mixture whose weights are a K-sampled Dirichlet
parent (the membership pair table log pi^kp[c], the plate contraction into
the weights, their (E z, E log z) moments) and memberships with a uniform
prior; the one-hot draws, unary factors, log P_MP, weights and moments of the
E-step, the clamped M-step, Algorithm 1 through qem_step and the captured
graph, and the full 2048-member workload."""
import numpy as np
import pytest

import qem_synth as S
from oracle import mpiw as M

from _parity import compare_estep, gpu_run, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu


def _flat(seed, n=9, C=4, J=5):
    """Memberships with a uniform prior (no weights node)."""
    m = S.mixture(seed, n_groups=n, C=C, n_obs=J)
    nodes = [S.Node("z", n, C, "categorical", "categorical", q0=(1.0 / C, 1.0))]
    return S.Model("flat_mixture", nodes, [S.Obs(0, "gauss_mixture", m.obs[0].x, var=m.obs[0].var,
                                                 cov=m.obs[0].cov)], None)


SMALL = {
    "mixture_c3_k13": (lambda: S.mixture(1, n_groups=11, C=3, n_obs=4), 13),
    "mixture_c4_k64": (lambda: S.mixture(2, n_groups=7, C=4, n_obs=6), 64),
    "flat_c4_k16": (lambda: _flat(3), 16),
    # 600 x 64 = 38400 child messages into the single weights instance: the
    # gather runs as one workgroup per subset, then the subset sums in order
    "mixture_wide_gather_k64": (lambda: S.mixture(4, n_groups=600, C=4, n_obs=3), 64),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(SMALL))
def test_categorical_estep_parity(name, prec):
    make, K = SMALL[name]
    model = make()
    g = gpu_run(model, K, prec, seed=66, it=2)
    o = oracle_run(model, K, seed=66, it=2)
    compare_estep(g, o, prec)
    assert g["status"][0] == 0
    z = g["z"][-1]
    assert np.all((z == 0.0) | (z == 1.0)) and np.all(z.sum(-1) == 1.0)


def test_categorical_stage_mstep_matches_oracle():
    """EMA and the clamped M-step of the memberships and the weights."""
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model, K = SMALL["mixture_c3_k13"][0](), 13
    seed, it, lam = 21, 1, 0.5
    say("[gpu] categorical EMA + M-step vs oracle")
    q = QEM(model, K, "fp64")
    q.estep(seed, it)
    q.mstep(lam)
    torch.cuda.synchronize()
    qs0 = M.q_init(model)
    zs = M.sample(model, qs0, K, it, seed)
    _, _, m_one = M.estep(model, qs0, zs, K)
    m = M.ema(M.mean_params(model, qs0), m_one, lam)
    qs, hits = M.set_params(model, m)
    for v in range(2):
        assert rel_err(q.tensor(v, _lib.T_MEMA).cpu().numpy(), m[v]) < 1e-12, v
    assert rel_err(q.tensor(1, _lib.T_QPARAM).cpu().numpy()[..., 0], qs[1]["p"]) < 1e-12
    assert rel_err(q.tensor(0, _lib.T_QPARAM).cpu().numpy()[..., 0], qs[0]["alpha"]) < 1e-9
    assert q.read_status()[1] == hits


@pytest.mark.parametrize("name", ["mixture_c3_k13", "flat_c4_k16"])
def test_categorical_qem_loop_and_graph_vs_oracle(name):
    """Six iterations of Algorithm 1 through qem_step and through qem_run."""
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    make, K = SMALL[name]
    model = make()
    nv = len(model.nodes)
    say(f"[gpu] categorical QEM loop and graph vs oracle: {name} fp64")
    m_ref, hist_ref = M.qem(model, K, 6, 0.3, seed=9)
    q = QEM(model, K, "fp64")
    hist = q.run(6, 0.3, seed=9, record=True)
    assert rel_err(hist, hist_ref) < 1e-10, (hist, hist_ref)
    r = QEM(model, K, "fp64")
    r.run_graph(9, 1, 0.3, 6)
    assert rel_err(r.logphat(), hist_ref[-1]) < 1e-10
    for v in range(nv):
        assert rel_err(q.tensor(v, _lib.T_MEMA).cpu().numpy(), m_ref[v]) < 1e-9, v
        assert rel_err(r.tensor(v, _lib.T_MEMA).cpu().numpy(), m_ref[v]) < 1e-9, v


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_categorical_full_size(prec):
    """2048 memberships, C = 4, 10 observations each, K = 64: every element
    of the E-step against the oracle."""
    model = S.mixture(0)
    say(f"[gpu] mixture full size 2048 x C=4, K=64, {prec}")
    g = gpu_run(model, 64, prec, seed=4, it=1)
    o = oracle_run(model, 64, seed=4, it=1)
    compare_estep(g, o, prec)
