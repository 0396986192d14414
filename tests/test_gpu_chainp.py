"""AR(1) chains under a K-sampled parent (appendix F's region x day chains)
against the oracle: each series eliminated once per sample of its parent,
the message over the parent's samples gathered into the parent, the reverse
pass summed over them.

Small cases compare every element: samples, unary factors, log P_MP, the
per-parent-sample messages, the messages into the parent, weights and
moments.  K = 16, 32, 64 and 128 take the exponential GEMMs on MFMA (one,
two and eight blocks per series); K = 12, 13 and 20 the per-sample VALU
kernels.  Also: the shortest chain (T = 2), a chain directly under the
single-instance root, series assigned to parent instances out of order (some
parents with none, some with several), a steep transition (variance 0.01)
whose steps exceed the GEMM's range bound at the initial proposal and take
the per-entry log-sum-exp, and a narrow initial proposal (variance 0.05)
whose FP32 steps run as FP32 GEMMs.  The full workload (92 regions x 109 days, K = 64)
compares the messages of sampled regions against the oracle run on that
region alone, with the samples of the full model's counters, and checks the
normalisation of every weight row.
"""
import numpy as np
import pytest

import qem_synth as S
from oracle import mpiw as M

from _parity import TOL, compare_estep, gpu_run, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu


def _under_root(seed, n_series=4, T=6):
    """Chains hanging directly under the single-instance root."""
    m = S.ar_regions(seed, n_regions=n_series, T=T)
    nodes = [m.nodes[0],
             S.Node("x", n_series * T, 1, "gauss", "normal", parents=(0,),
                    parent_index=np.zeros(n_series * T, np.int32), a=0.7, b=0.1,
                    var=0.2, chain_len=T, init_b=-0.2, init_var=0.4)]
    return S.Model("ar_under_root", nodes, [S.Obs(1, "gauss", m.obs[0].x, var=m.obs[0].var)], K=m.K)


def _shuffled(seed, n_regions=5, n_series=7, T=5):
    """Series assigned to region levels out of order: region 1 has none,
    others one or several."""
    m = S.ar_regions(seed, n_regions=n_regions, T=T)
    owner = np.array([3, 0, 4, 3, 2, 0, 3], np.int32)[:n_series]
    rng = np.random.default_rng(seed)
    y = m.obs[0].x.reshape(n_regions, T, 1, 1)[:1].repeat(n_series, 0)
    y = y + 0.3 * rng.normal(size=y.shape)
    m.nodes[2] = S.Node("x", n_series * T, 1, "gauss", "normal", parents=(1,),
                        parent_index=np.repeat(owner, T), a=0.8, b=0.0, var=0.1, chain_len=T, init_b=0.0,
                        init_var=0.3)
    m.obs[0] = S.Obs(2, "gauss", y.reshape(-1, 1, 1), var=m.obs[0].var)
    return m


def _tight(seed, n_regions=3, T=6):
    """A narrow initial proposal for the chain: small sample ranges per step."""
    m = S.ar_regions(seed, n_regions=n_regions, T=T)
    m.nodes[2].q0 = (0.0, 0.05)
    return m


SMALL = {
    "regions_k16": (lambda: S.ar_regions(3, n_regions=5, T=7), 16),
    "regions_k32": (lambda: S.ar_regions(12, n_regions=3, T=5), 32),
    "regions_k64": (lambda: S.ar_regions(13, n_regions=3, T=6), 64),
    "regions_k128": (lambda: S.ar_regions(14, n_regions=2, T=4), 128),
    "steep_k16": (lambda: S.ar_regions(15, n_regions=3, T=6, a=1.0, var=0.01), 16),
    "tight_k16": (lambda: _tight(19), 16),
    "regions_t2_k16": (lambda: S.ar_regions(22, n_regions=3, T=2), 16),
    "under_root_k32": (lambda: _under_root(23, n_series=3, T=5), 32),
    "tight_k64": (lambda: _tight(20), 64),
    "tight_k128": (lambda: _tight(21, n_regions=2, T=4), 128),
    "regions_ragged_k13": (lambda: S.ar_regions(4, n_regions=4, T=6), 13),
    "regions_t2": (lambda: S.ar_regions(5, n_regions=3, T=2), 12),
    "under_root": (lambda: _under_root(6), 20),
    "shuffled": (lambda: _shuffled(7), 16),
}


def _compare_chain_messages(g, o, v, T, prec):
    """Per-parent-sample messages (rows t >= 1) and the message into the parent."""
    from paper_2503_08264_amd import _lib
    q = g["ctx"]
    m_ref, _, L_ref = o["st"].msg[v]
    m = q.tensor(v, _lib.T_MSG).cpu().numpy()
    L = q.tensor(v, _lib.T_ROOTL).cpu().numpy()
    tol = TOL[prec]["logphat"]
    assert m.shape == m_ref.shape and L.shape == L_ref.shape
    assert rel_err(m[:, :, 1:], m_ref[:, :, 1:]) <= tol, rel_err(m[:, :, 1:], m_ref[:, :, 1:])
    assert rel_err(L, L_ref) <= tol, rel_err(L, L_ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(SMALL))
def test_chain_under_parent_estep_parity(name, prec):
    make, K = SMALL[name]
    model = make()
    v = len(model.nodes) - 1
    g = gpu_run(model, K, prec, seed=31, it=2)
    o = oracle_run(model, K, seed=31, it=2)
    compare_estep(g, o, prec)
    _compare_chain_messages(g, o, v, model.nodes[v].chain_len, prec)
    assert g["status"][0] == 0


def test_chain_under_parent_adjoint_scale():
    """The reverse pass scaled by g = 2.5 (the source-term identity): every
    weight, the chain's included, is 2.5 times the unscaled one."""
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model = S.ar_regions(8, n_regions=4, T=5)
    K = 16
    say("[gpu] chain under a parent: reverse pass scaled by 2.5, fp64")
    q = QEM(model, K, "fp64")
    q.sample(3, 1)
    q.logfactors()
    q.contract_fwd()
    q.contract_bwd()
    torch.cuda.synchronize()
    w1 = [q.tensor(v, _lib.T_W).cpu().numpy().copy() for v in range(3)]
    q.contract_bwd(torch.tensor([2.5], dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    for v in range(3):
        assert rel_err(q.tensor(v, _lib.T_W).cpu().numpy(), 2.5 * w1[v]) < 1e-14, v


@pytest.mark.parametrize("case", ["shuffled_k16", "steep_k32", "regions_k20"])
def test_chain_under_parent_loop_and_graph_vs_oracle(case):
    """Five iterations of Algorithm 1: qem_step, and qem_run's captured
    graph, against the oracle's loop (FP64).  The steep case starts on the
    per-entry path and moves to the GEMM as the proposal narrows."""
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model, K = {"shuffled_k16": (_shuffled(11), 16),
                "steep_k32": (S.ar_regions(16, n_regions=3, T=6, a=1.0, var=0.01), 32),
                "regions_k20": (S.ar_regions(17, n_regions=3, T=5), 20)}[case]
    say(f"[gpu] chain under a parent: QEM loop and graph vs oracle, {case} fp64")
    m_ref, hist_ref = M.qem(model, K, 5, 0.3, seed=4)
    q = QEM(model, K, "fp64")
    hist = q.run(5, 0.3, seed=4, record=True)
    assert rel_err(hist, hist_ref) < 1e-10, (hist, hist_ref)
    r = QEM(model, K, "fp64")
    r.run_graph(4, 1, 0.3, 5)
    assert rel_err(r.logphat(), hist_ref[-1]) < 1e-10
    for v in range(3):
        assert rel_err(q.tensor(v, _lib.T_MEMA).cpu().numpy(), m_ref[v]) < 1e-9, v
        assert rel_err(r.tensor(v, _lib.T_MEMA).cpu().numpy(), m_ref[v]) < 1e-9, v


def _region_model(model, r):
    """The workload restricted to region r: the root, region r's level and its chain."""
    T = model.nodes[2].chain_len
    sub = S.ar_regions(0, n_regions=1, T=T)
    sub.nodes[2].q0 = model.nodes[2].q0
    sub.obs[0] = S.Obs(2, "gauss", model.obs[0].x.reshape(-1, T, 1, 1)[r].reshape(-1, 1, 1),
                       var=model.obs[0].var)
    return sub


@pytest.mark.parametrize("prec,q0var", [("fp32", None), ("fp64", None), ("fp32", 0.05)])
def test_chain_under_parent_full_size_sampled_regions(prec, q0var):
    """92 regions x 109 days, K = 64, the fused step: the message of sampled
    regions into their level (and the per-sample messages of a few level
    samples) against the oracle on that region alone; every weight row of
    every node sums to 1.  With the narrow initial proposal the FP32 steps
    run as FP32 GEMMs."""
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model = S.ar_regions(0)
    if q0var is not None:
        model.nodes[2].q0 = (0.0, q0var)
    K, seed, it = 64, 17, 1
    R, T = model.nodes[1].n, model.nodes[2].chain_len
    say(f"[gpu] chain under a parent, full size {R}x{T} K={K} {prec}")
    q = QEM(model, K, prec)
    q.step(seed, it, 0.3)
    torch.cuda.synchronize()
    L = q.tensor(2, _lib.T_ROOTL).cpu().numpy()
    m = q.tensor(2, _lib.T_MSG)
    lp = q.logphat()
    flags, _, _ = q.read_status()
    assert flags == 0 and np.isfinite(lp)
    tol = TOL[prec]
    qs = M.q_init(model)
    for r in (0, 45, 91):
        sub = _region_model(model, r)
        zs = [M.sample_instances(model, qs, K, it, seed, 0, [0]),
              M.sample_instances(model, qs, K, it, seed, 1, [r]),
              M.sample_instances(model, qs, K, it, seed, 2, np.arange(r * T, (r + 1) * T))]
        us = M.unary(sub, M.q_init(sub), zs, K)
        st = M.contract(sub, zs, us)
        m_ref, _, L_ref = st.msg[2]
        assert rel_err(L[r], L_ref[0]) <= tol["logphat"], (r, rel_err(L[r], L_ref[0]))
        for kb in (0, 31, 63):
            mr = m[r, kb, 1:].cpu().numpy()
            assert rel_err(mr, m_ref[0, kb, 1:]) <= tol["logphat"], (r, kb)
    for v in range(3):
        w = q.tensor(v, _lib.T_W).double().cpu().numpy()
        np.testing.assert_allclose(w.sum(-1), 1.0, atol=1e-4 if prec == "fp32" else 1e-12)
