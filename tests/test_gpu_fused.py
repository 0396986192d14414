"""The fused iteration (qem_step: sampling with the unary factor, the
linear-Gaussian pair table inside the plate forward kernel, moments inside
the plate backward kernel, one M-step launch for all nodes) against
the six stage calls made one by one, and a few iterations of it against the
oracle's Algorithm 1.

From the same parameters, samples, factors (pair tables included), u-tilde,
weights and log P_MP are the same bits either way; the fused moments add the same FP64 terms in
another fixed order, so moments and the updated parameters agree to a few
ulps, and both contexts are set to the same parameters before the next
iteration.
"""
import numpy as np
import pytest

import qem_synth as S
from oracle import mpiw as M

from _parity import rel_err, say

pytestmark = pytest.mark.gpu

def _shuffled(seed):
    m = S.nested_gaussian(seed, n_schools=6, n_classes=5, n_students=3, dim=4)
    rng = np.random.default_rng(seed)
    m.nodes[2].parent_index = rng.permutation(m.nodes[2].parent_index).astype(np.int32)
    return m


def _tight_ar(seed):
    """AR chains with a narrow initial proposal (FP32 steps as FP32 GEMMs)."""
    m = S.ar_regions(seed, n_regions=4, T=7)
    m.nodes[2].q0 = (0.0, 0.05)
    return m


CASES = {
    "normal_normal": (lambda: S.normal_normal(3), 8),
    "nested_ragged": (lambda: S.nested_gaussian(1, n_schools=6, n_classes=5, n_students=3, dim=3), 13),
    "nested_dim4": (lambda: S.nested_gaussian(2, n_schools=5, n_classes=7, n_students=4), 64),
    "nested_k32_d3": (lambda: S.nested_gaussian(3, n_schools=4, n_classes=6, n_students=2, dim=3), 32),
    "nested_k128_d2": (lambda: S.nested_gaussian(4, n_schools=3, n_classes=5, n_students=2, dim=2), 128),
    # K = 64 leaf plates of dimension 1 and 3: the class draws inside the
    # class-level forward (odd dimensions share Box-Muller pairs across samples)
    "nested_k64_d1": (lambda: S.nested_gaussian(11, n_schools=4, n_classes=6, n_students=2, dim=1), 64),
    "nested_k64_d3": (lambda: S.nested_gaussian(12, n_schools=4, n_classes=6, n_students=2, dim=3), 64),
    "chain_ragged": (lambda: S.chain(2, n_series=5, T=9), 20),
    "gamma_poisson": (lambda: S.gamma_poisson(4, n_groups=9, n_obs=7), 12),
    "gamma_poisson_ef": (lambda: S.gamma_poisson(4, n_groups=9, n_obs=7, qfamily="gamma_ef"), 12),
    "logistic": (lambda: S.logistic(5, n_groups=6, n_obs=10, D=3), 11),
    "occupancy": (lambda: S.occupancy(2, n_sites=30, n_visits=4), 12),
    # a root with more than 32768 child messages: the root gather as one workgroup per subset
    "occupancy_wide": (lambda: S.occupancy(7, n_sites=1200, n_visits=4), 32),
    "tiny_tree": (lambda: S.tiny_tree(1, K=5), 5),
    # classes assigned to schools out of order: the indexed child gather
    "nested_shuffled": (lambda: _shuffled(9), 64),
    # 4096 class instances: the one-wave-per-instance plate kernels
    "nested_wpi1": (lambda: S.nested_gaussian(7, n_schools=128, n_classes=32, n_students=2, dim=2), 64),
    # AR(1) chains under a sampled region level, ragged K
    "ar_regions": (lambda: S.ar_regions(3, n_regions=6, T=7), 13),
    "ar_regions_k64": (lambda: S.ar_regions(4, n_regions=5, T=8), 64),
    "ar_regions_tight_k64": (lambda: _tight_ar(5), 64),
    # Dirichlet latents with categorical counts (moments of (z, log z), per-instance M-step)
    "dirichlet_c3": (lambda: S.dirichlet_categorical(6, n_groups=11, C=3, n_obs=10), 16),
    # categorical memberships under K-sampled Dirichlet mixture weights
    "mixture_c4": (lambda: S.mixture(8, n_groups=13, C=4, n_obs=5), 16),
    # two-parent contraction on MFMA (FP32; FP64 runs the exact kernels)
    "gamma_poisson_k64": (lambda: S.gamma_poisson(9, n_groups=10, n_obs=6), 64),
    "logistic_k64": (lambda: S.logistic(10, n_groups=8, n_obs=6, D=3), 64),
}


def _snapshot(q, nv):
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEMError
    torch.cuda.synchronize()
    get = lambda v, k: q.tensor(v, k).double().cpu().numpy().copy()

    def table(v):
        try:
            return get(v, _lib.T_F)
        except QEMError:   # no materialised pair table for this node
            return np.zeros(0)
    return {
        "exact": {**{k: [get(v, kind) for v in range(nv)] for k, kind in
                     (("z", _lib.T_Z), ("u", _lib.T_U), ("ut", _lib.T_UT), ("w", _lib.T_W))},
                  "F": [table(v) for v in range(nv)]},
        "close": {k: [get(v, kind) for v in range(nv)] for k, kind in
                  (("mone", _lib.T_MONE), ("mema", _lib.T_MEMA), ("qp", _lib.T_QPARAM))},
        "status": q.read_status(),
    }


def _resync(a, b, nv):
    """Start the next iteration of both contexts from the same parameters
    (the fused moments may differ from the stage call's in the last ulp)."""
    import torch
    from paper_2503_08264_amd import _lib
    for v in range(nv):
        for kind in (_lib.T_MEMA, _lib.T_QPARAM):
            a.tensor(v, kind).copy_(b.tensor(v, kind))
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_fused_step_equals_stage_calls(name, prec):
    from paper_2503_08264_amd.api import QEM
    make, K = CASES[name]
    model = make()
    nv = len(model.nodes)
    seed, lam = 99, 0.4
    say(f"[gpu] fused step vs stage calls: {name} K={K} {prec}")
    a = QEM(model, K, prec)
    b = QEM(model, K, prec)
    for it in (1, 2, 3):
        a.step(seed, it, lam)
        b.sample(seed, it)
        b.logfactors()
        b.contract_fwd()
        b.contract_bwd()
        b.moments()
        b.mstep(lam)
        sa, sb = _snapshot(a, nv), _snapshot(b, nv)
        assert sa["status"] == sb["status"], (it, sa["status"], sb["status"])
        for key in sa["exact"]:
            for v in range(nv):
                assert np.array_equal(sa["exact"][key][v], sb["exact"][key][v], equal_nan=True), (it, key, v)
        for key in sa["close"]:
            for v in range(nv):
                assert rel_err(sa["close"][key][v], sb["close"][key][v]) < 1e-13, (it, key, v)
        _resync(a, b, nv)


def test_fused_bexp_chain_step_equals_stage_calls():
    from paper_2503_08264_amd.api import QEM
    model = S.chain(3, n_series=4, T=11)
    K, seed, lam = 64, 5, 0.3
    say("[gpu] fused step vs stage calls: chain bf16exp")
    a = QEM(model, K, "bf16exp")
    b = QEM(model, K, "bf16exp")
    for it in (1, 2):
        a.step(seed, it, lam)
        b.sample(seed, it)
        b.logfactors()
        b.contract_fwd()
        b.contract_bwd()
        b.moments()
        b.mstep(lam)
        sa, sb = _snapshot(a, 1), _snapshot(b, 1)
        assert sa["status"] == sb["status"]
        for key in sa["exact"]:
            assert np.array_equal(sa["exact"][key][0], sb["exact"][key][0]), (it, key)
        for key in sa["close"]:
            assert rel_err(sa["close"][key][0], sb["close"][key][0]) < 1e-13, (it, key)
        _resync(a, b, 1)


@pytest.mark.parametrize("name", ["nested_dim4", "gamma_poisson", "logistic", "ar_regions"])
def test_fused_qem_loop_vs_oracle_fp64(name):
    """Six iterations of Algorithm 1 through qem_step against the oracle's loop."""
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    make, K = CASES[name]
    model = make()
    say(f"[gpu] fused QEM loop vs oracle: {name} K={K} fp64")
    q = QEM(model, K, "fp64")
    hist = q.run(6, 0.3, seed=21, record=True)
    m_ref, hist_ref = M.qem(model, K, 6, 0.3, seed=21)
    assert rel_err(hist, hist_ref) < 1e-10, (hist, hist_ref)
    for v in range(len(model.nodes)):
        assert rel_err(q.tensor(v, _lib.T_MEMA).cpu().numpy(), m_ref[v]) < 1e-9, v
