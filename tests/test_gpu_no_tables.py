"""Contexts created with QEM_CREATE_NO_TABLES, where the pairwise log-factor of
linear-Gaussian plates and chains is evaluated from the samples inside the
forward and reverse kernels instead of being kept as a K x K table per
instance, against contexts that keep the tables.

The recomputed factor is the same expression in the same precision and the
reductions run in the same order, so every output (samples, unary factors,
u-tilde, messages, weights, moments, EMA state, Q parameters, log P_MP and the
status word) must be the same bits, through the stage calls, through the fused
step, through the captured graph, and at the full benchmark size.
"""
import numpy as np
import pytest

import qem_synth as S

from _parity import say

pytestmark = pytest.mark.gpu

CASES = {
    "nested_dim4": (lambda: S.nested_gaussian(2, n_schools=5, n_classes=7, n_students=4), 64),
    "nested_k32_d3": (lambda: S.nested_gaussian(3, n_schools=4, n_classes=6, n_students=2, dim=3), 32),
    "nested_k128_d2": (lambda: S.nested_gaussian(4, n_schools=3, n_classes=5, n_students=2, dim=2), 128),
    "nested_k256_d1": (lambda: S.nested_gaussian(6, n_schools=3, n_classes=4, n_students=2, dim=1), 256),
    # 4096 class instances: the one-wave-per-instance plate kernels
    "nested_wpi1": (lambda: S.nested_gaussian(7, n_schools=128, n_classes=32, n_students=2, dim=2), 64),
    "chain_ragged": (lambda: S.chain(2, n_series=5, T=9), 20),
    "chain_k256": (lambda: S.chain(3, n_series=3, T=17), 256),
    "chain_k512": (lambda: S.chain(4, n_series=2, T=6), 512),
    # rows far below the step factor's bound: the bounded log-sum-exp's fallback
    "chain_tight": (lambda: S.chain(6, n_series=4, T=8, var=1e-3), 64),
}

KINDS = ("T_Z", "T_U", "T_UT", "T_MSG", "T_W", "T_MONE", "T_MEMA", "T_QPARAM")


def _pair(model, K, prec):
    from paper_2503_08264_amd.api import QEM
    a = QEM(model, K, prec, chain_tables=True)   # every table kept
    b = QEM(model, K, prec, tables=False)
    return a, b


def _recomputed_nodes(a, b, nv):
    """Nodes whose table the no-tables context does not keep (at least one)."""
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEMError
    out = []
    for v in range(nv):
        try:
            a.info(v, _lib.T_F)
        except QEMError:
            continue
        try:
            b.info(v, _lib.T_F)
        except QEMError:
            out.append(v)
    assert out, "no node runs without its table"
    assert b.nbytes < a.nbytes
    return out


def _assert_same(a, b, nv, tag, kinds=KINDS):
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEMError
    torch.cuda.synchronize()
    for name in kinds:
        kind = getattr(_lib, name)
        for v in range(nv):
            try:
                ta = a.tensor(v, kind)
            except QEMError:
                continue
            tb = b.tensor(v, kind)
            if kind == _lib.T_MSG and a.model.nodes[v].chain_len > 1:
                ta, tb = ta[:, 1:], tb[:, 1:]   # a chain's row 0 is not written
            assert torch.equal(ta, tb) or (ta.isnan() == tb.isnan()).all() and torch.equal(
                ta.nan_to_num(0.0), tb.nan_to_num(0.0)), (tag, name, v)
    assert a.read_status() == b.read_status(), tag


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_no_tables_stage_calls(name, prec):
    make, K = CASES[name]
    model = make()
    nv = len(model.nodes)
    say(f"[gpu] no-tables stage calls: {name} K={K} {prec}")
    a, b = _pair(model, K, prec)
    _recomputed_nodes(a, b, nv)
    for it in (1, 2):
        for q in (a, b):
            q.estep(7, it)
            q.mstep(0.4)
        _assert_same(a, b, nv, (name, prec, it))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_no_tables_fused_step(name, prec):
    make, K = CASES[name]
    model = make()
    nv = len(model.nodes)
    say(f"[gpu] no-tables fused step: {name} K={K} {prec}")
    a, b = _pair(model, K, prec)
    for it in (1, 2, 3):
        a.step(11, it, 0.3)
        b.step(11, it, 0.3)
        _assert_same(a, b, nv, (name, prec, it))


def test_no_tables_adjoint_scale():
    """The reverse pass scaled by a device-side d(loss)/d(log P_MP)."""
    import torch
    model = S.nested_gaussian(5, n_schools=4, n_classes=6, n_students=3)
    K = 64
    say("[gpu] no-tables reverse pass with an adjoint scale")
    a, b = _pair(model, K, "fp32")
    g = torch.tensor([-0.75], dtype=torch.float64, device="cuda")
    for q in (a, b):
        q.sample(3, 1)
        q.logfactors()
        q.contract_fwd()
        q.contract_bwd(g)
    _assert_same(a, b, len(model.nodes), "adjoint", ("T_Z", "T_U", "T_UT", "T_MSG", "T_W"))


def test_no_tables_graph_and_ema_options():
    """Graph replays with the Theorem 1 step and the second-sample normaliser."""
    model = S.nested_gaussian(8, n_schools=6, n_classes=5, n_students=3)
    K = 64
    say("[gpu] no-tables graph replay with EMA options")
    a, b = _pair(model, K, "fp32")
    for q in (a, b):
        q.set_ema(0.6, True)
        q.run_graph(13, 1, 0.5, 4)
    _assert_same(a, b, len(model.nodes), "graph")


def test_no_tables_full_size():
    """The benchmark hierarchy (256 schools x 32 classes, dim 4, K = 64, FP32):
    one fused step with and without the class-level table, compared whole."""
    import torch
    model = S.nested_gaussian(0)
    K = 64
    say("[gpu] no-tables full size: nested 256x32x16 dim 4 K=64 fp32")
    a, b = _pair(model, K, "fp32")
    rec = _recomputed_nodes(a, b, len(model.nodes))
    say(f"    recomputed nodes {rec}; workspace {a.nbytes >> 20} MiB -> {b.nbytes >> 20} MiB")
    for it in (1, 2):
        a.step(1000, it, 0.3)
        b.step(1000, it, 0.3)
        _assert_same(a, b, len(model.nodes), ("full", it))
    assert np.isfinite(b.read_status()[2])
    del a, b
    torch.cuda.empty_cache()

