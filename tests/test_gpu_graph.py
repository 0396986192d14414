"""qem_run (one iteration, and eight in a row, captured as HIP graphs,
replayed with a device iteration counter) against eager qem_step calls,
replay by replay, with other eager GPU work and synchronisations between the
replays."""
import numpy as np
import pytest

import qem_synth as S

from _parity import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replays_equal_eager_steps(prec):
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model = S.nested_gaussian(2, n_schools=16, n_classes=8, n_students=4)
    K, seed, lam = 32, 11, 0.3
    say(f"[gpu] graph replay vs eager, {prec}")
    a = QEM(model, K, prec)
    b = QEM(model, K, prec)

    def state(q):
        torch.cuda.synchronize()
        return ([q.tensor(v, _lib.T_MEMA).cpu().numpy().copy() for v in range(3)],
                [q.tensor(v, _lib.T_W).cpu().numpy().copy() for v in range(3)], q.logphat())

    for t in range(1, 5):
        a.step(seed, t, lam)
        b.run_graph(seed, t, lam, 1)
        junk = torch.randn(1 << 16, device="cuda").square().sum()   # unrelated eager work
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        ma, wa, la = state(a)
        mb, wb, lb = state(b)
        assert la == lb, (t, la, lb)
        for x, y in zip(ma + wa, mb + wb):
            assert np.array_equal(x, y), t
    # several replays in one call continue the iteration numbering
    for t in range(5, 8):
        a.step(seed, t, lam)
    b.run_graph(seed, 5, lam, 3)
    ma, wa, la = state(a)
    mb, wb, lb = state(b)
    assert la == lb
    for x, y in zip(ma + wa, mb + wb):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_eight_iteration_graph_equals_eager_steps(prec):
    """11 iterations per call: one replay of the eight-iteration graph and
    three of the one-iteration graph; two calls with eager work between."""
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model = S.nested_gaussian(4, n_schools=12, n_classes=6, n_students=3)
    K, seed, lam = 64, 23, 0.25
    say(f"[gpu] eight-iteration graph vs eager, {prec}")
    a = QEM(model, K, prec)
    b = QEM(model, K, prec)
    for call in range(2):
        t0 = 1 + 11 * call
        for t in range(t0, t0 + 11):
            a.step(seed, t, lam)
        b.run_graph(seed, t0, lam, 11)
        junk = torch.randn(1 << 16, device="cuda").square().sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert a.logphat() == b.logphat(), call
        for v in range(3):
            for kind in (_lib.T_MEMA, _lib.T_QPARAM, _lib.T_W):
                assert torch.equal(a.tensor(v, kind), b.tensor(v, kind)), (call, v, kind)


def test_rebinding_the_workspace_recaptures_the_graphs():
    """After qem_bind_workspace moves the context to a new buffer, qem_run
    must not replay graphs that address the old one: the new buffer holds
    the same bits as eager qem_step calls, and the old buffer is left as it
    was."""
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model = S.nested_gaussian(5, n_schools=8, n_classes=6, n_students=3)
    K, seed, lam = 32, 31, 0.3
    say("[gpu] rebind workspace, then qem_run")
    a = QEM(model, K, "fp64")
    b = QEM(model, K, "fp64")
    b.run_graph(seed, 1, lam, 3)                 # graphs captured on the first buffer
    torch.cuda.synchronize()
    old = b.ws
    old_copy = old.clone()
    b.bind_workspace()                           # back to Q_0 on a second buffer
    assert b.ws.data_ptr() != old.data_ptr()
    for t in range(1, 4):
        a.step(seed, t, lam)
    b.run_graph(seed, 1, lam, 3)
    torch.cuda.synchronize()
    assert a.logphat() == b.logphat()
    for v in range(3):
        for kind in (_lib.T_MEMA, _lib.T_QPARAM, _lib.T_W):
            assert torch.equal(a.tensor(v, kind), b.tensor(v, kind)), (v, kind)
    assert torch.equal(old, old_copy)
