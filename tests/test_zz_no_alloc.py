"""qem_enc_bwd_noalloc (the encoder's backward pass with its partial
gradients in the library's own device array) against qem_enc_bwd with a
caller scratch buffer, through the C ABI: the same kernels in the same order,
so the gradients must be the same bits.  Two calls in a row, the second on a
smaller batch, so stale partials of the first call would show; then the
oracle's backprop on the second batch, and the host-side rejections."""
import ctypes

import numpy as np
import pytest

import qem_synth as S
from oracle import encoder as E

from _parity import say

pytestmark = pytest.mark.gpu


def _grads(enc, feat, target, noalloc):
    import torch
    n = feat.shape[0]
    out, act = enc.forward(feat, keep_act=True)
    dout = torch.empty((n, 2), dtype=torch.float32, device=enc.device)
    kl = torch.empty(n, dtype=torch.float64, device=enc.device)
    st = enc.lib.qem_enc_loss(out.data_ptr(), target.data_ptr(), n, dout.data_ptr(), kl.data_ptr(), None, enc._s())
    assert st == 0
    grad = torch.full((E.NPARAM,), float("nan"), dtype=torch.float32, device=enc.device)
    if noalloc:
        st = enc.lib.qem_enc_bwd_noalloc(enc.w.data_ptr(), feat.data_ptr(), act.data_ptr(), dout.data_ptr(), n,
                                         grad.data_ptr(), enc._s())
    else:
        scratch = torch.empty(int(enc.lib.qem_enc_scratch_bytes(n)) // 4 + 1, dtype=torch.float32,
                              device=enc.device)
        st = enc.lib.qem_enc_bwd(enc.w.data_ptr(), feat.data_ptr(), act.data_ptr(), dout.data_ptr(), n,
                                 grad.data_ptr(), scratch.data_ptr(), enc._s())
    assert st == 0, enc.lib.qem_last_error(None)
    torch.cuda.synchronize()
    return grad.cpu().numpy(), out


def test_noalloc_bwd_matches_workspace_bwd():
    import torch
    from paper_2503_08264_amd.encoder import Encoder
    rng = np.random.default_rng(11)
    master = rng.normal(0, 0.25, E.NPARAM).astype(np.float32)
    enc = Encoder(seed=0)
    enc.master.copy_(torch.as_tensor(master))
    assert enc.lib.qem_enc_to_bf16(enc.master.data_ptr(), enc.w.data_ptr(), enc._s()) == 0
    # 1000 groups (32 chunks, a ragged last one), then 77 (3 chunks)
    for n, seed in ((1000, 3), (77, 4)):
        say(f"[gpu] qem_enc_bwd_noalloc n={n}")
        model = S.logistic(seed, n_groups=n)
        ob = model.obs[0]
        feat = enc.features(ob.x, ob.cov)
        target_np = np.stack([rng.normal(size=n), rng.uniform(0.05, 2.0, size=n)], 1)
        target = torch.as_tensor(target_np, device="cuda")
        g_ref, _ = _grads(enc, feat, target, noalloc=False)
        g_na, out = _grads(enc, feat, target, noalloc=True)
        assert np.all(np.isfinite(g_na))
        np.testing.assert_array_equal(g_na, g_ref)
    # the second (smaller) call against the oracle's backprop as well
    f_o = E.features(ob.x, ob.cov)
    p = E.bf16_round(master)
    out_o, cache = E.forward(p, f_o)
    _, d_o = E.kl_loss(out_o, target_np)
    g_o = E.backward(p, cache, d_o)
    assert np.max(np.abs(g_na - g_o)) < 1e-3 * np.max(np.abs(g_o))


def test_noalloc_bwd_rejects_sizes_beyond_its_scratch():
    from paper_2503_08264_amd import _lib
    lib = _lib.load()
    dummy = ctypes.c_void_p(256)   # never dereferenced: the size check comes first
    assert lib.qem_enc_bwd_noalloc(dummy, dummy, dummy, dummy, 16385, dummy, None) == _lib.QEM_E_SHAPE
    assert lib.qem_enc_bwd_noalloc(dummy, dummy, dummy, dummy, 0, dummy, None) == _lib.QEM_E_SHAPE
    assert lib.qem_enc_bwd_noalloc(None, dummy, dummy, dummy, 10, dummy, None) == _lib.QEM_E_INVALID
