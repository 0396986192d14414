"""The two-parent contraction on MFMA (FP32 mode, K = 64 and 128): per
instance the log-sum-exp over k as the exponential GEMM A' B'^T and the
reverse pass as the transposed product, against the oracle.  An instance's
range bound picks the FP32 GEMM (<= 60), the FP64 GEMM (<= 600) or the exact
VALU kernels; one case mixes the two GEMM tiers and one mixes the FP64 GEMM
with the exact kernels, so every instance must be done exactly once."""
import numpy as np
import pytest

import qem_synth as S
from oracle import mpiw as M

from _parity import compare_estep, gpu_run, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu


def _wide_lambda(seed, n=24):
    """Gamma-Poisson with a wide initial proposal for the rates: log-rate
    ranges of several units, so some instances exceed the GEMM's bound."""
    m = S.gamma_poisson(seed, n_groups=n, n_obs=6)
    m.nodes[2].q0 = (0.8, 1.0)
    m.nodes[0].q0 = (3.0, 1.0)
    return m


def _bounds(model, K, seed, it):
    """The per-instance bound max_ka |ga1^ka| range_k gk_i^k: Gamma-Poisson
    ga1 = alpha - 1, gk = log lambda; logistic ga1 = -exp(-2 log sigma) / 2,
    gk = b^2."""
    qs = M.q_init(model)
    zs = M.sample(model, qs, K, it, seed)
    if model.name == "logistic":
        g1 = np.abs(np.exp(-2.0 * zs[1][0, :, 0]) / 2.0).max()
        gk = zs[2][..., 0] ** 2
    else:
        g1 = np.abs(zs[0][0, :, 0] - 1.0).max()
        gk = np.log(zs[2][..., 0])
    return g1 * (gk.max(1) - gk.min(1))


CASES = {
    "gamma_poisson_k64": (lambda: S.gamma_poisson(6, n_groups=20, n_obs=8), 64),
    "gamma_poisson_k128": (lambda: S.gamma_poisson(7, n_groups=12, n_obs=8), 128),
    "logistic_k64": (lambda: S.logistic(8, n_groups=16, n_obs=10, D=3), 64),
    "wide_k64": (lambda: _wide_lambda(9), 64),
}


@pytest.mark.parametrize("name", list(CASES))
def test_twoparent_mfma_parity(name):
    make, K = CASES[name]
    model = make()
    b = _bounds(model, K, 41, 2)
    if name == "wide_k64":     # FP32 and FP64 GEMMs in one launch
        assert (b > 60.0).any() and (b <= 60.0).any(), b
    if name == "logistic_k64":   # FP64 GEMM and the exact kernels in one launch
        assert (b > 600.0).any() and (b <= 600.0).any(), b
    g = gpu_run(model, K, "fp32", seed=41, it=2)
    o = oracle_run(model, K, seed=41, it=2)
    compare_estep(g, o, "fp32")
    assert g["status"][0] == 0


def test_twoparent_mfma_adjoint_scale():
    """The reverse pass scaled by g = 3: the weights of every node scale by 3."""
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    model, K = CASES["gamma_poisson_k64"][0](), 64
    say("[gpu] two-parent MFMA reverse pass scaled by 3")
    q = QEM(model, K, "fp32")
    q.sample(5, 1)
    q.logfactors()
    q.contract_fwd()
    q.contract_bwd()
    torch.cuda.synchronize()
    w1 = [q.tensor(v, _lib.T_W).cpu().numpy().astype(np.float64) for v in range(3)]
    q.contract_bwd(torch.tensor([3.0], dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    for v in range(3):
        assert rel_err(q.tensor(v, _lib.T_W).cpu().numpy(), 3.0 * w1[v]) < 1e-5, v
