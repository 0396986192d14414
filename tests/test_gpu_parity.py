"""GPU parity of the E-step against the CPU oracle, through the C ABI.

Small cases compare every element (ragged K that is not a multiple of the
vector width, several tiles, several plate levels).  Full benchmark sizes
compare everything the oracle finishes in seconds, sampled instances where
it does not, and properties that hold at any size.
"""
import os

import numpy as np
import pytest

import qem_synth as S
from oracle import mpiw as M

from _parity import TOL, compare_estep, gpu_run, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

def _shuffled_classes(seed):
    """Classes assigned to schools in no particular order, so each school's
    children are not a contiguous run (the indexed child gather)."""
    m = S.nested_gaussian(seed, n_schools=7, n_classes=5, n_students=3, dim=3)
    rng = np.random.default_rng(seed)
    m.nodes[2].parent_index = rng.permutation(m.nodes[2].parent_index).astype(np.int32)
    return m


SMALL = {
    "normal_normal": lambda: S.normal_normal(3),
    "nested_ragged": lambda: S.nested_gaussian(1, n_schools=6, n_classes=5, n_students=3, dim=3),
    "chain_ragged": lambda: S.chain(2, n_series=5, T=9),
    # a step variance of 1e-3: most rows of a step lie far below the factor's
    # bound, so the forward's bounded log-sum-exps fall back to the row maximum
    "chain_tight": lambda: S.chain(6, n_series=4, T=8, var=1e-3),
    "gamma_poisson": lambda: S.gamma_poisson(4, n_groups=9, n_obs=7),
    "logistic": lambda: S.logistic(5, n_groups=6, n_obs=10, D=3),
    "nested_shuffled": lambda: _shuffled_classes(8),
}
SMALL_K = {"normal_normal": 8, "nested_ragged": 13, "chain_ragged": 20, "chain_tight": 64, "gamma_poisson": 12, "logistic": 11,
           "nested_shuffled": 16}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(SMALL))
def test_small_estep_parity(name, prec):
    model = SMALL[name]()
    K = SMALL_K[name]
    g = gpu_run(model, K, prec, seed=1234, it=3)
    o = oracle_run(model, K, seed=1234, it=3)
    compare_estep(g, o, prec)
    flags, hits, lp = g["status"]
    assert flags == 0


def test_normal_normal_qem_loop_fp64():
    """20 iterations of Algorithm 1 (K = 8, lam = 0.3), GPU vs oracle."""
    import torch
    from paper_2503_08264_amd.api import QEM
    from paper_2503_08264_amd import _lib
    model = S.normal_normal(0)
    say("[gpu] normal_normal QEM loop fp64")
    q = QEM(model, 8, "fp64")
    hist = q.run(20, 0.3, seed=77, record=True)
    m_ref, hist_ref = M.qem(model, 8, 20, 0.3, seed=77)
    assert rel_err(hist, hist_ref) < 1e-10
    for v in range(2):
        assert rel_err(q.tensor(v, _lib.T_MEMA).cpu().numpy(), m_ref[v]) < 1e-10


def test_nested_gaussian_full_size_fp32():
    """The 3-level Gaussian at full size (256 schools x 32 classes, K = 64), FP32,
    in the launch shapes the benchmark times."""
    model = S.nested_gaussian(0)
    g = gpu_run(model, 64, "fp32", seed=9, it=1)
    o = oracle_run(model, 64, seed=9, it=1)
    compare_estep(g, o, "fp32")


def test_nested_gaussian_full_size_fp64():
    model = S.nested_gaussian(0)
    g = gpu_run(model, 64, "fp64", seed=9, it=1)
    o = oracle_run(model, 64, seed=9, it=1)
    compare_estep(g, o, "fp64")


def _series_model(model, series):
    """The same chain restricted to a subset of its independent series."""
    T = model.nodes[0].chain_len
    sub = S.chain(0, n_series=len(series), T=T)
    x = model.obs[0].x.reshape(-1, T, 1, 1)[series].reshape(-1, 1, 1)
    sub.obs[0] = S.Obs(0, "gauss", x, var=model.obs[0].var)
    return sub


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_chain_full_size_sampled_series(prec):
    """1024 series x T = 64, K = 256: per-series log-sum-exp and weights of
    sampled series against the oracle (series are independent), and
    sum_k w = 1 for every step of every series."""
    import torch
    from paper_2503_08264_amd import _lib
    model = S.chain(0)
    K = 256
    g = gpu_run(model, K, prec, seed=5, it=2)
    q = g["ctx"]
    L = q.tensor(0, _lib.T_ROOTL).cpu().numpy()
    w = g["w"][0].reshape(1024, 64, K)
    np.testing.assert_allclose(w.sum(-1), 1.0, atol=1e-4 if prec == "fp32" else 1e-12)
    for gi in (0, 517, 1023):
        # the oracle draws the samples of series gi with the counters of the full model
        z = M.sample_instances(model, M.q_init(model), K, 2, 5, 0, np.arange(gi * 64, gi * 64 + 64))
        sub = _series_model(model, [gi])
        qs = M.q_init(sub)
        us = M.unary(sub, qs, [z.reshape(64, K, 1)], K)
        st = M.contract(sub, [z.reshape(64, K, 1)], us)
        ws = M.reverse(sub, [z.reshape(64, K, 1)], st)
        tol = TOL[prec]
        assert rel_err(L[gi], st.logphat) <= tol["logphat"]
        assert np.max(np.abs(w[gi] - ws[0])) <= tol["w"]
        assert rel_err(g["z"][0].reshape(1024, 64, K)[gi], z[..., 0]) <= tol["z"]


def test_gamma_poisson_parity_128():
    """K = 128 two-parent contraction on 48 groups, every element."""
    model = S.gamma_poisson(2, n_groups=48)
    g = gpu_run(model, 128, "fp32", seed=3, it=1)
    o = oracle_run(model, 128, seed=3, it=1)
    compare_estep(g, o, "fp32")


def _oracle_threads():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.mark.parametrize("it", [1, 3])
def test_gamma_poisson_full_size(it):
    """2048 groups x 64 counts, K = 128, FP32, in the launch shapes the
    benchmark times: samples, unary factors, log P_MP, every weight and every
    moment against the oracle (its chunks of groups evaluated on several host
    threads), the messages m_i[ka, kb] of sampled groups, and the joint root's
    weights normalised.  Iteration 3 of the bench's loop has the proposal of
    the M-step after two iterations (narrower, mostly in the FP32 GEMM tier),
    iteration 1 the broad initial one."""
    from paper_2503_08264_amd import _lib
    model = S.gamma_poisson(0)
    K, seed = 128, 8
    q = None
    if it == 1:
        g = gpu_run(model, K, "fp32", seed=seed, it=1)
        o = oracle_run(model, K, seed=seed, it=1, workers=_oracle_threads())
    else:
        # two QEM iterations on both sides (same draws), then the E-step of the third
        g, o = _after_iterations(model, K, seed, it, lam=0.3)
    compare_estep(g, o, "fp32", model=model)
    q = g["ctx"]
    m = q.tensor(2, _lib.T_MSG).double().cpu().numpy()
    for i in (0, 1000, 2047):
        assert rel_err(m[i], o["st"].msg[2][i]) < 1e-4
    for v in range(3):
        np.testing.assert_allclose(g["w"][v].sum(-1), 1.0, atol=1e-4)
    W = q.tensor(-1, _lib.T_PAIR_W).cpu().numpy()
    assert abs(W.sum() - 1.0) < 1e-10
    assert g["status"][0] == 0


def _qparam_array(nd, q):
    """The oracle's proposal of one node in the [n, dim, 2] layout of the
    proposal-parameter tensor (Gaussian (mean, var), Gamma (shape, rate))."""
    if nd.qfamily == "gauss":
        return np.stack([q["mean"], q["var"]], -1)
    return np.stack([q["shape"], q["rate"]], -1)


def _after_iterations(model, K, seed, it, lam):
    """The E-step of iteration `it` at the proposal the oracle's own loop
    (FP64, Algorithm 1) reaches after it - 1 iterations from Q_0: that
    proposal is written into the GPU's parameter tensor (oracle -> GPU only),
    then both sides draw iteration `it`'s samples from it."""
    import torch
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    say(f"[gpu] {model.name} K={K} fp32 seed={seed}: E-step of iteration {it} at the oracle's Q_{it - 1}")
    prev = M.WORKERS
    M.WORKERS = _oracle_threads()
    try:
        ms, _ = M.qem(model, K, it - 1, lam, seed)
        qs = M.set_params(model, ms)[0]
    finally:
        M.WORKERS = prev
    q = QEM(model, K, "fp32")
    for v, nd in enumerate(model.nodes):
        q.tensor(v, _lib.T_QPARAM).copy_(torch.as_tensor(_qparam_array(nd, qs[v]).reshape(nd.n, nd.dim, 2)))
    torch.cuda.synchronize()
    q.sample(seed, it)
    q.logfactors()
    q.contract_fwd()
    q.contract_bwd()
    q.moments()
    torch.cuda.synchronize()
    N = len(model.nodes)
    g = {
        "z": [q.tensor(v, _lib.T_Z).double().cpu().numpy() for v in range(N)],
        "u": [q.tensor(v, _lib.T_U).double().cpu().numpy() for v in range(N)],
        "w": [q.tensor(v, _lib.T_W).double().cpu().numpy() for v in range(N)],
        "mone": [q.tensor(v, _lib.T_MONE).cpu().numpy() for v in range(N)],
        "logphat": q.logphat(), "status": q.read_status(), "ctx": q,
    }
    o = oracle_run(model, K, seed=seed, it=it, qs=qs, workers=_oracle_threads())
    return g, o


def test_logistic_full_size():
    """The mixed-effects logistic model at full size (8192 groups x 50
    Bernoulli observations, 8 covariates, K = 64, FP32) in the launch shapes
    the benchmark times: samples, unary factors, log P_MP, every weight and
    every moment against the oracle, and sum_k w = 1 for every group."""
    model = S.logistic(0)
    K = 64
    g = gpu_run(model, K, "fp32", seed=21, it=1)
    o = oracle_run(model, K, seed=21, it=1, workers=_oracle_threads())
    compare_estep(g, o, "fp32", model=model)
    for v in range(3):
        np.testing.assert_allclose(g["w"][v].sum(-1), 1.0, atol=1e-4)
    assert g["status"][0] == 0


def test_logistic_parity_64():
    model = S.logistic(3, n_groups=40)
    g = gpu_run(model, 64, "fp32", seed=21, it=1)
    o = oracle_run(model, 64, seed=21, it=1)
    compare_estep(g, o, "fp32")


@pytest.mark.parametrize("prec,K", [("fp32", 64), ("fp64", 32)])
@pytest.mark.parametrize("n_obs", [70, 131])
def test_logistic_many_observations(n_obs, prec, K):
    """More than 64 observations per group: the FP32 Bernoulli-logit table
    folds its product of softplus factors into the log every 64 terms, and
    131 leaves a tail that is not a multiple of 4.  The table element by
    element against the oracle's, evaluated on the GPU's own samples, within
    the error bound of a J-term sum: 2 J eps sum_o |term_o| plus J times one
    term's function error (exp, log and product rounding); then the whole
    E-step against the oracle.  In FP32 the positive parts of the softplus
    terms are half of (eta + |eta|) with the eta summed apart, so sum_o
    |eta_o| joins the magnitudes that the sums round."""
    from paper_2503_08264_amd import _lib
    n = 5
    model = S.logistic(12, n_groups=n, n_obs=n_obs, D=3)
    g = gpu_run(model, K, prec, seed=6, it=1)
    F = g["ctx"].tensor(2, _lib.T_F).double().cpu().numpy().reshape(n, K, K)
    ob = model.obs[0]
    H = M._bern_table(ob, g["z"][0], g["z"][2], slice(0, n))
    s = np.einsum("njd,bd->nbj", ob.cov, g["z"][0][0])                    # [n, Kb, J]
    eta = s[:, :, None, :] + g["z"][2][:, None, :, 0, None]                # [n, Kb, K, J]
    y = ob.x[:, None, None, :]
    scale = (np.abs(y * eta) + np.logaddexp(0.0, eta) + (np.abs(eta) if prec == "fp32" else 0.0)).sum(-1)
    eps, fe = (2.0 ** -24, 2e-7) if prec == "fp32" else (2.0 ** -53, 1e-15)
    bound = 2 * n_obs * eps * scale + n_obs * (eps + fe)
    err = np.abs(F - H)
    say(f"[gpu] Bernoulli-logit table J={n_obs} {prec}: max err {err.max():.3e}, max err/bound {(err / bound).max():.3f}")
    assert np.all(err <= bound)
    o = oracle_run(model, K, seed=6, it=1)
    compare_estep(g, o, prec)


def test_status_flags_and_determinism_fp64():
    """FP64 results are bitwise identical run to run (fixed-order reductions)."""
    model = S.nested_gaussian(1, n_schools=16, n_classes=8, n_students=4)
    a = gpu_run(model, 32, "fp64", seed=4, it=1)
    b = gpu_run(model, 32, "fp64", seed=4, it=1)
    assert a["logphat"] == b["logphat"]
    for x, y in zip(a["w"], b["w"]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ess_matches_oracle(prec):
    """qem_ess: the marginal ESS 1 / sum_k w^2 of every instance and their
    mean, against the oracle's ESS of its own weights (3-level nested
    Gaussian, several nodes)."""
    from paper_2503_08264_amd import _lib
    model = S.nested_gaussian(2, n_schools=6, n_classes=9, n_students=4, dim=3)
    K = 37
    g = gpu_run(model, K, prec, seed=13, it=1)
    o = oracle_run(model, K, seed=13, it=1)
    ess_o = M.ess(o["w"])
    q = g["ctx"]
    for v in range(len(model.nodes)):
        e, mean = q.ess(v)
        e = e.cpu().numpy()
        tol = 1e-10 if prec == "fp64" else 2e-4
        assert rel_err(e, ess_o[v]) <= tol * K, (v, rel_err(e, ess_o[v]))
        assert abs(mean.item() - e.mean()) <= 1e-12 * K
        assert np.all((e >= 1.0 - 1e-6) & (e <= K + 1e-6))
