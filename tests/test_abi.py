"""Host-only checks of the C ABI (no GPU needed).

* Every function declared in include/qem.h is exported by libqem.so.
* The ctypes mirrors match the C struct layouts (a probe compiled with gcc
  against include/qem.h prints sizeof/offsetof).
* qem_create validates model descriptions on the host and reports errors.
"""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import qem_synth as S
from paper_2503_08264_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qem.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qem_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported():
    lib = _lib.load()
    names = _declared()
    assert "qem_create" in names and "qem_contract_fwd" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "qem.h"
#define P(T, F) printf("%s.%s %zu\n", #T, #F, offsetof(T, F));
int main(void) {
  printf("qem_node_desc %zu\nqem_obs_desc %zu\nqem_model_desc %zu\nqem_tensor_info %zu\n",
         sizeof(qem_node_desc), sizeof(qem_obs_desc), sizeof(qem_model_desc), sizeof(qem_tensor_info));
  P(qem_node_desc, parent_index) P(qem_node_desc, a) P(qem_node_desc, chain_len) P(qem_node_desc, init_b)
  P(qem_node_desc, q0a) P(qem_node_desc, q0b)
  P(qem_obs_desc, var) P(qem_obs_desc, x) P(qem_obs_desc, cov)
  P(qem_model_desc, nodes) P(qem_model_desc, obs)
  P(qem_tensor_info, dtype) P(qem_tensor_info, shape)
  return 0;
}
"""


def test_ctypes_layout_matches_header():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write(PROBE)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line.strip())
    mirror = {"qem_node_desc": _lib.NodeDesc, "qem_obs_desc": _lib.ObsDesc,
              "qem_model_desc": _lib.ModelDesc, "qem_tensor_info": _lib.TensorInfo}
    for name, cls in mirror.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
    for key, val in got.items():
        if "." in key:
            sname, field = key.split(".")
            assert getattr(mirror[sname], field).offset == int(val), key


def _desc(model):
    """Build C descriptors without touching the device (observation pointers are fake)."""
    N = len(model.nodes)
    nodes = (_lib.NodeDesc * N)()
    keep = []
    for v, nd in enumerate(model.nodes):
        d = nodes[v]
        d.n, d.dim = nd.n, nd.dim
        d.qfamily = _lib.QFAMILY[nd.qfamily]
        d.prior = _lib.PRIOR[nd.prior]
        ps = list(nd.parents) + [-1, -1]
        d.parent0, d.parent1 = ps[0], ps[1]
        if ps[0] >= 0 and model.nodes[ps[0]].n > 1:
            arr = np.ascontiguousarray(nd.parent_index, dtype=np.int32)
            keep.append(arr)
            d.parent_index = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.a, d.b, d.var, d.shape, d.rate = nd.a, nd.b, nd.var, nd.shape, nd.rate
        d.chain_len, d.init_b, d.init_var = nd.chain_len, nd.init_b, nd.init_var
        d.q0a, d.q0b = nd.q0
    obs = (_lib.ObsDesc * max(1, len(model.obs)))()
    for o, ob in enumerate(model.obs):
        od = obs[o]
        od.node, od.kind, od.n_per, od.coef, od.var = ob.node, _lib.OBS[ob.kind], ob.x.shape[1], ob.coef, ob.var
        od.x = 0x1000
        if ob.cov is not None:
            od.cov, od.n_cov = 0x2000, (ob.cov.shape[2] if ob.cov.ndim == 3 else 0)
    return nodes, obs, _lib.ModelDesc(N, len(model.obs), nodes, obs), keep


def _create(model, K, prec="fp32", flags=0):
    lib = _lib.load()
    nodes, obs, md, keep = _desc(model)
    ctx = ctypes.c_void_p()
    st = lib.qem_create_ex(ctypes.byref(ctx), ctypes.byref(md), K, _lib.PREC[prec], flags, None)
    err = lib.qem_last_error(None).decode()
    nbytes = lib.qem_workspace_bytes(ctx) if st == 0 else 0
    if st == 0:
        lib.qem_destroy(ctx)
    return st, err, nbytes


@pytest.mark.parametrize("name", ["normal_normal", "nested_gaussian", "chain", "gamma_poisson", "logistic",
                                  "ar_regions"])
def test_create_accepts_benchmark_models(name):
    small = {"normal_normal": {}, "nested_gaussian": dict(n_schools=4, n_classes=3, n_students=2),
             "chain": dict(n_series=3, T=5), "gamma_poisson": dict(n_groups=5), "logistic": dict(n_groups=5),
             "ar_regions": dict(n_regions=3, T=4)}
    m = S.make(name, 0, **small[name])
    st, err, nbytes = _create(m, 8)
    assert st == _lib.QEM_OK, err
    assert nbytes > 0 and nbytes % 256 == 0


def test_workspace_size_for_nested_gaussian():
    """The dominant buffer is the class-level factor tensor [8192, 64, 64] in FP32."""
    m = S.nested_gaussian(0)
    st, err, nbytes = _create(m, 64, "fp32")
    assert st == 0, err
    assert 8192 * 64 * 64 * 4 < nbytes < 2 * 8192 * 64 * 64 * 4


def test_no_tables_workspace():
    """Without the class-level table the workspace loses its [8192, 64, 64]
    FP32 part; chains lose theirs outside BF16-exp mode and keep it in it."""
    m = S.nested_gaussian(0)
    st, err, full = _create(m, 64, "fp32")
    st2, err2, lean = _create(m, 64, "fp32", _lib.CREATE_NO_TABLES)
    assert st == 0 and st2 == 0, (err, err2)
    assert full - lean >= 8192 * 64 * 64 * 4
    assert lean < 8192 * 64 * 64 * 4
    c = S.chain(0, n_series=8, T=16)
    for prec, drops in (("fp32", True), ("fp64", True), ("bf16exp", False)):
        # chains keep their table only when asked (and always in BF16-exp mode)
        a = _create(c, 64, prec, _lib.CREATE_CHAIN_TABLES)[2]
        b = _create(c, 64, prec, _lib.CREATE_NO_TABLES)[2]
        d = _create(c, 64, prec)[2]
        assert (a - b >= 8 * 15 * 64 * 64 * 4) if drops else a == b, prec
        assert d == b, prec
        assert _create(c, 64, prec, _lib.CREATE_CHAIN_TABLES | _lib.CREATE_NO_TABLES)[2] == b, prec


def test_create_rejects_unknown_flags():
    st, err, _ = _create(S.normal_normal(0), 8, "fp64", 0x4)
    assert st == _lib.QEM_E_INVALID and "flags" in err


def test_create_rejects_bad_descriptions():
    m = S.normal_normal(0)
    assert _create(m, 0)[0] == _lib.QEM_E_SHAPE
    assert _create(m, 513)[0] == _lib.QEM_E_SHAPE
    bad = S.normal_normal(0)
    bad.nodes[1].parents = (1,)              # a node cannot be its own parent
    st, err, _ = _create(bad, 8)
    assert st == _lib.QEM_E_INVALID and "precede" in err
    bad = S.nested_gaussian(0, n_schools=3, n_classes=2, n_students=2)
    bad.nodes[2].parent_index = np.array([0, 0, 1, 1, 2, 7], np.int32)   # out of range
    st, err, _ = _create(bad, 8)
    assert st == _lib.QEM_E_SHAPE and "parent_index" in err
    bad = S.chain(0, n_series=2, T=5)
    bad.nodes[0].n = 9                        # not a multiple of T
    assert _create(bad, 8)[0] == _lib.QEM_E_SHAPE
    bad = S.gamma_poisson(0, n_groups=3)
    bad.nodes[0].q0 = (0.0, 1.0)              # Gamma shape must be positive
    assert _create(bad, 8)[0] == _lib.QEM_E_INVALID
    assert _create(S.gamma_poisson(0, n_groups=3), 300)[0] == _lib.QEM_E_SHAPE   # two-parent K <= 256


def test_bernoulli_table_lds_limit_counts_the_staged_covariates():
    """The Bernoulli-logit table kernel keeps, per group, the n_per x K table
    (FP32), the outcomes and their sums, and stages the n_per x n_cov
    covariates and the K x (n_cov + 1) padded beta samples in FP64: the
    whole must fit 64 KiB of LDS.  150 observations of 8 covariates at
    K = 64 use 54 KiB; 200 use 52 KiB of table alone, 69 KiB with the staged
    values, and are refused."""
    assert _create(S.logistic(0, n_groups=3, n_obs=150, D=8), 64)[0] == _lib.QEM_OK
    st, err, _ = _create(S.logistic(0, n_groups=3, n_obs=200, D=8), 64)
    assert st == _lib.QEM_E_SHAPE and "covariates" in err


def test_create_rejects_unsupported_structure():
    m = S.gamma_poisson(0, n_groups=3)
    m.nodes[1] = S.Node("beta", 2, 1, "gamma", "gamma", q0=(2.0, 1.0))   # pair parent with 2 instances
    st, err, _ = _create(m, 8)
    assert st == _lib.QEM_E_UNSUPPORTED and "single-instance roots" in err


def test_chain_under_parent_plan():
    """A chain under a sampled parent keeps, per series and parent sample,
    u-tilde and messages (FP64) and weights; a series takes one parent
    instance; no BF16-exp mode; nothing hangs under a chain."""
    m = S.ar_regions(0, n_regions=3, T=4)
    st, err, nbytes = _create(m, 16, "fp32")
    assert st == _lib.QEM_OK, err
    assert nbytes >= 3 * 16 * 4 * 16 * (8 + 8 + 4)
    bad = S.ar_regions(0, n_regions=3, T=4)
    pidx = bad.nodes[2].parent_index.copy()
    pidx[5] = 2                                  # series 1 (instances 4..7) under two regions
    bad.nodes[2].parent_index = pidx
    st, err, _ = _create(bad, 16)
    assert st == _lib.QEM_E_INVALID and "one parent instance" in err
    st, err, _ = _create(m, 64, "bf16exp")
    assert st == _lib.QEM_E_UNSUPPORTED and "BF16-exp" in err
    under = S.ar_regions(0, n_regions=2, T=3)
    under.nodes.append(S.Node("c", 6, 1, "gauss", "normal", parents=(2,),
                              parent_index=np.arange(6, dtype=np.int32), a=1.0, b=0.0, var=1.0))
    st, err, _ = _create(under, 8)
    assert st == _lib.QEM_E_UNSUPPORTED and "children of chain" in err


def test_dirichlet_plan_and_rules():
    """Dirichlet latents: C >= 2 components, the Dirichlet prior and no
    parent, categorical counts only on them, nothing under them."""
    m = S.dirichlet_categorical(0, n_groups=4, C=3, n_obs=5)
    st, err, nbytes = _create(m, 16, "fp32")
    assert st == _lib.QEM_OK, err
    bad = S.dirichlet_categorical(0, n_groups=4, C=3, n_obs=5)
    bad.nodes[0].dim = 1
    assert _create(bad, 16)[0] == _lib.QEM_E_SHAPE
    bad = S.dirichlet_categorical(0, n_groups=4, C=3, n_obs=5)
    bad.nodes[0].prior = "normal"
    st, err, _ = _create(bad, 16)
    assert st == _lib.QEM_E_UNSUPPORTED and "Dirichlet" in err
    under = S.dirichlet_categorical(0, n_groups=4, C=3, n_obs=5)
    under.nodes.append(S.Node("c", 4, 3, "gauss", "normal", parents=(0,), parent_index=np.arange(4, dtype=np.int32)))
    st, err, _ = _create(under, 16)
    assert st == _lib.QEM_E_UNSUPPORTED and "under a Dirichlet" in err
    g = S.normal_normal(0)
    g.obs.append(S.Obs(1, "categorical", np.zeros((g.nodes[1].n, 2))))
    st, err, _ = _create(g, 8)
    assert st == _lib.QEM_E_UNSUPPORTED and "categorical" in err


def test_categorical_plan_and_rules():
    """Categorical latents: C >= 2, the categorical prior, a Dirichlet parent
    over the same categories (or none), mixture observations with means."""
    m = S.mixture(0, n_groups=5, C=3, n_obs=4)
    st, err, nbytes = _create(m, 16, "fp32")
    assert st == _lib.QEM_OK, err
    assert nbytes >= 5 * 16 * 16 * 4          # the membership pair table [n, K, K]
    bad = S.mixture(0, n_groups=5, C=3, n_obs=4)
    bad.nodes[0].dim = 4                      # weights over 4 components, memberships over 3
    st, err, _ = _create(bad, 16)
    assert st == _lib.QEM_E_UNSUPPORTED and "same categories" in err
    bad = S.mixture(0, n_groups=5, C=3, n_obs=4)
    bad.obs[0].cov = None
    st, err, _ = _create(bad, 16)
    assert st == _lib.QEM_E_INVALID and "means" in err


def test_iteration_numbers_are_checked_before_launch():
    """qem_step / qem_run / qem_sample reject iteration numbers the Philox
    counter word cannot hold, t = 0 under the Theorem 1 step t^-p (whose step
    would be infinite), and iterations whose second-sample stream (top bit
    flipped) would collide with a later first sample.  Valid numbers get as
    far as the unbound-workspace check."""
    lib = _lib.load()
    nodes, obs, md, keep = _desc(S.normal_normal(0))
    ctx = ctypes.c_void_p()
    assert lib.qem_create_ex(ctypes.byref(ctx), ctypes.byref(md), 8, _lib.PREC["fp64"], 0, None) == 0
    try:
        E_INV, E_STATE = _lib.QEM_E_INVALID, _lib.QEM_E_STATE
        assert lib.qem_step(ctx, 1, 0, 0.3) == E_STATE          # t = 0 is fine with the constant weight
        assert lib.qem_step(ctx, 1, 1 << 32, 0.3) == E_INV
        assert lib.qem_sample(ctx, 1, 1 << 32) == E_INV
        assert lib.qem_sample(ctx, 1, (1 << 32) - 1) == E_STATE
        assert lib.qem_run(ctx, 1, (1 << 32) - 4, 0.3, 4) == E_STATE
        assert lib.qem_run(ctx, 1, (1 << 32) - 4, 0.3, 5) == E_INV
        assert lib.qem_set_ema(ctx, 0.6, 0) == 0
        assert lib.qem_step(ctx, 1, 0, 0.3) == E_INV
        assert "t >= 1" in lib.qem_last_error(ctx).decode()
        assert lib.qem_run(ctx, 1, 0, 0.3, 3) == E_INV
        assert lib.qem_step(ctx, 1, 1, 0.3) == E_STATE
        assert lib.qem_run(ctx, 1, 1, 0.3, 3) == E_STATE
        assert lib.qem_set_ema(ctx, 0.0, 1) == 0
        assert lib.qem_step(ctx, 1, 1 << 31, 0.3) == E_INV
        assert lib.qem_step(ctx, 1, (1 << 31) - 1, 0.3) == E_STATE
        assert lib.qem_run(ctx, 1, (1 << 31) - 2, 0.3, 3) == E_INV
        assert lib.qem_run(ctx, 1, 5, 0.3, 0) == E_STATE         # nothing to run still needs a workspace
    finally:
        lib.qem_destroy(ctx)


def test_status_flags_match_header():
    """The binding's status-flag constants are the header's."""
    txt = open(HEADER).read()
    vals = dict(re.findall(r"#define (QEM_FLAG_[A-Z_]+)\s+(0x[0-9a-fA-F]+)u", txt))
    assert int(vals["QEM_FLAG_NONFINITE_LOGPHAT"], 16) == _lib.FLAG_NONFINITE
    assert int(vals["QEM_FLAG_VAR_FLOOR"], 16) == _lib.FLAG_VAR_FLOOR
    assert int(vals["QEM_FLAG_GAMMA_MEAN"], 16) == _lib.FLAG_GAMMA_MEAN
    assert int(vals["QEM_FLAG_NEG_INF_ROW"], 16) == _lib.FLAG_NEG_INF_ROW
    assert len({int(v, 16) for v in vals.values()}) == len(vals)   # distinct bits
