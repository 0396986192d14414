"""Python binding of the QEM C ABI: argument marshalling only.

Every step of the E-step and M-step runs in the HIP kernels of libqem.so; this
module turns a model description into the C structs, allocates the workspace
as one torch device buffer, exposes workspace tensors as torch views, and
forwards calls with the names of the C ABI.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_double, c_int32, c_uint32, c_void_p
from typing import List, Optional

import numpy as np

from . import _lib
from ._lib import QEMError


def _torch():
    import torch
    return torch


_DT = {_lib.DT_F64: "float64", _lib.DT_F32: "float32", _lib.DT_U32: "int32", _lib.DT_BF16: "bfloat16"}


class QEM:
    """One QEM context: a model, K samples per latent instance, a precision.

    ``model`` has ``nodes`` and ``obs`` lists with the fields of
    ``qem_node_desc`` / ``qem_obs_desc`` (see include/qem.h); observation
    arrays are copied to the device once and kept alive here.
    """

    def __init__(self, model, K: int, prec: str = "fp32", device: str = "cuda", stream=None, tables: bool = True,
                 chain_tables: bool = False):
        torch = _torch()
        self.lib = _lib.load()
        self.model = model
        self.K = int(K)
        self.prec = prec
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise QEMError("the QEM library runs on a HIP device only")
        self._keep = []
        N = len(model.nodes)
        nodes = (_lib.NodeDesc * N)()
        for v, nd in enumerate(model.nodes):
            d = nodes[v]
            d.n, d.dim = nd.n, nd.dim
            d.qfamily = _lib.QFAMILY[nd.qfamily]
            d.prior = _lib.PRIOR[nd.prior]
            ps = list(nd.parents) + [-1, -1]
            d.parent0, d.parent1 = ps[0], ps[1]
            if ps[0] >= 0 and model.nodes[ps[0]].n > 1:
                arr = np.ascontiguousarray(nd.parent_index, dtype=np.int32)
                self._keep.append(arr)
                d.parent_index = arr.ctypes.data_as(POINTER(c_int32))
            d.a, d.b, d.var = nd.a, nd.b, nd.var
            d.shape, d.rate = nd.shape, nd.rate
            d.chain_len = nd.chain_len
            d.init_b, d.init_var = nd.init_b, nd.init_var
            d.q0a, d.q0b = nd.q0
        obs = (_lib.ObsDesc * max(1, len(model.obs)))()
        self.obs_dev = []   # device copies of each observation set: (x, cov or None)
        for o, ob in enumerate(model.obs):
            x = torch.as_tensor(np.ascontiguousarray(ob.x, dtype=np.float64), device=self.device)
            self._keep.append(x)
            self.obs_dev.append((x, None))
            od = obs[o]
            od.node, od.kind = ob.node, _lib.OBS[ob.kind]
            od.n_per = int(ob.x.shape[1])
            od.coef = ob.coef
            od.var = ob.var
            od.x = x.data_ptr()
            if ob.cov is not None:
                cv = torch.as_tensor(np.ascontiguousarray(ob.cov, dtype=np.float64), device=self.device)
                self._keep.append(cv)
                self.obs_dev[-1] = (x, cv)
                od.cov = cv.data_ptr()
                od.n_cov = int(ob.cov.shape[2]) if ob.cov.ndim == 3 else 0   # mixture means: [C]
        md = _lib.ModelDesc(N, len(model.obs), nodes, obs)
        self._desc = (nodes, obs, md)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        ctx = c_void_p()
        flags = (0 if tables else _lib.CREATE_NO_TABLES) | (_lib.CREATE_CHAIN_TABLES if chain_tables else 0)
        st = self.lib.qem_create_ex(byref(ctx), byref(md), self.K, _lib.PREC[prec], flags,
                                    c_void_p(stream.cuda_stream))
        _lib.check(self.lib, None, st, "qem_create_ex")
        self.ctx = ctx
        self.nbytes = int(self.lib.qem_workspace_bytes(ctx))
        # calls that rewrite the forward state (samples, factors, messages)
        self.generation = 0
        self.bind_workspace()

    def bind_workspace(self):
        """qem_bind_workspace on a fresh torch buffer (the context starts over
        from Q_0; views from ``tensor`` taken before refer to the old buffer)."""
        torch = _torch()
        ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        base = ws.data_ptr()
        pad = (-base) % 256
        self.generation += 1
        self._call("qem_bind_workspace", c_void_p(base + pad), self.nbytes)
        self.ws, self._pad = ws, pad

    # ------------------------------------------------------------ plumbing
    def _call(self, name, *args):
        st = getattr(self.lib, name)(self.ctx, *args)
        _lib.check(self.lib, self.ctx, st, name)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.qem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self, node: int, kind: int) -> _lib.TensorInfo:
        ti = _lib.TensorInfo()
        self._call("qem_tensor", node, kind, byref(ti))
        return ti

    def tensor(self, node: int, kind: int):
        """A torch view of a workspace tensor (no copy)."""
        torch = _torch()
        ti = self.info(node, kind)
        off = self._pad + ti.offset
        raw = self.ws[off: off + ti.bytes]
        dt = getattr(torch, _DT[ti.dtype])
        return raw.view(dt).view(tuple(ti.shape[: ti.ndim]))

    # ------------------------------------------------------------ the C ABI
    def init(self, node: int = -1):
        self._call("qem_init", node)

    def init_from_q(self, node: int = -1):
        self._call("qem_init_from_q", node)

    def sample(self, seed: int, it: int):
        self.generation += 1
        self._call("qem_sample", seed, it)

    def logfactors(self):
        self.generation += 1
        self._call("qem_logfactors")

    def contract_fwd(self):
        self.generation += 1
        self._call("qem_contract_fwd")

    def contract_bwd(self, dlogphat=None):
        self._call("qem_contract_bwd", c_void_p(0 if dlogphat is None else dlogphat.data_ptr()))

    def moments(self):
        self._call("qem_moments")

    def mstep(self, lam: float):
        self._call("qem_mstep", lam)

    def ess(self, node: int, mean_only: bool = False):
        """Marginal ESS of node's instances (device FP64 [n]) and their mean
        (device FP64 [1]), from this E-step's weights (qem_ess)."""
        torch = _torch()
        n = self.model.nodes[node].n
        e = torch.empty(n, dtype=torch.float64, device=self.device)
        m = torch.empty(1, dtype=torch.float64, device=self.device)
        self._call("qem_ess", node, c_void_p(e.data_ptr()), c_void_p(m.data_ptr()))
        return m if mean_only else (e, m)

    def step(self, seed: int, it: int, lam: float):
        self.generation += 1
        self._call("qem_step", seed, it, lam)

    def set_ema(self, p: float = 0.0, second_sample: bool = False):
        """EMA options of step / run_graph: the Theorem 1 step t^-p (p > 0) and
        the second-sample normaliser."""
        self._call("qem_set_ema", float(p), int(bool(second_sample)))

    def run_graph(self, seed: int, iter0: int, lam: float, n_iter: int):
        """qem_run: n_iter iterations replayed from one captured HIP graph."""
        self.generation += 1
        self._call("qem_run", seed, iter0, lam, n_iter)

    def read_status(self):
        flags, hits, lp = c_uint32(), c_uint32(), c_double()
        st = self.lib.qem_read_status(self.ctx, byref(flags), byref(hits), byref(lp))
        if st not in (_lib.QEM_OK, _lib.QEM_E_NONFINITE):
            _lib.check(self.lib, self.ctx, st, "qem_read_status")
        return int(flags.value), int(hits.value), float(lp.value)

    def timing(self, enable: bool):
        self._call("qem_timing", 1 if enable else 0)

    def timing_read(self, node: int, phase: str):
        """(total milliseconds, launches) of one phase of one node since tracing was enabled."""
        ms, n = c_double(), ctypes.c_int64()
        self._call("qem_timing_read", node, _lib.PHASES.index(phase), byref(ms), byref(n))
        return float(ms.value), int(n.value)

    # ------------------------------------------------------------ conveniences
    def estep(self, seed: int, it: int):
        self.sample(seed, it)
        self.logfactors()
        self.contract_fwd()
        self.contract_bwd()
        self.moments()

    def run(self, iters: int, lam: float, seed: int, start: int = 1, record: bool = False) -> List[float]:
        """Algorithm 1 for ``iters`` iterations from the current Q; returns the
        log P_MP of each iteration when ``record`` (one host read per iteration)."""
        hist = []
        for t in range(start, start + iters):
            self.step(seed, t, lam)
            if record:
                hist.append(self.read_status()[2])
        return hist

    def logphat(self) -> float:
        return float(self.tensor(-1, _lib.T_LOGPHAT).item())
