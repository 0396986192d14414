"""The contraction as a differentiable function of the unary log-factors.

``QEMContract`` wraps the forward contraction (qem_contract_fwd, log P_MP of
Eq. Prmp) and its hand-written adjoint (qem_contract_bwd).  The gradient of
log P_MP with respect to the unary factor u_v[i, k] is the marginal weight
w_v[i, k] of sample k of latent instance i: this is the source-term trick the
paper uses to obtain MPIW moments by reverse-mode differentiation (section
3.2).  The adjoint kernels recompute each level's exponentials from the
per-level partial log-sum-exps saved by the forward pass (the messages m_v),
not from a stored normalised [P, K, K] tensor.

Inputs are the unary tensors of every node (shape [n_v, K], the context's
precision); the forward copies them into the context's workspace, so the
pairwise factors of the last qem_logfactors call are reused.  The backward
reads the forward's factors and messages from the workspace, so it must run
before any later call that rewrites them (sampling, log-factors, another
forward, a step or run): the context counts such calls and the backward
raises if one came in between.
"""
from __future__ import annotations

import torch

from . import _lib


class QEMContract(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, *us):
        for v, u in enumerate(us):
            q.tensor(v, _lib.T_U).copy_(u.detach())
        q.contract_fwd()
        ctx.q = q
        ctx.gen = q.generation
        ctx.dtypes = [u.dtype for u in us]
        return q.tensor(-1, _lib.T_LOGPHAT).clone().reshape(())

    @staticmethod
    def backward(ctx, g):
        q = ctx.q
        if q.generation != ctx.gen:
            raise RuntimeError("QEMContract.backward: the context was used for another forward pass (or sample, "
                               "log-factors, step, run) after this graph's forward; its factors and messages are gone")
        g64 = g.detach().to(device=q.device, dtype=torch.float64).reshape(1).contiguous()
        q.contract_bwd(g64)
        grads = [q.tensor(v, _lib.T_W).to(dt).clone() for v, dt in enumerate(ctx.dtypes)]
        return (None, *grads)


def contract(q, us):
    """log P_MP as a differentiable function of the unary factors ``us``."""
    return QEMContract.apply(q, *us)
