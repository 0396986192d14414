"""Learned initialisation of QEM's proposal (the amortised encoder).

An MLP (18 -> 64 -> 64 -> 2, exact GELU, BF16 weights, FP32 accumulation)
maps a group's data summary to the mean and log variance of that group's
Gaussian proposal factor.  It is trained on the posterior moments that plain
QEM produces on training datasets (KL objective of appendix B: maximum
likelihood of the proposal under the estimated posterior), and used to set
Q_0 for new datasets.  Plain QEM is the fallback: at t = 0 the learned and
the prior initialisation are compared by log P_MP and effective sample size,
and the learned one is kept only if it is not worse.

Every arithmetic step runs in the qem_enc_* kernels of libqem.so; this module
orchestrates them (data movement, the training loop, the evaluation protocol).
"""
from __future__ import annotations

import argparse
import json
import time
from ctypes import c_void_p
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import _lib
from .api import QEM

NPARAM = 5506
N_GLOBAL_ROWS = 9   # beta (8 dimensions) and log sigma


def _torch():
    import torch
    return torch


def _ptr(t):
    return c_void_p(t.data_ptr())


def _check(st, what):
    if st != _lib.QEM_OK:
        lib = _lib.load()
        raise _lib.QEMError(f"{what}: {_lib.STATUS_NAMES.get(st, st)}: {lib.qem_last_error(None).decode()}")


class Encoder:
    """Device-resident encoder parameters (FP32 master, BF16 copy) and Adam state."""

    def __init__(self, device="cuda", seed: int = 0, stream=None):
        torch = _torch()
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        rng = np.random.default_rng(seed)
        parts = []
        for fan_in, fan_out in ((18, 64), (64, 64), (64, 2)):
            parts.append(rng.normal(0.0, np.sqrt(2.0 / (fan_in + fan_out)), size=fan_in * fan_out))
            parts.append(np.zeros(fan_out))
        self.master = torch.as_tensor(np.concatenate(parts).astype(np.float32), device=self.device)
        assert self.master.numel() == NPARAM
        self.w = torch.empty(NPARAM, dtype=torch.int16, device=self.device)
        self.m1 = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.m2 = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.step_count = 0
        _check(self.lib.qem_enc_to_bf16(_ptr(self.master), _ptr(self.w), self._s()), "qem_enc_to_bf16")

    def _s(self):
        return c_void_p(self.stream.cuda_stream)

    # ------------------------------------------------------------------ kernels
    def features(self, y, cov):
        """Raw group summaries [n, 18] from outcomes y [n, J] and covariates
        cov [n, J, 8] (host arrays or device tensors, FP64)."""
        torch = _torch()
        y = torch.as_tensor(np.ascontiguousarray(y, dtype=np.float64) if isinstance(y, np.ndarray) else y,
                            device=self.device)
        cov = torch.as_tensor(np.ascontiguousarray(cov, dtype=np.float64) if isinstance(cov, np.ndarray) else cov,
                              device=self.device)
        n, J = y.shape
        feat = torch.empty((n, 18), dtype=torch.float32, device=self.device)
        _check(self.lib.qem_enc_features(_ptr(y), _ptr(cov), n, J, cov.shape[2], _ptr(feat), self._s()),
               "qem_enc_features")
        return feat

    def forward(self, feat, keep_act: bool = False):
        torch = _torch()
        n = feat.shape[0]
        out = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        act = torch.empty((n, 128), dtype=torch.float32, device=self.device) if keep_act else None
        _check(self.lib.qem_enc_fwd(_ptr(self.w), _ptr(feat), n, _ptr(out), _ptr(act) if act is not None else None,
                                    self._s()), "qem_enc_fwd")
        return out, act

    def loss_grad(self, feat, target):
        """Mean KL loss (device scalar) and the parameter gradient."""
        torch = _torch()
        n = feat.shape[0]
        out, act = self.forward(feat, keep_act=True)
        dout = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        kl = torch.empty(n, dtype=torch.float64, device=self.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        _check(self.lib.qem_enc_loss(_ptr(out), _ptr(target), n, _ptr(dout), _ptr(kl), _ptr(loss), self._s()),
               "qem_enc_loss")
        grad = torch.empty(NPARAM, dtype=torch.float32, device=self.device)
        scratch = torch.empty(int(self.lib.qem_enc_scratch_bytes(n)) // 4 + 1, dtype=torch.float32,
                              device=self.device)
        _check(self.lib.qem_enc_bwd(_ptr(self.w), _ptr(feat), _ptr(act), _ptr(dout), n, _ptr(grad), _ptr(scratch),
                                    self._s()), "qem_enc_bwd")
        return loss, grad

    def adam(self, grad, lr=3e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        _check(self.lib.qem_enc_adam(_ptr(self.master), _ptr(self.w), _ptr(grad), _ptr(self.m1), _ptr(self.m2),
                                     self.step_count, lr, b1, b2, eps, self._s()), "qem_enc_adam")

    def train(self, feat, target, steps: int = 1500, lr: float = 3e-3, batch: int = 8192, seed: int = 0,
              log_every: int = 0):
        """Adam on minibatches of groups; returns the loss history (host reads every log_every)."""
        torch = _torch()
        n = feat.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        hist = []
        for it in range(steps):
            if batch < n:
                idx = torch.randint(0, n, (batch,), generator=g).to(self.device)
                f, t = feat[idx].contiguous(), target[idx].contiguous()
            else:
                f, t = feat, target
            cos = 0.5 * (1 + np.cos(np.pi * it / steps))
            loss, grad = self.loss_grad(f, t)
            self.adam(grad, lr=lr * (0.1 + 0.9 * cos))
            if log_every and (it % log_every == 0 or it == steps - 1):
                hist.append((it, float(loss.item())))
        return hist

    def pool(self, feat, J: int):
        """Input rows [9, 18] of the global head from one dataset's raw group
        summaries (groups of J observations)."""
        torch = _torch()
        rows = torch.empty((N_GLOBAL_ROWS, 18), dtype=torch.float32, device=self.device)
        _check(self.lib.qem_enc_pool(_ptr(feat), feat.shape[0], J, _ptr(rows), self._s()), "qem_enc_pool")
        return rows

    def features_ctx(self, feat, rows, J: int):
        """Group features with the dataset context of the pooled rows."""
        torch = _torch()
        out = torch.empty_like(feat)
        _check(self.lib.qem_enc_features_ctx(_ptr(feat), _ptr(rows), feat.shape[0], J, _ptr(out), self._s()),
               "qem_enc_features_ctx")
        return out

    def set_q(self, q: QEM, node: int, feat):
        """Write the encoder's proposal for every instance of a scalar Gaussian node and derive m_0."""
        out, _ = self.forward(feat)
        qp = q.tensor(node, _lib.T_QPARAM)
        _check(self.lib.qem_enc_apply(_ptr(out), feat.shape[0], _ptr(qp), self._s()), "qem_enc_apply")
        q.init_from_q(node)

    def set_globals(self, q: QEM, rows, beta_node: int = 0, sigma_node: int = 1):
        """As the global head: write the proposals of beta (8 dimensions) and
        log sigma from the pooled rows of this dataset (means predicted as
        residuals of the rows' plug-in estimates) and derive their m_0."""
        out, _ = self.forward(rows)
        qb = q.tensor(beta_node, _lib.T_QPARAM)
        qs = q.tensor(sigma_node, _lib.T_QPARAM)
        _check(self.lib.qem_enc_apply_residual(_ptr(out), _ptr(rows), 8, _ptr(qb), self._s()),
               "qem_enc_apply_residual")
        _check(self.lib.qem_enc_apply_residual(c_void_p(out.data_ptr() + 8 * 2 * 4),
                                               c_void_p(rows.data_ptr() + 8 * 18 * 4), 1, _ptr(qs), self._s()),
               "qem_enc_apply_residual")
        q.init_from_q(beta_node)
        q.init_from_q(sigma_node)


# ---------------------------------------------------------------------- data

def _targets(q: QEM, node: int, n: int, var_floor: float, rows=None, out=None):
    """qem_enc_targets on the EMA mean parameters of `node` ([n, 2] rows of
    (E z, E z^2)) into out [n, 2] (FP64, device)."""
    torch = _torch()
    m = q.tensor(node, _lib.T_MEMA)
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float64, device=q.device)
    _check(q.lib.qem_enc_targets(_ptr(m), n, var_floor, _ptr(rows) if rows is not None else None, _ptr(out),
                                 c_void_p(q.stream.cuda_stream)), "qem_enc_targets")
    return out


def posterior_targets(q: QEM, node: int):
    """(mean, var) of a scalar node's EMA moments, FP64 on the device
    (variance floored at 1e-8)."""
    return _targets(q, node, q.model.nodes[node].n, 1e-8)


def global_targets(q: QEM, beta_node: int = 0, sigma_node: int = 1, grows=None):
    """(mean, var) of the global latents' EMA moments: beta's 8 dimensions,
    then log sigma (variance floored at 1e-10).  With grows (the global
    head's pooled rows), the means are taken relative to each row's plug-in
    feature: the residuals the head is trained to predict."""
    torch = _torch()
    db = q.model.nodes[beta_node].dim
    out = torch.empty((db + 1, 2), dtype=torch.float64, device=q.device)
    _targets(q, beta_node, db, 1e-10, grows[:db] if grows is not None else None, out[:db])
    _targets(q, sigma_node, 1, 1e-10, grows[db:] if grows is not None else None, out[db:])
    return out


def plain_qem(model, K: int, iters: int, lam: float, seed: int, prec="fp32") -> QEM:
    q = QEM(model, K, prec)
    q.run_graph(seed, 1, lam, iters)
    return q


def dataset_inputs(enc: Encoder, y, cov):
    """Raw summaries, pooled rows of the global head, and the group encoder's
    context features of one dataset."""
    J = int(y.shape[1])
    raw = enc.features(y, cov)
    rows = enc.pool(raw, J)
    return raw, rows, enc.features_ctx(raw, rows, J)


def training_set(make_model, seeds, K: int, iters: int, lam: float, enc: Encoder, node: int = 2,
                 verbose: bool = False):
    """Training data from plain QEM on several datasets: the group encoder's
    context features and the posterior targets of group node `node`, and the
    global head's pooled rows with the posterior targets of beta and log sigma
    (9 rows per dataset; means relative to each row's plug-in feature, the
    residuals the head predicts)."""
    torch = _torch()
    feats, targets, grows, gtargets = [], [], [], []
    for s in seeds:
        model = make_model(s)
        q = plain_qem(model, K, iters, lam, seed=10_000 + s)
        targets.append(posterior_targets(q, node))
        x, cov = q.obs_dev[0]
        _, rows, ctx = dataset_inputs(enc, x, cov)
        feats.append(ctx)
        grows.append(rows)
        gtargets.append(global_targets(q, grows=rows))
        torch.cuda.synchronize()
        q.close()
        if verbose:
            print(f"[training set] dataset {s} done", flush=True)
    return torch.cat(feats), torch.cat(targets), torch.cat(grows), torch.cat(gtargets)


# ---------------------------------------------------------------------- evaluation

@dataclass
class Run:
    wall: List[float] = field(default_factory=list)          # seconds since start, per iteration
    snaps: List[list] = field(default_factory=list)          # m_ema per node after each iteration
    init_wall: float = 0.0
    choice: str = "prior"
    init_scores: dict = field(default_factory=dict)


def _snapshot(q: QEM):
    return [q.tensor(v, _lib.T_MEMA).clone() for v in range(len(q.model.nodes))]


def _restore(q: QEM, snap):
    for v, m in enumerate(snap):
        q.tensor(v, _lib.T_MEMA).copy_(m)
    q.mstep(0.0)


def score(q: QEM, snap, R: int, seed: int, se_target: float = 0.0, R_max: int = 0):
    """Mean log P_MP of R independent E-steps at the fixed Q of `snap`, its
    standard error and the mean marginal ESS of node 2.  With se_target > 0,
    draws are added 8 at a time (up to R_max) until the standard error of the
    mean is at most se_target."""
    torch = _torch()
    _restore(q, snap)
    lps, ess = [], []

    def draw(r):
        q.sample(seed, 1_000_000 + r)
        q.logfactors()
        q.contract_fwd()
        q.contract_bwd()
        ess.append(float(q.ess(2, mean_only=True).item()))
        lps.append(q.logphat())

    for r in range(R):
        draw(r)
    while se_target > 0.0 and len(lps) < R_max and np.std(lps, ddof=1) / np.sqrt(len(lps)) > se_target:
        for r in range(len(lps), min(R_max, len(lps) + 8)):
            draw(r)
    torch.cuda.synchronize()
    n = len(lps)
    return float(np.mean(lps)), float(np.std(lps, ddof=1) / np.sqrt(n)) if n > 1 else 0.0, float(np.mean(ess))


def _fwd_logphat(q: QEM, seed: int):
    """log P_MP of one forward E-step at the current Q, as a device scalar."""
    q.sample(seed, 1_000_000)
    q.logfactors()
    q.contract_fwd()
    return q.tensor(-1, _lib.T_LOGPHAT).clone()


def learned_init(q: QEM, enc: Encoder, head: Optional[Encoder], node: int):
    """Set Q_0 from the encoder (and the global head).  Returns the learned
    and the prior snapshots."""
    prior_snap = _snapshot(q)
    x, cov = q.obs_dev[0]
    _, rows, ctx = dataset_inputs(enc, x, cov)
    enc.set_q(q, node, ctx)
    if head is not None:
        head.set_globals(q, rows)
    return _snapshot(q), prior_snap


def run_qem(model, K, iters, lam, seed, enc: Optional[Encoder] = None, node: int = 2, fallback_R: int = 4,
            force_learned: bool = False, head: Optional[Encoder] = None, lam1: Optional[float] = None):
    """Algorithm 1 from the prior (enc None) or the learned initialisation (the
    group encoder, and the global head when given), timing every iteration.

    The learned run's clock includes encoder inference and the fallback check:
    one forward E-step gives log P_MP at the prior Q_0, the first QEM iteration
    gives it at the learned Q_0, and if the learned one is lower the run
    restarts from the prior (iteration 1 redone).  The kernels of both paths
    are warmed up before the clock starts; the initial scores (fallback_R
    draws, log P_MP and ESS) are taken after the run.  lam1, when given, is
    the EMA weight of iteration 1 only (1 starts the EMA from iteration 1's
    moments, so the initial proposal's mean parameters leave no memory)."""
    torch = _torch()
    run = Run()
    q = QEM(model, K, "fp32")
    q.run_graph(seed, 1, lam, 1)           # capture the step graph outside the timed region
    if lam1 is not None:
        q.step(seed, 1, lam1)               # warm-up of the eager first step
    if enc is not None:                     # warm-up of the timed path, discarded
        lp = _fwd_logphat(q, seed + 1)
        learned_init(q, enc, head, node)
        bool((q.tensor(-1, _lib.T_LOGPHAT) >= lp).item())
    q.init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lp_prior = None
    if enc is not None:
        lp_prior = _fwd_logphat(q, seed + 1)
        learned_snap, prior_snap = learned_init(q, enc, head, node)
        run.choice = "learned"
    torch.cuda.synchronize()
    run.init_wall = time.perf_counter() - t0
    def step(t):
        if t == 1 and lam1 is not None:
            q.step(seed, 1, lam1)
        else:
            q.run_graph(seed, t, lam, 1)

    for t in range(1, iters + 1):
        step(t)
        if t == 1 and lp_prior is not None and not force_learned:
            if not bool((q.tensor(-1, _lib.T_LOGPHAT) >= lp_prior).item()):
                run.choice = "prior"
                _restore(q, prior_snap)
                step(t)
        run.snaps.append(_snapshot(q))
        torch.cuda.synchronize()
        run.wall.append(time.perf_counter() - t0)
    if enc is not None:
        lp_l, _, ess_l = score(q, learned_snap, fallback_R, seed + 1)
        lp_p, _, ess_p = score(q, prior_snap, fallback_R, seed + 1)
        run.init_scores = dict(learned=(lp_l, ess_l), prior=(lp_p, ess_p))
    return q, run


def time_to_converge(scores, wall, target, hold: int = 5):
    """First iteration whose score is >= target and stays so for `hold` iterations."""
    for t in range(len(scores) - hold + 1):
        if all(s >= target for s in scores[t:t + hold]):
            return t, wall[t]
    return None, None


def _score_iters(iters: int, dense: int, every: int, tail: int):
    """Iterations whose snapshots are scored: every one up to `dense`, then
    every `every`-th, and every one of the last `tail` (where L* is taken)."""
    idx = set(range(0, min(dense, iters)))
    idx.update(range(dense, iters, every))
    idx.update(range(max(0, iters - tail), iters))
    return sorted(idx)


def evaluate(make_model, eval_seed: int, enc: Encoder, K: int, iters: int, lam: float, R: int,
             score_every: int = 1, head: Optional[Encoder] = None, dense: int = 0, se_target: float = 0.0,
             R_max: int = 0, lam1: Optional[float] = None):
    """The time-to-converge protocol on one held-out dataset: plain QEM from
    the prior and learned-init QEM, the same lambda, each iteration's Q_t
    scored by the mean log P_MP of R independent E-steps (adaptively more, to
    a standard error of se_target, when se_target > 0); L* = the mean score of
    plain QEM over its last 10% of iterations; t* = the first scored
    iteration whose score is >= L* - 0.1 (and, as a looser band, L* - 1)
    and stays so for 5 scored iterations.  plain_tail_drift = the mean
    score of the last 10% minus that of the 10% before it: how flat plain
    QEM's tail is, i.e. whether L* is a converged value."""
    plain_q, plain = run_qem(make_model(eval_seed), K, iters, lam, seed=eval_seed + 500)
    learned_q, learned = run_qem(make_model(eval_seed), K, iters, lam, seed=eval_seed + 500, enc=enc, head=head,
                                 lam1=lam1)
    tail = max(1, iters // 10)
    idx = (_score_iters(iters, dense, score_every, 2 * tail) if dense > 0 else list(range(0, iters, score_every)))
    psc = [score(plain_q, plain.snaps[t], R, 7, se_target, R_max) for t in idx]
    lsc = [score(learned_q, learned.snaps[t], R, 7, se_target, R_max) for t in idx]
    ps, ls = [x[0] for x in psc], [x[0] for x in lsc]
    last = [j for j, t in enumerate(idx) if t >= iters - tail]
    prev = [j for j, t in enumerate(idx) if iters - 2 * tail <= t < iters - tail]
    L_star = float(np.mean([ps[j] for j in last]))
    drift = L_star - float(np.mean([ps[j] for j in prev])) if prev else None
    tp, wp = time_to_converge(ps, [plain.wall[t] for t in idx], L_star - 0.1)
    tl, wl = time_to_converge(ls, [learned.wall[t] for t in idx], L_star - 0.1)
    tp1, wp1 = time_to_converge(ps, [plain.wall[t] for t in idx], L_star - 1.0)
    tl1, wl1 = time_to_converge(ls, [learned.wall[t] for t in idx], L_star - 1.0)
    res = dict(eval_seed=eval_seed, L_star=L_star, L_star_se=float(np.sqrt(np.sum([psc[j][1] ** 2 for j in last]))
                                                                   / len(last)),
               plain_tail_drift=drift, score_se_max=float(max(x[1] for x in psc + lsc)),
               draws_max=None if not se_target else R_max,
               plain_iter=None if tp is None else idx[tp], plain_wall_s=wp,
               learned_iter=None if tl is None else idx[tl], learned_wall_s=wl,
               speedup=(wp / wl) if (wp and wl) else None,
               plain_iter_1nat=None if tp1 is None else idx[tp1], learned_iter_1nat=None if tl1 is None else idx[tl1],
               speedup_1nat=(wp1 / wl1) if (wp1 and wl1) else None, learned_choice=learned.choice,
               init_scores=learned.init_scores, plain_scores=ps, learned_scores=ls, score_iters=idx,
               plain_s_per_iter=plain.wall[-1] / iters, learned_init_s=learned.init_wall)
    plain_q.close()
    learned_q.close()
    return res


def main():
    ap = argparse.ArgumentParser(description="train the encoder and compare learned vs plain initialisation")
    ap.add_argument("--groups", type=int, default=8192)
    ap.add_argument("--train-sets", type=int, default=32)
    ap.add_argument("--train-iters", type=int, default=250)
    ap.add_argument("--iters", type=int, default=250)
    ap.add_argument("--K", type=int, default=64)
    ap.add_argument("--lam", type=float, default=0.3)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--head-steps", type=int, default=6000)
    ap.add_argument("--R", type=int, default=16)
    ap.add_argument("--score-every", type=int, default=1)
    ap.add_argument("--eval-seed", type=int, default=0)
    ap.add_argument("--eval-seeds", default="",
                    help="comma-separated held-out dataset seeds (overrides --eval-seed)")
    ap.add_argument("--dense", type=int, default=0,
                    help="score every iteration up to this one, then every --score-every-th and the tail")
    ap.add_argument("--se", type=float, default=0.0, help="standard error target of each score (nats)")
    ap.add_argument("--R-max", type=int, default=64)
    args = ap.parse_args()
    import qem_synth as S
    torch = _torch()

    def make(s):
        return S.logistic(s, n_groups=args.groups)

    enc = Encoder(seed=1)
    head = Encoder(seed=3)
    t0 = time.perf_counter()
    feat, target, grows, gtargets = training_set(make, range(100, 100 + args.train_sets), args.K,
                                                 args.train_iters, args.lam, enc, verbose=True)
    t1 = time.perf_counter()
    hist = enc.train(feat, target, steps=args.steps, log_every=max(1, args.steps // 10))
    ghist = head.train(grows, gtargets, steps=args.head_steps,
                       log_every=max(1, args.head_steps // 10))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    seeds = [int(x) for x in args.eval_seeds.split(",")] if args.eval_seeds else [args.eval_seed]
    runs = []
    for es in seeds:
        r = evaluate(make, es, enc, args.K, args.iters, args.lam, args.R, args.score_every, head=head,
                     dense=args.dense, se_target=args.se, R_max=args.R_max)
        runs.append(r)
        print(json.dumps({k: r[k] for k in ("eval_seed", "L_star", "L_star_se", "plain_tail_drift", "score_se_max",
                                            "plain_iter", "learned_iter", "speedup", "plain_iter_1nat",
                                            "learned_iter_1nat", "speedup_1nat", "learned_choice")}), flush=True)
    out = dict(train_data_s=t1 - t0, train_s=t2 - t1, loss_hist=hist, head_loss_hist=ghist, groups=args.groups,
               train_sets=args.train_sets, K=args.K, lam=args.lam, R=args.R, se_target=args.se, runs=runs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
