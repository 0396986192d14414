#!/usr/bin/env python3
"""Benchmark: QEM E-step factor-evals/s on one MI355X.

Workload (the benchmark's headline configuration): the 3-level nested
Gaussian hierarchy, mu in R^4, 256 schools, 32 classes per school (8192 class
latents), 16 students per class, diagonal-Gaussian proposals, K = 64 samples
per latent, FP32 factor tensors ([8192, 64, 64] at the class level).

One step is one iteration of Algorithm 1 through the C ABI (qem_step):
sampling, log-factors, forward contraction (log P_MP), reverse pass
(marginal weights), moments, EMA and M-step.  Inputs are resident in HBM
before the timed region.  A factor-eval is one entry of one log-factor
tensor: 8192*64*64 + 256*64*64 pairwise entries plus 8449*64 unary entries
per step.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed (dual) FP32 instructions, which this build
# does not emit: 256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA x 2.4 GHz
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_nested_gaussian_k64_fp32.txt")
# the source files that define each reported kernel (and its launch shape)
KERNEL_SOURCES = {"plate_fwd": ["k_contract.hip", "dev_common.h", "dev_pair.h", "dev_sample.h", "dev_unary.h"],
                  "plate_bwd": ["k_contract.hip", "dev_common.h"],
                  "pairtable": ["k_factors.hip", "dev_common.h", "dev_pair.h"]}


def kernel_source_digest(kernel: str) -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2503_08264_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size),
    or None when absent or taken on different kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get(f"{kernel}_source_digest") != kernel_source_digest(kernel):
        return None
    v = vals.get(f"{kernel}_hbm_bytes_per_launch")
    return float(v) if v else None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(reps: int = 2):
    """The FP64 oracle on the host: `reps` full E-steps of the same workload,
    once on one thread and once on up to 16 threads (the oracle evaluates
    independent chunks of instances on its worker threads; sampling, the
    sums across instances and the moments stay serial)."""
    from threadpoolctl import threadpool_limits
    import qem_synth as S
    from oracle import mpiw as M
    model = S.nested_gaussian(0)
    K = 64
    evals = factor_evals(model, K) * reps
    threads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))
    rates = {}
    for nt in sorted({1, threads}):
        M.WORKERS = nt
        try:
            with threadpool_limits(limits=nt):
                t0 = time.perf_counter()
                for r in range(reps):
                    qs = M.q_init(model)
                    zs = M.sample(model, qs, K, r + 1, 1000)
                    M.estep(model, qs, zs, K)
                dt = time.perf_counter() - t0
        finally:
            M.WORKERS = 1
        rates[nt] = (evals / dt, dt)
    v, dt = rates[threads]
    return {"value": v, "unit": "factor-evals/s", "cores": threads, "kind": "oracle",
            "value_1_thread": rates[1][0], "cpu": cpu_model(),
            "sample": f"{reps} full E-steps (sample, log-factors, contraction, reverse pass, moments) "
                      f"of the same nested-Gaussian workload in FP64 numpy: {dt:.1f} s on {threads} threads, "
                      f"{rates[1][1]:.1f} s on 1"}


SCRUB_BYTES = 512 << 20       # twice the 256 MB Infinity Cache
PROBE_BYTES = 128 << 20       # about the class-level pair table (134 MB)


def kernel_times(q, model, cls, steps, seed, it, lam, scrub=None):
    """Per-launch durations of the class-level plate kernels over `steps`
    eager iterations, HIP events around every kernel on the context's
    stream; with `scrub`, a write over it (torch, same stream) before each
    iteration.  Returns ({name: {avg_us, launches}}, next iteration)."""
    import torch
    q.timing(True)
    for _ in range(steps):
        if scrub is not None:
            scrub.fill_(1.0)
        q.step(seed, it, lam)
        it += 1
    torch.cuda.synchronize()
    per = {}
    for name in ("plate_fwd", "plate_bwd", "pairtable", "sample"):
        tms, n = q.timing_read(cls, name)
        if n:   # the pair table (and the sampling) have no launch of their own when fused
            per[name] = {"avg_us": 1e3 * tms / n, "launches": n}
    q.timing(False)
    return per, it


def stream_ceilings(reps: int = 7):
    """Rates of the library's calibration streams (qem_stream_probe) over a
    128 MiB buffer, each pass behind a 512 MiB scrub: plain and nontemporal
    16-byte writes and reads in 16 KB chunks per workgroup, the median of
    `reps` passes (HIP events on torch's current stream).  write_gbs and
    read_gbs are the better of the plain and nontemporal streams."""
    import ctypes
    import torch
    from paper_2503_08264_amd import _lib
    lib = _lib.load()
    buf = torch.empty(PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
    scrub = torch.empty(SCRUB_BYTES // 4, dtype=torch.float32, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib, None, lib.qem_stream_probe(buf.data_ptr(), PROBE_BYTES, 0, sink.data_ptr(), stream),
               "qem_stream_probe")
    out = {"bytes": PROBE_BYTES, "scrub_bytes": SCRUB_BYTES}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for mode, name in enumerate(("write_plain", "write_nt", "read_plain", "read_nt")):
        ts = []
        for _ in range(reps):
            scrub.fill_(1.0)
            ev0.record()
            _lib.check(lib, None, lib.qem_stream_probe(buf.data_ptr(), PROBE_BYTES, mode, sink.data_ptr(), stream),
                       "qem_stream_probe")
            ev1.record()
            torch.cuda.synchronize()
            ts.append(ev0.elapsed_time(ev1))
        ms = sorted(ts)[len(ts) // 2]
        out[f"{name}_gbs"] = round(PROBE_BYTES / (ms * 1e-3) / 1e9, 1)
    out["write_gbs"] = max(out["write_plain_gbs"], out["write_nt_gbs"])
    out["read_gbs"] = max(out["read_plain_gbs"], out["read_nt_gbs"])
    del buf, scrub
    return out


def factor_evals(model, K: int) -> int:
    n = 0
    for nd in model.nodes:
        n += nd.n * K                      # unary entries
        if nd.parents:
            n += nd.n * K * K              # pairwise entries
    return n


WORKLOADS = {
    # name: (builder, K, precision, node whose pairwise kernels are reported)
    "nested_gaussian": (lambda S: S.nested_gaussian(0), 64, "fp32", 2),
    "normal_normal": (lambda S: S.normal_normal(0), 8, "fp64", 1),
    "chain_fp32": (lambda S: S.chain(0), 256, "fp32", 0),
    "chain_fp64": (lambda S: S.chain(0), 256, "fp64", 0),
    "chain_bf16exp": (lambda S: S.chain(0), 256, "bf16exp", 0),
    "gamma_poisson": (lambda S: S.gamma_poisson(0), 128, "fp32", 2),
    "gamma_poisson_ef": (lambda S: S.gamma_poisson(0, qfamily="gamma_ef"), 128, "fp32", 2),
    "logistic": (lambda S: S.logistic(0), 64, "fp32", 2),
    "occupancy": (lambda S: S.occupancy(0), 30, "fp32", 1),
    "ar_regions": (lambda S: S.ar_regions(0), 64, "fp32", 2),
    "dirichlet": (lambda S: S.dirichlet_categorical(0), 64, "fp32", 0),
    "mixture": (lambda S: S.mixture(0), 64, "fp32", 1),
}


# A bounded sample of each workload for the oracle's timing (its E-step on
# fewer independent groups where the full one takes minutes on the host; the
# rate is per factor-eval, so it carries over to the full size)
CPU_SAMPLES = {
    "nested_gaussian": (lambda S: S.nested_gaussian(0), "the full workload"),
    "normal_normal": (lambda S: S.normal_normal(0), "the full workload"),
    "chain_fp32": (lambda S: S.chain(0, n_series=16), "16 of the 1024 series"),
    "chain_fp64": (lambda S: S.chain(0, n_series=16), "16 of the 1024 series"),
    "chain_bf16exp": (lambda S: S.chain(0, n_series=16), "16 of the 1024 series"),
    "gamma_poisson": (lambda S: S.gamma_poisson(0, n_groups=128), "128 of the 2048 groups"),
    "gamma_poisson_ef": (lambda S: S.gamma_poisson(0, n_groups=128, qfamily="gamma_ef"), "128 of the 2048 groups"),
    "logistic": (lambda S: S.logistic(0, n_groups=512), "512 of the 8192 groups"),
    "occupancy": (lambda S: S.occupancy(0), "the full workload"),
    "ar_regions": (lambda S: S.ar_regions(0, n_regions=4), "4 of the 92 regions"),
    "dirichlet": (lambda S: S.dirichlet_categorical(0), "the full workload"),
    "mixture": (lambda S: S.mixture(0), "the full workload"),
}


def workload_evals(model, K: int) -> int:
    """Factor-evals of one E-step: every unary entry, every pair entry, K^3
    combinations per two-parent instance and per step of a chain under a
    sampled parent."""
    evals = sum(nd.n * K for nd in model.nodes)
    for nd in model.nodes:
        if nd.chain_len > 1:
            evals += (nd.n // nd.chain_len) * (nd.chain_len - 1) * K * K * (K if nd.parents else 1)
        elif len(nd.parents) == 2 or (nd.prior == "normal_logscale"):
            evals += nd.n * K * K * K
        elif nd.parents:
            evals += nd.n * K * K
    return evals


def cpu_only(workload: str, reps: int = 1):
    """The FP64 oracle's E-step on a bounded sample of `workload` (CPU_SAMPLES),
    on 1 thread and on up to 16, in factor-evals/s; one JSON line."""
    from threadpoolctl import threadpool_limits
    import qem_synth as S
    from oracle import mpiw as M
    build, what = CPU_SAMPLES[workload]
    K = WORKLOADS[workload][1]
    model = build(S)
    evals = workload_evals(model, K) * reps
    threads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))
    out = {"workload": workload, "sample": what, "K": K, "factor_evals_per_estep": evals // reps, "cpu": cpu_model()}
    for nt in sorted({1, threads}):
        M.WORKERS = nt
        try:
            with threadpool_limits(limits=nt):
                t0 = time.perf_counter()
                for r in range(reps):
                    qs = M.q_init(model)
                    zs = M.sample(model, qs, K, r + 1, 1000)
                    M.estep(model, qs, zs, K)
                dt = time.perf_counter() - t0
        finally:
            M.WORKERS = 1
        out[f"threads_{nt}"] = {"s_per_estep": dt / reps, "factor_evals_per_s": evals / dt}
    out["cores"] = threads
    print(json.dumps(out), flush=True)


def copy_calibration(nbytes: int = 1 << 30, reps: int = 3):
    """A plain device copy of known size, for scaling rocprofv3 byte counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stream-probe", action="store_true",
                    help="skip the calibration streams behind the roofline's stream ceiling")
    ap.add_argument("--workload", default="nested_gaussian", choices=sorted(WORKLOADS))
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--cpu-only", action="store_true",
                    help="time only the FP64 oracle's E-step on a bounded sample of --workload (host only)")
    ap.add_argument("--ema-p", type=float, default=0.0,
                    help="EMA step t^-p of Theorem 1 instead of the constant weight (0 keeps the constant)")
    ap.add_argument("--second-sample", action="store_true",
                    help="rescale the moments by P_MP(z) / P_MP(z_new) of a second sample")
    ap.add_argument("--no-tables", action="store_true",
                    help="recompute the linear-Gaussian pair factors instead of keeping their tables")
    ap.add_argument("--chain-tables", action="store_true",
                    help="keep the FP32/FP64 chain step-factor tables (recomputed by default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the E-step here runs on a single MI355X; "
              "a multi-GPU run would split the outermost plate across GPUs and all-reduce "
              "the partial root messages, which is not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.cpu_only:
        cpu_only(args.workload)
        return
    if args.workload != "nested_gaussian" or args.ema_p > 0.0 or args.second_sample:
        return other_workload(args)

    import torch
    import qem_synth as S
    from paper_2503_08264_amd.api import QEM

    model = S.nested_gaussian(0)
    K = 64
    q = QEM(model, K, "fp32", tables=not args.no_tables)
    lam, seed = 0.3, 1000
    it = 1
    for _ in range(args.warmup):
        q.step(seed, it, lam)
        it += 1
    torch.cuda.synchronize()

    # timed region: K iterations replayed from the captured HIP graph of one step
    s = q.stream
    q.run_graph(seed, it, lam, 1)          # capture outside the timed region
    it += 1
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(s)
    q.run_graph(seed, it, lam, args.steps)
    ev1.record(s)
    torch.cuda.synchronize()
    it += args.steps
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    flags, hits, logphat = q.read_status()

    # per-kernel durations: the same steps launched eagerly with HIP events
    # bracketing every kernel on the context's stream, first with the caches
    # as the previous step left them (warm), then with a 512 MiB scrub written
    # before every step so the Infinity Cache holds none of the step's data
    # when it starts (cold; the scrub is not inside any timed kernel)
    cls = 2
    warm, it = kernel_times(q, model, cls, args.steps, seed, it, lam, scrub=None)
    scrub = torch.empty(SCRUB_BYTES // 4, dtype=torch.float32, device="cuda")
    cold, it = kernel_times(q, model, cls, args.steps, seed, it, lam, scrub=scrub)
    del scrub
    per = cold
    R = model.nodes[cls].n
    tab = 0 if args.no_tables else R * K * K * 4   # the class-level table, when kept
    # without a sampling launch of the class node its plate forward draws the
    # class samples itself: it then also writes u (FP32) and reads the
    # proposal (mean, variance) and observation statistics (mean, sum of
    # squares) of each instance, 4 x dim doubles
    drawn = "sample" not in per
    algo = {
        # the step evaluates the class-level pair table inside the plate forward
        # kernel: F written + u-tilde (FP64) + messages written (FP64) + class
        # samples (dim 4) + school samples read once; u-tilde is read and the
        # class samples are read, or both are written when the kernel draws them
        "plate_fwd": tab + R * K * 8 + R * K * 8 + R * K * 4 * 4 + 256 * K * 4 * 4
                     + (R * K * 4 + R * 4 * 4 * 8 if drawn else 0),
        # F read + u-tilde + messages read + parent weights read + weights written,
        # and the fused moments: samples read (dim 4) + (m1, m2) written (FP64)
        "plate_bwd": tab + R * K * 8 + R * K * 8 + 256 * K * 4 + R * K * 4 + R * K * 4 * 4 + R * 4 * 2 * 8,
        # F written + class and school samples read (dim 4)
        "pairtable": R * K * K * 4 + R * K * 4 * 4 + 256 * K * 4 * 4,
    }
    per = {k: v for k, v in per.items() if k in algo}
    warm = {k: v for k, v in warm.items() if k in algo}
    dom = max(per, key=lambda k: per[k]["avg_us"])
    d = dict(per[dom], algo_bytes=algo[dom])
    if args.no_tables:
        # recomputed factors leave the pair kernels bound by FP32 arithmetic:
        # per pair, d subtractions and d multiply-adds for the distance, one
        # multiply-add for the factor, two adds, one exp and one multiply-add
        # (backward) or max + subtract + add (forward): 3d + 7 flops
        dim = model.nodes[cls].dim
        algo_flops = R * K * K * (3 * dim + 7)
        achieved = algo_flops / (d["avg_us"] * 1e-6) / 1e12
        roofline = {"kernel": f"class-level {dom}", "bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / ALU_PEAK_TFLOPS, "traffic": None,
                    "avg_us": d["avg_us"], "algo_flops_per_launch": algo_flops}
    else:
        achieved = d["algo_bytes"] / (d["avg_us"] * 1e-6) / 1e9
        roofline = {"kernel": f"class-level {dom}", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(dom),
                    "avg_us": d["avg_us"], "algo_bytes_per_launch": d["algo_bytes"], "cache": "cold",
                    "class_samples_drawn_in_plate_fwd": drawn,
                    "kernels": {k: {"avg_us": round(v["avg_us"], 2),
                                    "frac": round(algo[k] / (v["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
                                for k, v in per.items() if k in algo},
                    "warm": {k: {"avg_us": round(v["avg_us"], 2),
                                 "frac": round(algo[k] / (v["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
                             for k, v in warm.items() if k in algo}}
        if not args.no_stream_probe:
            ceil = stream_ceilings()
            roofline["stream_ceiling"] = ceil
            ref = ceil["write_gbs"] if dom in ("plate_fwd", "pairtable") else ceil["read_gbs"]
            roofline["frac_of_stream_ceiling"] = achieved / ref
    evals = factor_evals(model, K)
    out = {
        "metric": "QEM E-step factor-evals/s",
        "value": evals / (ms_per_step * 1e-3),
        "unit": "factor-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "nested_gaussian_3level_K64_fp32", "schools": 256, "classes_per_school": 32,
                   "students_per_class": 16, "dim": 4, "K": K, "factor_evals_per_step": evals,
                   "pair_tables": "recomputed" if args.no_tables else "kept",
                   "logphat_last": logphat, "status_flags": flags},
        "roofline": roofline,
        "kernels_us": {k: round(v["avg_us"], 2) for k, v in per.items()},
        "kernels_us_warm": {k: round(v["avg_us"], 2) for k, v in warm.items()},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def other_workload(args):
    """Step time and per-kernel durations of another benchmark hierarchy (the
    same JSON fields; not the headline line)."""
    import torch
    import qem_synth as S
    from paper_2503_08264_amd import _lib
    from paper_2503_08264_amd.api import QEM
    build, K, prec, node = WORKLOADS[args.workload]
    model = build(S)
    q = QEM(model, K, prec, tables=not args.no_tables, chain_tables=args.chain_tables)
    if args.ema_p > 0.0 or args.second_sample:
        q.set_ema(args.ema_p, args.second_sample)
    lam, seed, it = 0.3, 1000, 1
    for _ in range(args.warmup):
        q.step(seed, it, lam)
        it += 1
    q.run_graph(seed, it, lam, 1)
    it += 1
    s = q.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(s)
    q.run_graph(seed, it, lam, args.steps)
    ev1.record(s)
    torch.cuda.synchronize()
    it += args.steps
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    flags, hits, logphat = q.read_status()
    q.timing(True)
    for _ in range(args.steps):
        q.step(seed, it, lam)
        it += 1
    torch.cuda.synchronize()
    per = {}
    for v in range(len(model.nodes)):
        for ph in _lib.PHASES:
            tms, n = q.timing_read(v, ph)
            if n:
                per[f"{model.nodes[v].name}.{ph}"] = round(1e3 * tms / args.steps, 2)
    for ph in _lib.PHASES:
        tms, n = q.timing_read(-1, ph)
        if n:
            per[f"global.{ph}"] = round(1e3 * tms / args.steps, 2)
    q.timing(False)
    evals = workload_evals(model, K)
    print(json.dumps({"metric": "QEM E-step factor-evals/s", "value": evals / (ms_per_step * 1e-3),
                      "unit": "factor-evals/s", "ms_per_step": ms_per_step, "workload": args.workload,
                      "K": K, "dtype": prec, "factor_evals_per_step": evals,
                      "pair_tables": "recomputed" if args.no_tables else "kept",
                      "chain_tables": ("formed in the fold" if prec == "bf16exp" else
                                       "kept" if args.chain_tables else "recomputed"),
                      "ema": {"p": args.ema_p, "second_sample": args.second_sample}, "logphat_last": logphat,
                      "status_flags": flags, "phase_us_per_step": per}), flush=True)


if __name__ == "__main__":
    main()
