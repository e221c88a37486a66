"""Benchmark of the SK MCMCMC hot path on one MI355X.

A step is one pass of the whole hot path over every chain: propose (Philox, Floyd,
star-graph candidates), score (J.S on the matrix cores, fused energy epilogue) and
select (node rule, move).  The headline workload is SK N=1024 with 256 chains x 128
candidates per step, Gaussian J ~ N(0, 1/N), flip sets of 1..128 spins, beta = 2,
split-BF16 scoring; the FP64 scoring path is timed on the same instance.

Prints one JSON line (metric, value, roofline of the scoring kernel, CPU baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "candidate configs scored/s + steps-to-thermalize, SK N=1024, mixed vs FP64"
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 matrix peak
PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 matrix peak


def _time_path(w, precision, steps, warmup, J, scale):
    import torch
    from paper_2102_05613_amd import native
    cfg = native.make_config(w.N, w.M, w.chains, w.kmin, w.kmax, precision=precision, seed=w.seed)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    stream = torch.cuda.current_stream()
    t = 0
    for _ in range(warmup):
        ctx.propose(t)
        ctx.score_candidates()
        ctx.select(t, w.beta0)
        t += 1
    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for i in range(steps):
        ctx.propose(t)
        ev_s[i].record(stream)
        ctx.score_candidates()
        ev_e[i].record(stream)
        ctx.select(t, w.beta0)
        t += 1
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    score_ms = [a.elapsed_time(b) for a, b in zip(ev_s, ev_e)]
    _, _, summ = ctx.measure()
    ctx.close()
    return {"total_ms": total_ms, "wall_s": wall, "score_ms_avg": float(np.mean(score_ms)),
            "score_ms_min": float(np.min(score_ms)), "moves": summ["moves"], "near_ties": summ["near_ties"]}


def _cpu_baseline(w, J, scale, sample_chains):
    import oracle
    t0 = time.perf_counter()
    oracle.run(J, scale, w.N, w.M, sample_chains, w.kmin, w.kmax, w.seed, [w.beta0])
    dt = time.perf_counter() - t0
    return {"value": sample_chains * w.M / dt, "unit": "candidates/s", "cores": 1, "kind": "oracle",
            "sample": f"1 step of {sample_chains} chains (x{w.M} candidates, plain pair-sum energies of all "
                      f"{w.M + 1} nodes) of the same workload, {dt:.1f} s on 1 core"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sk_n1024_m128_split")
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--cpu-chains", type=int, default=160)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent chains would shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2102_05613_amd import inputs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    w = inputs.workload(args.workload)
    J, scale = w.couplings_matrix()
    split = _time_path(w, "split_bf16", args.steps, args.warmup, J, scale)
    fp64_steps = args.fp64_steps if args.fp64_steps is not None else max(3, args.steps // 5)
    fp64 = _time_path(w, "fp64", fp64_steps, min(args.warmup, 2), J, scale)

    cand = w.chains * w.M
    ms_step = split["total_ms"] / args.steps
    value = cand / (ms_step / 1e3)
    fp64_ms_step = fp64["total_ms"] / fp64_steps
    flops_split = 3.0 * w.N * (w.N - 1) * cand     # three BF16 terms, strict upper triangle
    flops_fp64 = 1.0 * w.N * (w.N - 1) * cand
    achieved = flops_split / (split["score_ms_avg"] / 1e3) / 1e12
    achieved64 = flops_fp64 / (fp64["score_ms_avg"] / 1e3) / 1e12
    out = {
        "metric": METRIC, "value": value, "unit": "candidates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic (seeded Gaussian SK couplings)",
        "config": {"workload": w.name, "N": w.N, "M": w.M, "chains": w.chains, "kmin": w.kmin, "kmax": w.kmax,
                   "beta": w.beta0, "precision": "split_bf16 (hi+mid+lo, fp32 accumulate, fp64 epilogue)",
                   "parallelism": "single GPU, chains x candidates as matrix columns"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None,
                     "kernel": "k_score_split", "kernel_ms": split["score_ms_avg"],
                     "flops_per_launch": flops_split},
        "fp64_path": {"value": cand / (fp64_ms_step / 1e3), "unit": "candidates/s", "ms_per_step": fp64_ms_step,
                      "steps": fp64_steps, "kernel": "k_score_f64", "kernel_ms": fp64["score_ms_avg"],
                      "achieved_tflops": achieved64, "peak_tflops": PEAK_FP64_TFLOPS,
                      "frac": achieved64 / PEAK_FP64_TFLOPS},
        "split_vs_fp64": (fp64_ms_step / ms_step),
        "selection": {"moves": split["moves"], "near_ties": split["near_ties"]},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = _cpu_baseline(w, J, scale, args.cpu_chains)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
