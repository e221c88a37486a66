"""Benchmark of the SK MCMCMC hot path on one MI355X.

A step is one pass of the whole hot path over every chain: propose (Philox, Floyd,
star-graph candidates), score (J.S on the matrix cores, fused energy epilogue) and
select (node rule, move), as run by mc3_step_n (the next step's proposal overlaps the
current scoring).  Headline workload: SK N=1024, 256 chains x 128 candidates per step,
Gaussian J ~ N(0, 1/N), flip sets of 1..128 spins, beta = 2, split-BF16 scoring.  The
FP64 scoring path is timed on the same instance.

Steps-to-thermalize: the same instance and chains run for T steps with split-BF16
MCMCMC, FP64 MCMCMC and single-flip Metropolis (M = 1), in two settings: the paper's
(single-spin-flip edges, T = Tc = 1) and the benchmark workload's own (flip sets of
1..128 spins, beta = 2).  e(t) is the chain mean of the node-weighted energy per spin;
the reference is the lowest tail mean (last 25%) among the runs; t_1% is the first
step after which every window of max(10, T/100) steps has mean within 1% of it.

Prints one JSON line.
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


def _context(w, precision, rule, M, kmin, kmax, J, scale, mean_steps=0):
    from paper_2102_05613_amd import native
    cfg = native.make_config(w.N, M, w.chains, kmin, kmax, precision=precision, rule=rule, seed=w.seed,
                             mean_steps=mean_steps)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    return ctx


def _time_path(w, precision, steps, warmup, J, scale):
    """Time `steps` pipelined steps after `warmup`; the scoring kernel is timed live by
    HIP events on its stream (mc3_timing_*)."""
    import torch
    ctx = _context(w, precision, "mcmcmc", w.M, w.kmin, w.kmax, J, scale)
    stream = torch.cuda.current_stream()
    if warmup:
        ctx.step_n(0, warmup, w.beta0, w.beta0, 1)
    ctx.timing_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    ctx.step_n(warmup, steps, w.beta0, w.beta0, 1)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    score_ms, launches = ctx.timing_read()
    _, _, summ = ctx.measure()
    ctx.close()
    assert launches == steps
    return {"total_ms": total_ms, "wall_s": wall, "score_ms_avg": score_ms / launches,
            "moves": summ["moves"], "near_ties": summ["near_ties"]}


def _t_within(e, ref, window, tol=0.01):
    """First t such that every window [t', t'+window) with t' >= t has mean within
    tol*|ref| of ref; None if there is none."""
    T = len(e)
    if T < window:
        return None
    c = np.concatenate([[0.0], np.cumsum(e)])
    wm = (c[window:] - c[:-window]) / window          # window means for t' = 0..T-window
    ok = np.abs(wm - ref) <= tol * abs(ref)
    bad = np.nonzero(~ok)[0]
    if len(bad) == 0:
        return 0
    t = int(bad[-1]) + 1
    return t if t <= T - window else None


def _thermalize_study(w, J, scale, T, beta, k_edge, label):
    """MCMCMC (split-BF16 and FP64, M = w.M, flip sets of k_edge = (kmin, kmax)) and
    single-flip Metropolis on the same instance, chains and initial states."""
    import torch
    runs = {}
    specs = [("mcmcmc_split_bf16", "split_bf16", "mcmcmc", w.M, k_edge[0], k_edge[1]),
             ("mcmcmc_fp64", "fp64", "mcmcmc", w.M, k_edge[0], k_edge[1]),
             ("metropolis_m1_single_flip", "fp64", "metropolis", 1, 1, 1)]
    for name, prec, rule, M, kmin, kmax in specs:
        ctx = _context(w, prec, rule, M, kmin, kmax, J, scale, mean_steps=T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step_n(0, T, beta, beta, 1)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        means = ctx.read_means(0, T) / w.N
        ctx.close()
        runs[name] = {"wall_s": wall, "e_bar": means[:, 1], "M": M}
    tail = {name: float(np.mean(r["e_bar"][-T // 4:])) for name, r in runs.items()}
    ref = min(tail.values())
    window = max(10, T // 100)
    out = {"setting": label, "beta": beta, "flip_set_sizes": list(k_edge), "M": w.M, "chains": w.chains,
           "T": T, "window": window, "reference_energy_per_spin": ref}
    for name, r in runs.items():
        t = _t_within(r["e_bar"], ref, window)
        per_step_s = r["wall_s"] / T
        out[name] = {"t_steps": t if t is not None else f"> {T}",
                     "t_seconds": None if t is None else t * per_step_s,
                     "t_candidates": None if t is None else t * w.chains * r["M"],
                     "tail_energy_per_spin": tail[name], "ms_per_step": per_step_s * 1e3}
    return out


def _thermalize(w, J, scale, T):
    return {
        "definition": "t_1%: first step after which every window of max(10, T/100) steps of the chain-mean "
                      "node-weighted energy per spin stays within 1% of the reference; reference = lowest tail "
                      "mean (last 25% of steps) among the runs of the study",
        "paper_setting": _thermalize_study(w, J, scale, T, 1.0, (1, 1),
                                           "single-spin-flip edges at T = Tc = 1 (the paper's SK experiment)"),
        "configured_workload": _thermalize_study(w, J, scale, T, w.beta0, (w.kmin, w.kmax),
                                                 "the benchmark workload's own flip sets and beta"),
    }


def _cpu_baseline(w, J, scale, sample_chains):
    import oracle
    t0 = time.perf_counter()
    oracle.run(J, scale, w.N, w.M, sample_chains, w.kmin, w.kmax, w.seed, [w.beta0])
    dt = time.perf_counter() - t0
    return {"value": sample_chains * w.M / dt, "unit": "candidates/s", "cores": 1, "kind": "oracle",
            "sample": f"1 step of {sample_chains} chains (x{w.M} candidates; plain pair-sum energies of all "
                      f"{w.M + 1} nodes) of the same workload, {dt:.1f} s on 1 core"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="sk_n1024_m128_split")
    ap.add_argument("--fp64-steps", type=int, default=40)
    ap.add_argument("--thermalize-steps", type=int, default=20000)
    ap.add_argument("--cpu-chains", type=int, default=160)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="counter-collection run: one plain 512 MiB device copy (calibrates FETCH_SIZE/WRITE_SIZE), "
                         "then --steps split steps; prints nothing else")
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
    if args.profile:
        src = torch.ones(512 * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        ctx = _context(w, "split_bf16", "mcmcmc", w.M, w.kmin, w.kmax, J, scale)
        ctx.step_n(0, args.steps, w.beta0, w.beta0, 1)
        ctx.sync()
        ctx.close()
        print(json.dumps({"profile_run": True, "copy_bytes": 512 * 2 ** 20, "steps": args.steps}))
        return
    split = _time_path(w, "split_bf16", args.steps, args.warmup, J, scale)
    fp64 = _time_path(w, "fp64", args.fp64_steps, min(args.warmup, 2), J, scale)

    cand = w.chains * w.M
    ms_step = split["total_ms"] / args.steps
    value = cand / (ms_step / 1e3)
    fp64_ms_step = fp64["total_ms"] / args.fp64_steps
    flops_split = 3.0 * w.N * (w.N - 1) * cand     # three BF16 terms, strict upper triangle
    flops_fp64 = 1.0 * w.N * (w.N - 1) * cand
    achieved = flops_split / (split["score_ms_avg"] / 1e3) / 1e12
    achieved64 = flops_fp64 / (fp64["score_ms_avg"] / 1e3) / 1e12
    out = {
        "metric": METRIC, "value": value, "unit": "candidates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic (seeded Gaussian SK couplings)",
        "config": {"workload": w.name, "N": w.N, "M": w.M, "chains": w.chains, "kmin": w.kmin, "kmax": w.kmax,
                   "beta": w.beta0, "precision": "split_bf16 (hi+mid+lo, fp32 accumulate, fp64 epilogue)"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None,
                     "kernel": "k_score_split", "kernel_ms": split["score_ms_avg"],
                     "flops_per_launch": flops_split},
        "fp64_path": {"value": cand / (fp64_ms_step / 1e3), "unit": "candidates/s", "ms_per_step": fp64_ms_step,
                      "steps": args.fp64_steps, "kernel": "k_score_f64", "kernel_ms": fp64["score_ms_avg"],
                      "achieved_tflops": achieved64, "peak_tflops": PEAK_FP64_TFLOPS,
                      "frac": achieved64 / PEAK_FP64_TFLOPS},
        "split_vs_fp64": fp64_ms_step / ms_step,
        "selection": {"moves": split["moves"], "near_ties": split["near_ties"]},
    }
    if args.thermalize_steps > 0:
        out["steps_to_thermalize"] = _thermalize(w, J, scale, args.thermalize_steps)
    if not args.no_cpu:
        out["cpu_baseline"] = _cpu_baseline(w, J, scale, args.cpu_chains)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
