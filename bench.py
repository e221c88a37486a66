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
PEAK_CLOCK_GHZ = 2.4        # engine clock the published peaks assume
TIMING_EVERY = 16           # the headline's scoring launches bracketed by events: every 16th
PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 matrix peak
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_score_split_sk_n1024_m128_traffic.md")


def kernel_source_hash() -> str:
    """sha256 over the sources the split scoring kernel is built from, to tie counter
    measurements to the kernel they were taken on: the code only (line comments and
    blank lines dropped, so that a comment edit does not retire a measurement)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("common.hpp", "device_rng.hpp", "score_split.hpp"):
        with open(os.path.join(ROOT, "paper_2102_05613_amd", "csrc", name), encoding="utf-8") as f:
            for code in code_lines(f.read()):
                h.update(code.encode("utf-8") + b"\n")
    return h.hexdigest()


def code_lines(text: str):
    """The lines of a C++ source with line comments and trailing blanks removed, empty
    lines dropped (the sources hashed here hold no '//' inside string literals)."""
    out = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].rstrip()
        if code:
            out.append(code)
    return out


def _traffic_from_profile():
    """HBM bytes per scoring launch from the committed FETCH_SIZE / WRITE_SIZE counter
    runs (each scaled by the plain-copy calibration), or None when the kernel sources
    have changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None, "no counter profile"
    rec = None
    for line in open(TRAFFIC_PROFILE):
        line = line.strip()
        if line.startswith("{") and '"source_sha256"' in line:
            rec = json.loads(line)
    if rec is None:
        return None, "counter profile has no record"
    if rec["source_sha256"] != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    return rec, "measured"


def _context(w, precision, rule, M, kmin, kmax, J, scale, mean_steps=0, scorer="gemm", arity=0, law="uniform",
             energy_update="exact", recompute_every=0):
    from paper_2102_05613_amd import native
    cfg = native.make_config(w.N, M, w.chains, kmin, kmax, precision=precision, rule=rule, seed=w.seed,
                             mean_steps=mean_steps, scorer=scorer, arity=arity, law=law,
                             energy_update=energy_update, recompute_every=recompute_every)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    return ctx


def _time_path(w, precision, steps, warmup, J, scale, every=1, energy_update="exact"):
    """Time `steps` pipelined steps after `warmup`; the scoring kernel is timed live by
    HIP events on its stream (mc3_timing_*) around every `every`-th launch of the timed
    steps, so that the events' own cost (a few microseconds a record) stays out of the
    throughput of a fast step."""
    import torch
    ctx = _context(w, precision, "mcmcmc", w.M, w.kmin, w.kmax, J, scale, energy_update=energy_update)
    stream = torch.cuda.current_stream()
    if warmup:
        ctx.step_n(0, warmup, w.beta0, w.beta0, 1)
    ctx.timing_enable(True, every=every)
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
    assert launches == (steps + every - 1) // every
    return {"total_ms": total_ms, "wall_s": wall, "score_ms_avg": score_ms / launches, "timed_launches": launches,
            "moves": summ["moves"], "near_ties": summ["near_ties"]}


def _steady_state(w, J, scale, after, steps):
    """Steps per second of the headline path once the chains have settled: `steps`
    steps timed after `after` untimed ones (no events inside the timed steps)."""
    import torch
    ctx = _context(w, "split_bf16", "mcmcmc", w.M, w.kmin, w.kmax, J, scale)
    ctx.step_n(0, after, w.beta0, w.beta0, 1)
    ms = _timed_steps(ctx, after, steps, w.beta0, w.beta0, 1)
    summ = ctx.measure()[2]
    ctx.close()
    torch.cuda.synchronize()
    return {"after_steps": after, "steps": steps, "ms_per_step": ms / steps,
            "candidates_per_s": w.chains * w.M * steps / (ms / 1e3),
            "moves_per_chain_step": summ["moves"] / (summ["steps_done"] * w.chains),
            "note": "the same path and workload as the headline, timed once the chains have settled (fewer "
                    "moves, so fewer coupling rows for the exact energy update); not the headline value"}


def _kernel_pass(w, precision, launches, J, scale, warmup=8):
    """The scoring kernel's average duration over `launches` consecutive steps of the
    same workload, every launch bracketed by HIP events on its stream (a pass of its
    own after the throughput timing, whose events would otherwise be in the timed
    steps)."""
    ctx = _context(w, precision, "mcmcmc", w.M, w.kmin, w.kmax, J, scale)
    ctx.step_n(0, warmup, w.beta0, w.beta0, 1)
    ctx.timing_enable(True, every=1)
    ctx.step_n(warmup, launches, w.beta0, w.beta0, 1)
    score_ms, n = ctx.timing_read()
    ctx.close()
    assert n == launches
    return {"score_ms_avg": score_ms / n, "launches": n, "first_step": warmup}


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


def _run_means(w, J, scale, prec, rule, M, kmin, kmax, scorer, arity, law, T, beta0, beta1, total,
               chunk=200000):
    """Chain-mean node-weighted energy per spin of every step of a T-step run from the
    init states, and its wall time (steps issued in chunks with a sync after each, so a
    long run reports progress)."""
    import torch
    ctx = _context(w, prec, rule, M, kmin, kmax, J, scale, mean_steps=T, scorer=scorer, arity=arity, law=law)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s0 in range(0, T, chunk):
        ctx.step_n(s0, min(chunk, T - s0), beta0, beta1, total)
        ctx.sync()
    wall = time.perf_counter() - t0
    means = ctx.read_means(0, T) / w.N
    ctx.close()
    return means[:, 1], wall


def _thermalize_study(w, J, scale, beta, label, specs, window):
    """Runs on the same instance, chains and initial states at a fixed beta.  specs:
    (name, precision, rule, M, kmin, kmax, scorer, arity, law, T).  The reference energy
    is the lowest tail mean (last 25% of a run) among the runs: every run starts from
    random states, far above the equilibrium energy, and approaches it from above, so
    the lowest tail is the best-converged estimate; the long runs in the specs exist to
    provide it.  t_1% uses one window for every run."""
    runs = {}
    for name, prec, rule, M, kmin, kmax, scorer, arity, law, T in specs:
        e, wall = _run_means(w, J, scale, prec, rule, M, kmin, kmax, scorer, arity, law, T, beta, beta, 1)
        runs[name] = {"wall_s": wall, "e_bar": e, "M": M, "T": T, "scorer": scorer, "precision": prec,
                      "graph": "star" if arity == 0 else (f"line, {M + 1} nodes" if law == "line"
                                                          else f"{arity}-ary tree, {M + 1} nodes")}
        _log(f"thermalize {label[:30]}.. {name}: {T} steps in {wall:.1f} s")
    tail = {name: float(np.mean(r["e_bar"][-r["T"] // 4:])) for name, r in runs.items()}
    ref_name = min(tail, key=tail.get)
    ref = tail[ref_name]
    out = {"setting": label, "beta": beta, "chains": w.chains, "window": window,
           "reference_energy_per_spin": ref, "reference_run": ref_name}
    for name, r in runs.items():
        t = _t_within(r["e_bar"], ref, window)
        per_step_s = r["wall_s"] / r["T"]
        out[name] = {"T": r["T"], "t_steps": t if t is not None else f"> {r['T']}",
                     "t_seconds": None if t is None else t * per_step_s,
                     "t_candidates": None if t is None else t * w.chains * r["M"],
                     "M": r["M"], "tail_energy_per_spin": tail[name], "ms_per_step": per_step_s * 1e3,
                     "scorer": r["scorer"], "precision": r["precision"], "graph": r["graph"]}
    return out


def _ratios_vs(study, base):
    """t_1% of `base` over each other run's, per step, per candidate and per second."""
    b = study[base]
    out = {}
    for name, r in study.items():
        if not isinstance(r, dict) or name == base or "t_steps" not in r:
            continue
        if isinstance(r["t_steps"], int) and isinstance(b["t_steps"], int) and r["t_steps"] > 0:
            out[name] = {"per_step": b["t_steps"] / r["t_steps"],
                         "per_candidate": b["t_candidates"] / r["t_candidates"],
                         "per_second": b["t_seconds"] / r["t_seconds"]}
        else:
            out[name] = None
    return out


def _thermalize(w, J, scale, T, T_long):
    """The paper's SK comparison (Fig. fig_sk) on this instance and the benchmark
    workload's own setting.  T: the window's scale (window = T / 100); the graph runs
    take 2 T steps (the line graph 3 T, the FP64 pair-sum star T, slower per step);
    T_long: steps of the single-update Metropolis runs (field-update scorer,
    microseconds a step), long enough for them to converge too."""
    window = max(10, T // 100)
    T2, T3 = 2 * T, 3 * T
    paper = _thermalize_study(
        w, J, scale, 1.0,
        "the paper's SK comparison (Fig. fig_sk) on this instance: L = 1024, T = 1, single-spin-flip edges; "
        "line-graph addition process of 2^7 nodes, binary tree of depth 7, ternary of depth 5, 16-ary of "
        "depth 3 (uniform root), the 129-node star, against single-update Metropolis",
        [("line_2e7", "split_bf16", "mcmcmc", 127, 1, 1, "gemm", 1, "line", T3),
         ("binary_depth7", "fp64", "mcmcmc", 126, 1, 1, "delta", 2, "uniform", T2),
         ("ternary_depth5", "fp64", "mcmcmc", 120, 1, 1, "delta", 3, "uniform", T2),
         ("16ary_depth3", "fp64", "mcmcmc", 272, 1, 1, "delta", 16, "uniform", T2),
         ("star_129_split_bf16", "split_bf16", "mcmcmc", 128, 1, 1, "gemm", 0, "uniform", T2),
         ("star_129_fp64", "fp64", "mcmcmc", 128, 1, 1, "gemm", 0, "uniform", T),
         ("star_129_field_update", "fp64", "mcmcmc", 128, 1, 1, "delta", 0, "uniform", T2),
         ("metropolis_m1_single_flip", "fp64", "metropolis", 1, 1, 1, "delta", 0, "uniform", T_long)],
        window)
    paper["t1pct_ratio_metropolis_over_graph"] = _ratios_vs(paper, "metropolis_m1_single_flip")
    paper["paper_claim"] = ("thermalization time decreased by two orders of magnitude against local single-update "
                            "Metropolis (Sec. 'Numerical results', Fig. fig_sk; hardware and precision not stated)")
    own = _thermalize_study(
        w, J, scale, w.beta0, "the benchmark workload's own flip sets (1..128 sites) and beta = 2",
        [("mcmcmc_split_bf16", "split_bf16", "mcmcmc", w.M, w.kmin, w.kmax, "gemm", 0, "uniform", T2),
         ("mcmcmc_fp64", "fp64", "mcmcmc", w.M, w.kmin, w.kmax, "gemm", 0, "uniform", max(10 * window, T // 5)),
         ("metropolis_m1_single_flip", "fp64", "metropolis", 1, 1, 1, "delta", 0, "uniform", T_long)],
        window)
    own["t1pct_ratio_metropolis_over_graph"] = _ratios_vs(own, "metropolis_m1_single_flip")
    return {
        "definition": "e(t) = chain mean of the node-weighted energy per spin; t_1% = first step after which "
                      "every window of max(10, T/100) steps (T of the graph runs; one window for every run) "
                      "has mean within 1% of the reference; reference = the lowest tail mean (last 25% of a "
                      "run) among the runs of the study, long runs included",
        "paper_graph_shapes": paper,
        "configured_workload": own,
    }


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed_steps(ctx, step0, n, beta0, beta1, total, graph=False):
    """Wall time (torch events on the context's stream) of n steps of mc3_step_n, or of
    mc3_step_n_graph (the same steps replayed from a captured HIP graph)."""
    import torch
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    (ctx.step_n_graph if graph else ctx.step_n)(step0, n, beta0, beta1, total)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end)


def _small_workload(w, steps):
    """Latency-bound shapes: microseconds per step of the whole path (propose, score,
    select) for the configured rule and, at N = 32, the two M = 1 rules as well."""
    J, scale = w.couplings_matrix()
    variants = [("mcmcmc_m%d" % w.M, "mcmcmc", w.M, w.kmin, w.kmax)]
    if w.N == 32:
        variants += [("mcmcmc_m1_heat_bath", "mcmcmc", 1, 1, 1), ("metropolis_m1", "metropolis", 1, 1, 1)]
    out = {"N": w.N, "chains": w.chains, "precision": w.precision, "steps": steps,
           "beta": [w.beta0, w.beta1], "bound": "launch latency (no roofline applies)",
           "scorers": {"gemm": "pair sums on the matrix cores, one scoring and one selection launch per step",
                       "gemm_graph": "the same launches replayed from a captured HIP graph (mc3_step_n_graph)",
                       "delta": "FP64 field update, every step of a chain in one persistent workgroup"}}
    for name, rule, M, kmin, kmax in variants:
        out[name] = {"M": M}
        for scorer, graph in (("gemm", False), ("gemm_graph", True), ("delta", False)):
            ctx = _context(w, w.precision, rule, M, kmin, kmax, J, scale, scorer=scorer.split("_")[0])
            ctx.step_n(0, 100, w.beta0, w.beta0, 1)
            if graph:   # capture outside the timed steps: same schedule, same first step
                ctx.step_n_graph(100, 300, w.beta0, w.beta1, w.steps)
            ms = _timed_steps(ctx, 100, steps, w.beta0, w.beta1, w.steps, graph=graph)
            ctx.close()
            out[name][scorer] = {"us_per_step": ms * 1e3 / steps,
                                 "candidates_per_s": w.chains * M * steps / (ms / 1e3)}
    return out


def _batched_workload(args):
    """2000 heterogeneous instances (N = 64..2048, M = 8..256, 4 chains each) stepped
    by one propose, one score and one select launch per step, against one launch of
    each per instance."""
    from paper_2102_05613_amd import inputs, native
    descs = inputs.batch_descs(args.batch_instances)
    w = inputs.workload("sk_batch_rep_n1024_m128")
    beta = inputs.BATCH_BETA
    cfg = native.make_batch_config(descs, precision="split_bf16", seed=w.seed)
    ctx = native.Context(cfg)
    t0 = time.perf_counter()
    for i, J, scale in inputs.iter_batch_couplings(descs):
        ctx.init_couplings(J, scale, instance=i)
    load_s = time.perf_counter() - t0
    ctx.init_chains()
    _log(f"batch: {len(descs)} instances loaded in {load_s:.1f} s")
    ctx.step_n(0, 3, beta, beta, 1)
    ms = _timed_steps(ctx, 3, args.batch_steps, beta, beta, 1)
    # the scoring launches timed one by one in a pass of their own
    t = 3 + args.batch_steps
    n_one = max(2, args.batch_steps // 2)
    ctx.timing_enable(True)
    _timed_steps(ctx, t, n_one, beta, beta, 1)
    score_ms, launches = ctx.timing_read()
    ctx.timing_enable(False)
    t += n_one
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_per = max(1, args.batch_steps // 4)
    ctx.step_n_per_instance(t, n_per, beta, beta, 1)
    torch.cuda.synchronize()
    per_ms = (time.perf_counter() - t0) * 1e3 / n_per
    # the same steps replayed from a captured HIP graph: one replay launches a 272-step
    # body; a run needs at least 288 steps to replay once.  The capture (outside the
    # timing) is reused by a run starting at the same step modulo 272.
    graph = None
    if args.batch_graph_steps >= 288:
        t1 = t + n_per
        ctx.step_n_graph(t1, 288, beta, beta, 1)
        gms = _timed_steps(ctx, t1 + 2 * 272, args.batch_graph_steps, beta, beta, 1, graph=True)
        graph = {"ms_per_step": gms / args.batch_graph_steps, "steps": args.batch_graph_steps}
    ctx.close()
    # the same batch on the field-update scorer: every chain of every instance in one
    # persistent launch that iterates the steps (score by differences, select, update
    # the field), FP64; Gaussian couplings drawn on the device (same law)
    pcfg = native.make_batch_config(descs, precision="fp64", seed=w.seed, scorer="delta")
    pctx = native.Context(pcfg)
    for i in range(len(descs)):
        pctx.generate_couplings(native.MC3_J_GAUSS, (inputs.BATCH_SEED << 20) + i, instance=i)
    pctx.init_chains()
    pctx.step_n(0, 3, beta, beta, 1)
    pms = _timed_steps(pctx, 3, args.batch_steps, beta, beta, 1)
    psum = pctx.measure()[2]
    pctx.close()
    persistent = {"ms_per_step": pms / args.batch_steps, "steps": args.batch_steps,
                  "moves_per_chain_step": psum["moves"] / (psum["steps_done"] * sum(d[2] for d in descs)),
                  "kernel": "k_step_delta_star: one workgroup per chain, all 8000 chains in one launch per call, "
                            "steps iterated inside the kernel",
                  "precision": "fp64 (energy differences from the maintained fields)"}
    Ns = np.array([d[0] for d in descs], dtype=np.float64)
    Ms = np.array([d[1] for d in descs], dtype=np.float64)
    Np = np.ceil(Ns / 128) * 128
    cand = float(np.sum(Ms * inputs.BATCH_CHAINS))
    flops = float(np.sum(3.0 * Ns * (Ns - 1) * Ms * inputs.BATCH_CHAINS))
    jbytes = float(np.sum(3.0 * Np * (Np + 128)))   # split triangle incl. diagonal blocks, read once
    score_s = score_ms / launches / 1e3
    ms_step = ms / args.batch_steps
    return {"instances": len(descs), "chains_per_instance": inputs.BATCH_CHAINS, "beta": beta,
            "N_range": [int(Ns.min()), int(Ns.max())], "M_range": [int(Ms.min()), int(Ms.max())],
            "candidates_per_step": cand, "steps": args.batch_steps,
            "batched": {"ms_per_step": ms_step, "candidates_per_s": cand / (ms_step / 1e3),
                        "score_kernel_ms": score_s * 1e3,
                        "launches_per_step": "one scoring launch per tile width present, one selection, one "
                                             "exact-update launch, one proposal per 16 steps",
                        "score_timing": f"HIP events around each scoring launch of {n_one} steps after the "
                                        f"timed ones"},
            "per_instance_launches": {"ms_per_step": per_ms, "candidates_per_s": cand / (per_ms / 1e3),
                                      "steps": n_per, "launches_per_step": 3 * len(descs)},
            "speedup_batched": per_ms / ms_step,
            "persistent_field_update": {**persistent,
                                        "candidates_per_s": cand / (persistent["ms_per_step"] / 1e3)},
            "batched_graph_replay": None if graph is None else {
                **graph, "candidates_per_s": cand / (graph["ms_per_step"] / 1e3)},
            "score_roofline": {"flops_per_launch": flops, "achieved_tflops": flops / score_s / 1e12,
                               "frac_mfma_bf16": flops / score_s / 1e12 / PEAK_BF16_TFLOPS,
                               "j_bytes_per_launch": jbytes, "achieved_gbs_j_once": jbytes / score_s / 1e9,
                               "frac_hbm_j_once": jbytes / score_s / 1e9 / PEAK_HBM_GBS},
            "couplings_load_s": load_s}


def _large_workload(args):
    """N = 8192, 32 chains x M = 1024, 256-spin flip sets: split path timed at the
    anneal's start, the FP64 path on a few steps."""
    from paper_2102_05613_amd import inputs
    w = inputs.workload("sk_n8192_m1024_split")
    J, scale = w.couplings_matrix()
    out = {"N": w.N, "M": w.M, "chains": w.chains, "k": [w.kmin, w.kmax], "beta": [w.beta0, w.beta1]}
    for prec, steps in (("split_bf16", args.large_steps), ("fp64", max(2, args.large_steps // 8))):
        ctx = _context(w, prec, "mcmcmc", w.M, w.kmin, w.kmax, J, scale)
        ctx.step_n(0, 2, w.beta0, w.beta1, w.steps)
        ctx.timing_enable(True)
        ms = _timed_steps(ctx, 2, steps, w.beta0, w.beta1, w.steps)
        score_ms, launches = ctx.timing_read()
        ctx.close()
        cand = w.chains * w.M
        flops = (3.0 if prec == "split_bf16" else 1.0) * w.N * (w.N - 1) * cand
        peak = PEAK_BF16_TFLOPS if prec == "split_bf16" else PEAK_FP64_TFLOPS
        ach = flops / (score_ms / launches / 1e3) / 1e12
        out[prec] = {"steps": steps, "ms_per_step": ms / steps, "candidates_per_s": cand * steps / (ms / 1e3),
                     "score_kernel_ms": score_ms / launches, "achieved_tflops": ach, "peak_tflops": peak,
                     "frac": ach / peak}
        _log(f"large N=8192 {prec}: {ms / steps:.2f} ms/step")
    return out


SPLIT_RTOL = 1e-4   # split-BF16 energies against FP64: relative, with the same absolute floor


def _large_cross_check(steps, every):
    """The split path of the large workload run over the first `steps` steps of its
    anneal; at every `every`-th step the candidates it scores are scored again by the
    FP64 path from the same states (an FP64 context given the split chains' spins;
    flip sets and roots are functions of seed, chain and step, so both score the same
    candidates)."""
    import torch
    from paper_2102_05613_amd import inputs, native
    w = inputs.workload("sk_n8192_m1024_split")
    J, scale = w.couplings_matrix()
    split = _context(w, "split_bf16", "mcmcmc", w.M, w.kmin, w.kmax, J, scale)
    cfg = native.make_config(w.N, w.M, w.chains, w.kmin, w.kmax, precision="fp64", seed=w.seed)
    f64 = native.Context(cfg)
    f64.init_couplings(J, scale)
    Es = torch.zeros(w.chains * w.M, dtype=torch.float64, device="cuda")
    Ed = torch.zeros_like(Es)
    checks = []
    t = 0
    while t < steps:
        f64.init_chains(native.bits_to_spins(split.measure()[1], w.N))
        split.propose(t)
        split.score_candidates(Es)
        f64.propose(t)
        f64.score_candidates(Ed)
        es, ed = Es.cpu().numpy(), Ed.cpu().numpy()
        d = np.abs(es - ed)
        checks.append({"step": t, "abs_max": float(d.max()), "abs_mean": float(d.mean()),
                       "max_err_over_tolerance": float((d / (SPLIT_RTOL * (np.abs(ed) + 1.0))).max()),
                       "energy_abs_min": float(np.abs(ed).min())})
        n = min(every, steps - t)
        split.step_n(t, n, w.beta0, w.beta1, w.steps)
        t += n
    split.close()
    f64.close()
    worst = max(c["max_err_over_tolerance"] for c in checks)
    eps = w.N * 2.0 ** -24
    return {"every": every, "steps": steps, "candidates_per_check": w.chains * w.M,
            "tolerance": "|E_split - E_fp64| <= 1e-4 (|E_fp64| + 1)", "checks": checks,
            "max_err_over_tolerance": worst, "within_tolerance": bool(worst <= 1.0),
            "eps_bound": eps, "within_eps_bound": bool(max(c["abs_max"] for c in checks) <= eps),
            "note": "eps_bound = N 2^-24, the split path's bound on one energy's error (FP32 accumulation of N "
                    "terms); the 1e-4 absolute floor is below it at N = 8192, so candidates with energies near "
                    "zero (the random initial states) can exceed the relative tolerance while within the bound",
            "reference": "FP64 matrix-core scoring of the same candidates from the split chains' states"}


def _precision_report(w, J, scale, step=3):
    """Relative error of the split-BF16 energies of every candidate of one step against
    the FP64 scorer's energies of the same candidates (same seed and step; the FP64
    path itself is pinned to the oracle by the parity tests)."""
    import torch
    from paper_2102_05613_amd import native
    E = {}
    for prec in ("split_bf16", "fp64"):
        cfg = native.make_config(w.N, w.M, w.chains, w.kmin, w.kmax, precision=prec, seed=w.seed)
        ctx = native.Context(cfg)
        ctx.init_couplings(J, scale)
        ctx.init_chains()
        ctx.propose(step)
        out = torch.zeros(w.chains * w.M, dtype=torch.float64, device="cuda")
        ctx.score_candidates(out)
        E[prec] = out.cpu().numpy()
        ctx.close()
    rel = np.abs(E["split_bf16"] - E["fp64"]) / np.maximum(np.abs(E["fp64"]), 1e-300)
    d = np.abs(E["split_bf16"] - E["fp64"])
    # differences between nodes of one chain (what the weights see): E_v - E of the chain's first column
    ds, d64 = (E[p].reshape(w.chains, w.M) for p in ("split_bf16", "fp64"))
    dd = np.abs((ds - ds[:, :1]) - (d64 - d64[:, :1]))[:, 1:]
    # the split path's tolerance, 1e-4 relative with an absolute floor of 1e-4 (the
    # parity tests' rtol and atol): |E_split - E_fp64| <= 1e-4 (|E_fp64| + 1)
    over_tol = d / (SPLIT_RTOL * (np.abs(E["fp64"]) + 1.0))
    return {"candidates": int(rel.size), "tolerance": "|E_split - E_fp64| <= 1e-4 (|E_fp64| + 1)",
            "max_err_over_tolerance": float(over_tol.max()), "within_tolerance": bool(over_tol.max() <= 1.0),
            "eps_bound": w.N * 2.0 ** -24, "within_eps_bound": bool(d.max() <= w.N * 2.0 ** -24),
            "rel_max": float(rel.max()), "rel_p9999": float(np.quantile(rel, 0.9999)),
            "rel_mean": float(rel.mean()), "abs_max": float(d.max()), "abs_p9999": float(np.quantile(d, 0.9999)),
            "abs_mean": float(d.mean()), "energy_abs_mean": float(np.abs(E["fp64"]).mean()),
            "node_difference_abs_max": float(dd.max()), "node_difference_abs_p9999": float(np.quantile(dd, 0.9999)),
            "node_difference_abs_mean": float(dd.mean()),
            "reference": "FP64 matrix-core scoring of the same candidates",
            "note": "relative errors peak at candidates with energies near zero; the absolute error is the "
                    "FP32 accumulation's; node differences are E_v - E_0 within each chain"}


def _anneal_thermalize(T):
    """Steps to thermalize under the anneal workload (N = 256, 64 chains, M = 16, flip
    sets 1..4, beta 0.1 -> 3 over T steps, FP64 field-update scorer) against
    single-flip Metropolis under the same schedule."""
    import torch
    from paper_2102_05613_amd import inputs
    w = inputs.workload("sk_n256_anneal_m16")
    J, scale = w.couplings_matrix()
    runs = {}
    for name, rule, M, kmin, kmax in (("mcmcmc_m16", "mcmcmc", w.M, w.kmin, w.kmax),
                                      ("metropolis_m1_single_flip", "metropolis", 1, 1, 1)):
        ctx = _context(w, "fp64", rule, M, kmin, kmax, J, scale, mean_steps=T, scorer="delta")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step_n(0, T, w.beta0, w.beta1, T)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        runs[name] = {"wall_s": wall, "e_bar": ctx.read_means(0, T)[:, 1] / w.N, "M": M}
        ctx.close()
    tail = {k: float(np.mean(r["e_bar"][-T // 100:])) for k, r in runs.items()}
    ref = min(tail.values())
    window = max(10, T // 100)
    out = {"workload": w.name, "beta": [w.beta0, w.beta1], "T": T, "window": window,
           "reference_energy_per_spin": ref,
           "note": "reference = lowest mean over the last 1% of steps (the coldest part of the anneal)"}
    for k, r in runs.items():
        t = _t_within(r["e_bar"], ref, window)
        out[k] = {"t_steps": t if t is not None else f"> {T}", "final_energy_per_spin": tail[k],
                  "t_seconds": None if t is None else t * r["wall_s"] / T, "ms_per_step": r["wall_s"] / T * 1e3}
    return out


def _large_thermalize(T):
    """Steps to thermalize under the large workload's anneal (N = 8192, 32 chains,
    M = 1024, 256-spin flip sets, beta 0.2 -> 2.5 over T steps, split BF16) against
    single-flip Metropolis under the same schedule (pair-sum FP64 scorer: the
    field-update scorer stops at N = 4096)."""
    import torch
    from paper_2102_05613_amd import inputs
    w = inputs.workload("sk_n8192_m1024_split")
    J, scale = w.couplings_matrix()
    runs = {}
    for name, prec, rule, M, kmin, kmax in (("mcmcmc_split_bf16", "split_bf16", "mcmcmc", w.M, w.kmin, w.kmax),
                                            ("metropolis_m1_single_flip", "fp64", "metropolis", 1, 1, 1)):
        ctx = _context(w, prec, rule, M, kmin, kmax, J, scale, mean_steps=T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s0 in range(0, T, 1000):
            ctx.step_n(s0, min(1000, T - s0), w.beta0, w.beta1, T)
            ctx.sync()
            _log(f"large thermalize {name}: {s0 + min(1000, T - s0)} / {T}")
        wall = time.perf_counter() - t0
        runs[name] = {"wall_s": wall, "e_bar": ctx.read_means(0, T)[:, 1] / w.N, "M": M}
        ctx.close()
    tail = {k: float(np.mean(r["e_bar"][-max(1, T // 100):])) for k, r in runs.items()}
    ref = min(tail.values())
    window = max(10, T // 100)
    out = {"workload": w.name, "beta": [w.beta0, w.beta1], "T": T, "window": window,
           "reference_energy_per_spin": ref,
           "note": "reference = lowest mean over the last 1% of steps (the coldest part of the anneal)"}
    for k, r in runs.items():
        t = _t_within(r["e_bar"], ref, window)
        out[k] = {"t_steps": t if t is not None else f"> {T}", "final_energy_per_spin": tail[k],
                  "t_seconds": None if t is None else t * r["wall_s"] / T, "ms_per_step": r["wall_s"] / T * 1e3}
    return out


def _table_law_workload(steps=200):
    """The line of 2^7 nodes grown with probability 0.3 of adding at node 0's end
    (root-law table C(M, v) 0.3^v 0.7^(M-v)) on the headline instance: N = 1024, 256
    chains, single-spin-flip edges, beta = 1, split BF16 and FP64 pair sums (the line's
    paths are too long for the field update)."""
    import math
    import torch
    from paper_2102_05613_amd import inputs, native
    w = inputs.workload("sk_n1024_m128_split")
    J, scale = w.couplings_matrix()
    M = 127
    table = [math.comb(M, v) * 0.3 ** v * 0.7 ** (M - v) for v in range(M + 1)]
    out = {"N": w.N, "M": M, "chains": w.chains, "beta": 1.0, "table": "C(M, v) 0.3^v 0.7^(M-v)"}
    for prec, scorer in (("split_bf16", "gemm"), ("fp64", "gemm")):
        cfg = native.make_config(w.N, M, w.chains, 1, 1, precision=prec, seed=w.seed, scorer=scorer, arity=1,
                                 law="table", law_table=table)
        ctx = native.Context(cfg)
        ctx.init_couplings(J, scale)
        ctx.init_chains()
        ctx.step_n(0, 20, 1.0, 1.0, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step_n(20, steps, 1.0, 1.0, 1)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        summ = ctx.measure()[2]
        ctx.close()
        out[f"{prec}_{scorer}"] = {"ms_per_step": ms, "candidates_per_s": w.chains * M / (ms / 1e3),
                                   "moves_per_chain_step": summ["moves"] / (summ["steps_done"] * w.chains)}
    return out


def _set_variant(reps=20):
    """mc3_set_generation timed on seeded synthetic two-body laws: one set of n = 20
    (2^20 subsets) and 4096 sets of n = 12.  Work per subset X of size k: (n-k) k
    multiply-adds of FP64, n(n-1) 2^(n-2) over all subsets of a set."""
    import torch
    from paper_2102_05613_amd import native
    out = {}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0x5EED0006)
    for n, n_sets in ((20, 1), (12, 4096)):
        G = torch.rand((n_sets, n, n), dtype=torch.float64, device="cuda", generator=gen)
        G.diagonal(dim1=1, dim2=2).zero_()
        G = G / G.sum(dim=1, keepdim=True)
        native.set_generation(G)
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            native.set_generation(G)
        end.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(end) / reps
        flops = 2.0 * n_sets * n * (n - 1) * 2.0 ** (n - 2)
        out[f"n{n}_sets{n_sets}"] = {"ms": ms, "subsets_per_s": n_sets * 2.0 ** n / (ms / 1e3),
                                     "launches": n + 1, "achieved_gflops_fp64": flops / (ms / 1e3) / 1e9,
                                     "frac_fp64_peak": flops / (ms / 1e3) / 1e12 / PEAK_FP64_TFLOPS}
    out["note"] = ("one launch per subset size (levels of decreasing popcount); small sets are bound by the "
                   "launches, the largest by the levels' passes over 2^n entries")
    return out


def _scorer_comparison(w, J, scale, steps=10):
    """The headline workload (N = 1024, 256 chains x M = 128, flip sets 1..128, beta = 2)
    stepped with each scorer: split-BF16 and FP64 pair sums on the matrix cores, and the
    FP64 field update (energies as differences: |F| field reads and |F|^2/2 coupling
    gathers per candidate, the algorithmic minimum); then the autotuner's timed choice."""
    import torch
    from paper_2102_05613_amd import autotune, native
    out = {"steps": steps}
    for name, prec, scorer in (("pair_sum_split_bf16", "split_bf16", "gemm"), ("pair_sum_fp64", "fp64", "gemm"),
                               ("field_update_fp64", "fp64", "delta")):
        ctx = _context(w, prec, "mcmcmc", w.M, w.kmin, w.kmax, J, scale, scorer=scorer)
        ctx.step_n(0, 3, w.beta0, w.beta0, 1)
        ms = _timed_steps(ctx, 3, steps, w.beta0, w.beta0, 1)
        ctx.close()
        out[name] = {"ms_per_step": ms / steps, "candidates_per_s": w.chains * w.M * steps / (ms / 1e3)}
    make = lambda scorer, width: native.make_config(w.N, w.M, w.chains, w.kmin, w.kmax, precision="split_bf16",
                                                    seed=w.seed, scorer=scorer, tile_cols=width)

    def init(ctx):
        ctx.init_couplings(J, scale)
        ctx.init_chains()

    r = autotune.tune_scorer(make, init, beta=w.beta0, steps=steps)
    out["autotuner"] = {"choice": f"{r['scorer']}:{r['tile_cols']}", "ms_per_step": r["ms"]}
    torch.cuda.synchronize()
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(w, J, scale, sample_chains, threads):
    """The oracle as it stands on the host's cores: one step of `sample_chains` chains
    of the workload, split over `threads` threads (each a disjoint chain range with its
    own chain_base, so the chains are the ones the GPU runs; the oracle's C code
    releases the interpreter lock while it runs)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    threads = max(1, min(threads, sample_chains))
    bounds = [(sample_chains * i) // threads for i in range(threads + 1)]

    def part(i):
        lo, hi = bounds[i], bounds[i + 1]
        oracle.run(J, scale, w.N, w.M, hi - lo, w.kmin, w.kmax, w.seed, [w.beta0], chain_base=lo)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        list(pool.map(part, range(threads)))
    dt = time.perf_counter() - t0
    return {"value": sample_chains * w.M / dt, "unit": "candidates/s", "cores": threads, "kind": "oracle",
            "sample": f"1 step of {sample_chains} chains (x{w.M} candidates; plain pair-sum energies of all "
                      f"{w.M + 1} nodes) of the same workload, {dt:.1f} s wall on {threads} threads "
                      f"(about {dt * threads:.0f} thread-seconds)",
            "cpu": _cpu_model(), "host_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="sk_n1024_m128_split")
    ap.add_argument("--fp64-steps", type=int, default=40)
    ap.add_argument("--steady-steps", type=int, default=200,
                    help="headline steps timed after 1500 untimed ones (0 skips it)")
    ap.add_argument("--kernel-launches", type=int, default=200,
                    help="scoring launches timed one by one for the roofline figure (a pass of their own)")
    ap.add_argument("--thermalize-steps", type=int, default=20000)
    ap.add_argument("--metropolis-steps", type=int, default=2000000,
                    help="steps of the single-update Metropolis runs of the thermalization study")
    ap.add_argument("--cpu-chains", type=int, default=640)
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="oracle threads for the CPU baseline (capped by the host's CPUs)")
    ap.add_argument("--anneal-steps", type=int, default=100000)
    ap.add_argument("--large-cross-check-steps", type=int, default=400,
                    help="split steps of the large workload with an FP64 scoring cross-check every 100th step")
    ap.add_argument("--large-thermalize-steps", type=int, default=20000,
                    help="steps of the N=8192 anneal study (0, or --large-steps 0, skips it; 20000 is the "
                         "workload's schedule)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--ceiling-iters", type=int, default=12500,
                    help="rounds of the matrix-core ceiling loop (0 skips it)")
    ap.add_argument("--set-variant", type=int, default=1, help="0 skips the set-variant timing")
    ap.add_argument("--scorers", type=int, default=1, help="0 skips the scorer comparison at the headline shape")
    ap.add_argument("--small-steps", type=int, default=10000,
                    help="steps timed on the latency-bound N=32 and N=256 workloads (0 skips them)")
    ap.add_argument("--batch-instances", type=int, default=2000, help="0 skips the batched workload")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-graph-steps", type=int, default=560,
                    help="steps of the batch replayed from a captured HIP graph (0 skips; at least 288 to replay)")
    ap.add_argument("--large-steps", type=int, default=16, help="0 skips the N=8192 workload")
    ap.add_argument("--profile", action="store_true",
                    help="counter-collection run: one plain 512 MiB device copy (calibrates FETCH_SIZE/WRITE_SIZE), "
                         "then --steps split steps; prints nothing else")
    ap.add_argument("--profile-batch", action="store_true",
                    help="counter-collection run of the batched workload: one plain 512 MiB device copy, "
                         "then its 2000 instances with Gaussian couplings generated on the device (same law as "
                         "the benchmark's host-loaded ones) and --steps steps; prints nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(independent chains would shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2102_05613_amd import inputs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.profile_batch:
        from paper_2102_05613_amd import native
        src = torch.ones(512 * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        descs = inputs.batch_descs(args.batch_instances)
        bw = inputs.workload("sk_batch_rep_n1024_m128")
        ctx = native.Context(native.make_batch_config(descs, precision="split_bf16", seed=bw.seed))
        for i in range(len(descs)):
            ctx.generate_couplings(native.MC3_J_GAUSS, (inputs.BATCH_SEED << 20) + i, instance=i)
        ctx.init_chains()
        ctx.step_n(0, args.steps, inputs.BATCH_BETA, inputs.BATCH_BETA, 1)
        ctx.sync()
        ctx.close()
        print(json.dumps({"profile_run": True, "workload": "sk_batch_2000_instances", "steps": args.steps}))
        return
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
    split = _time_path(w, "split_bf16", args.steps, args.warmup, J, scale, every=TIMING_EVERY)
    _log(f"headline split: {split['total_ms'] / args.steps:.4f} ms/step")
    scored = _time_path(w, "split_bf16", args.steps, args.warmup, J, scale, every=TIMING_EVERY,
                        energy_update="scored")
    kpass = _kernel_pass(w, "split_bf16", args.kernel_launches, J, scale)
    _log(f"headline scoring kernel: {kpass['score_ms_avg'] * 1e3:.2f} us over {kpass['launches']} launches")
    ceiling = None
    if args.ceiling_iters > 0:
        from paper_2102_05613_amd import native
        ceiling = native.mfma_ceiling(args.ceiling_iters)
        ceiling["mix_tflops"] = {name: native.mfma_mix(m, args.ceiling_iters) for m, name in native.MFMA_MIXES.items()}
        _log(f"matrix-core ceiling: {ceiling['tflops']:.0f} TFLOP/s at {ceiling['clock_ghz']:.2f} GHz; "
             f"with the split kernel's traffic mix {ceiling['mix_tflops']['split_kernel']:.0f}")
    fp64 = _time_path(w, "fp64", args.fp64_steps, min(args.warmup, 2), J, scale)
    _log(f"headline fp64: {fp64['total_ms'] / args.fp64_steps:.4f} ms/step")
    steady = None
    if args.steady_steps > 0:
        steady = _steady_state(w, J, scale, 1500, args.steady_steps)
        _log(f"headline at steady state: {steady['ms_per_step']:.4f} ms/step")

    cand = w.chains * w.M
    ms_step = split["total_ms"] / args.steps
    value = cand / (ms_step / 1e3)
    fp64_ms_step = fp64["total_ms"] / args.fp64_steps
    flops_split = 3.0 * w.N * (w.N - 1) * cand     # three BF16 terms, strict upper triangle
    flops_fp64 = 1.0 * w.N * (w.N - 1) * cand
    Np = -(-w.N // 128) * 128
    Bp = -(-cand // 512) * 512
    algo_bytes = (3.0 * Np * (Np + 128)          # split J triangle (3 BF16 terms), read once
                  + (Np // 32) * Bp * 4.0        # flip-set words of every column
                  + (w.chains + 1) * (Np // 32) * 4.0   # base words
                  + (Np // 256) * Bp * 8.0)      # FP64 partial energies written
    traffic, traffic_note = _traffic_from_profile()
    achieved = flops_split / (kpass["score_ms_avg"] / 1e3) / 1e12
    achieved64 = flops_fp64 / (fp64["score_ms_avg"] / 1e3) / 1e12
    out = {
        "metric": METRIC, "value": value, "unit": "candidates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic (seeded Gaussian SK couplings)",
        "config": {"workload": w.name, "N": w.N, "M": w.M, "chains": w.chains, "kmin": w.kmin, "kmax": w.kmax,
                   "beta": w.beta0, "precision": "split_bf16 (hi+mid+lo, fp32 accumulate, fp64 epilogue)"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS,
                     "traffic": None if traffic is None else traffic["fetch_bytes"] + traffic["write_bytes"],
                     "traffic_detail": {"status": traffic_note, "algorithmic_bytes": algo_bytes,
                                        **({} if traffic is None else traffic)},
                     "kernel": "k_score_split", "kernel_ms": kpass["score_ms_avg"],
                     "kernel_timing": f"HIP events on the scoring stream around each of {kpass['launches']} "
                                      f"consecutive scoring launches (steps {kpass['first_step']}.."
                                      f"{kpass['first_step'] + kpass['launches'] - 1} of a separate pass after the "
                                      f"timed steps); in the timed steps, every {TIMING_EVERY}th launch: "
                                      f"{split['score_ms_avg']:.5f} ms over {split['timed_launches']} launches",
                     "flops_per_launch": flops_split,
                     "ceiling": None if ceiling is None else {
                         "kind": "plain loop of independent 32x32x16 BF16 MFMAs at the scoring kernel's occupancy "
                                 "(libmc3ceil.so), run right after the timed steps",
                         "tflops": ceiling["tflops"], "clock_ghz": ceiling["clock_ghz"],
                         "peak_at_clock_tflops": PEAK_BF16_TFLOPS * ceiling["clock_ghz"] / PEAK_CLOCK_GHZ,
                         "frac_of_ceiling": achieved / ceiling["tflops"] if ceiling["tflops"] > 0 else None,
                         "mix_tflops": ceiling["mix_tflops"],
                         "mix_note": "the same loop with, per 64 MFMAs, the split kernel's other traffic (32 LDS "
                                     "128-bit reads, 72 VALU, 5 global loads, 1 barrier), a 64x128 wave tile's "
                                     "(16, 120, 11, 1), or LDS reads alone",
                         "frac_of_split_mix": (achieved / ceiling["mix_tflops"]["split_kernel"]
                                               if ceiling["mix_tflops"]["split_kernel"] > 0 else None)}},
        "fp64_path": {"value": cand / (fp64_ms_step / 1e3), "unit": "candidates/s", "ms_per_step": fp64_ms_step,
                      "steps": args.fp64_steps, "kernel": "k_score_f64", "kernel_ms": fp64["score_ms_avg"],
                      "achieved_tflops": achieved64, "peak_tflops": PEAK_FP64_TFLOPS,
                      "frac": achieved64 / PEAK_FP64_TFLOPS},
        "split_vs_fp64": fp64_ms_step / ms_step,
        "steady_state": steady,
        "energy_update": {
            "headline": "exact: the carried energy advances by the FP64 difference of each move, from the |D*| "
                        "coupling rows of the sites the move flips",
            "exact_ms_per_step": ms_step, "scored_ms_per_step": scored["total_ms"] / args.steps,
            "scored": "the chosen candidate's split-BF16 energy carried instead (no coupling rows read)",
            "moves_per_chain_step": split["moves"] / ((args.warmup + args.steps) * w.chains)},
        "selection": {"moves": split["moves"], "near_ties": split["near_ties"],
                      "near_ties_per_1e4_chain_steps": split["near_ties"] * 1e4 / ((args.warmup + args.steps) * w.chains)},
    }
    out["precision_split_vs_fp64"] = {"headline": _precision_report(w, J, scale)}
    if args.thermalize_steps > 0:
        out["steps_to_thermalize"] = _thermalize(w, J, scale, args.thermalize_steps, args.metropolis_steps)
        out["steps_to_thermalize"]["anneal_workload"] = _anneal_thermalize(args.anneal_steps)
        _log("thermalization study done")
    other = {}
    if args.small_steps > 0:
        for name in ("sk_n32_pm1_m4", "sk_n256_anneal_m16"):
            other[name] = _small_workload(inputs.workload(name), args.small_steps)
            _log(f"{name} done")
    if args.batch_instances > 0:
        other["sk_batch_2000_instances"] = _batched_workload(args)
        _log("batched workload done")
    if args.large_steps > 0:
        other["sk_n8192_m1024_split"] = _large_workload(args)
        wl = inputs.workload("sk_n8192_m1024_split")
        Jl, sl = wl.couplings_matrix()
        out["precision_split_vs_fp64"]["sk_n8192_m1024"] = _precision_report(wl, Jl, sl)
        _log("large workload precision done")
        if args.large_cross_check_steps > 0:
            other["sk_n8192_m1024_split"]["fp64_cross_check"] = _large_cross_check(args.large_cross_check_steps, 100)
            _log("large workload FP64 cross-check done")
    if args.scorers:
        other["scorers_at_headline_flip_sizes"] = _scorer_comparison(w, J, scale)
        _log("scorer comparison done")
    if args.set_variant:
        other["root_law_table_biased_line"] = _table_law_workload()
        _log("root-law table workload done")
        other["set_variant_generation"] = _set_variant()
        _log("set variant done")
    if args.large_steps > 0 and args.large_thermalize_steps > 0:
        out.setdefault("steps_to_thermalize", {})["large_workload"] = _large_thermalize(args.large_thermalize_steps)
    if other:
        out["other_workloads"] = other
    if not args.no_cpu:
        out["cpu_baseline"] = _cpu_baseline(w, J, scale, args.cpu_chains,
                                            min(args.cpu_threads, os.cpu_count() or 1))
        _log("cpu baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
