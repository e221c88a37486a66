"""Autotuner: the split-BF16 scoring launch's tile width, and the scorer of a step.

A scoring work unit is a row-block pair of J times a tile of 128, 256 or 512
candidate columns, run by 2, 4 or 8 waves of 64 columns that share the pair's J
fragments through LDS.  By default the library picks the width from an instance's
column count (tile_cols = 0; a batch then mixes widths).  `tune_tile_cols` instead
times the scoring launch of the caller's own configuration at that default and at
every fixed width on the current device, and returns the fastest.  Timing
uses HIP events on the context's stream (`mc3_timing_enable`). The result is cached
in a JSON file keyed by the device and the configuration.

The choice changes time only, never a result: every column's partial sums run over
the same k order at every width.

`tune_scorer` times whole steps (mc3_step_n: proposal, scoring, selection, move) of
the caller's configuration with every scorer the library accepts for it -- the pair
sums on the matrix cores at each tile width, and the FP64 field update (energies as
differences, where its limits hold) -- and returns the fastest.  This is the measured
counterpart of the library's static MC3_SCORER_AUTO rule.  The scorers' results agree
within their precisions (bit for bit on +-1 couplings), not bit for bit in general.
"""
import hashlib
import json
import os
from typing import Callable, Dict, Optional, Sequence

from . import native

WIDTHS = (0, 128, 256, 512)   # 0: by each instance's column count


def config_key(cfg, device: str) -> str:
    """Cache key: the device name and every field of the configuration that shapes the
    scoring launch (not the tile width, the seed or the ring sizes)."""
    if isinstance(cfg, native.BatchConfig):
        inst = [(d.N, d.M, d.chains, d.kmin, d.kmax) for d in cfg.instances[:cfg.n_instances]]
    else:
        inst = [(cfg.N, cfg.M, cfg.chains, cfg.kmin, cfg.kmax)]
    shape = {"instances": inst, "precision": cfg.precision, "rule": cfg.rule, "scorer": cfg.scorer,
             "arity": cfg.arity, "law": cfg.law}
    digest = hashlib.sha256(json.dumps(shape, sort_keys=True).encode()).hexdigest()[:16]
    return f"{device}|{len(inst)} instance(s)|{digest}"


def time_scoring(make_cfg: Callable[[int], object], init: Callable[[object], None], width: int,
                 launches: int, warmup: int) -> float:
    """Mean duration (ms) of the scoring launch of make_cfg(width) on the current GPU:
    one proposal, `warmup` untimed launches, then `launches` launches bracketed by HIP
    events.  init(ctx) loads the couplings and the chains."""
    ctx = native.Context(make_cfg(width))
    try:
        init(ctx)
        ctx.propose(0)
        for _ in range(warmup):
            ctx.score_candidates()
        ctx.timing_enable(True, every=1)
        for _ in range(launches):
            ctx.score_candidates()
        ms, n = ctx.timing_read()
        ctx.timing_enable(False)
    finally:
        ctx.close()
    return ms / n


def _load(path: Optional[str]) -> Dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path, encoding="utf-8") as f:
        return json.load(f)


def _store(path: Optional[str], table: Dict) -> None:
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w", encoding="utf-8") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_tile_cols(make_cfg: Callable[[int], object], init: Callable[[object], None], launches: int = 20,
                   warmup: int = 3, widths: Sequence[int] = WIDTHS, cache_path: Optional[str] = None,
                   device: Optional[str] = None, timer=time_scoring, retune: bool = False) -> Dict:
    """The fastest split scoring tile width for make_cfg (a function of tile_cols
    returning a Config or BatchConfig).

    Returns {"tile_cols", "ms" (per width), "key", "cached"}.  With cache_path, an entry
    for the same key is returned without timing (unless retune), and a new result is
    written back."""
    if device is None:
        import torch
        device = torch.cuda.get_device_name(0)
    key = config_key(make_cfg(0), device)
    table = _load(cache_path)
    if not retune and key in table:
        hit = table[key]
        return {"tile_cols": int(hit["tile_cols"]), "ms": {int(w): v for w, v in hit["ms"].items()}, "key": key,
                "cached": True}
    ms = {int(w): float(timer(make_cfg, init, int(w), launches, warmup)) for w in widths}
    # ties: the widest fixed width, the default last
    best = min(ms, key=lambda w: (ms[w], -(w or -1)))
    table[key] = {"tile_cols": best, "ms": {str(w): v for w, v in ms.items()}}
    _store(cache_path, table)
    return {"tile_cols": best, "ms": ms, "key": key, "cached": False}


# (scorer, tile_cols) options of tune_scorer; tile widths apply to the split pair sums
SCORER_OPTIONS = tuple(("gemm", w) for w in WIDTHS) + (("delta", 0),)


def time_steps(make_cfg: Callable[[str, int], object], init: Callable[[object], None], scorer: str, width: int,
               steps: int, warmup: int, beta: float) -> float:
    """Mean wall time (ms) of one step of mc3_step_n for make_cfg(scorer, width) on the
    current GPU: `warmup` untimed steps, then `steps` steps between HIP events on the
    context's stream."""
    import torch
    ctx = native.Context(make_cfg(scorer, width))
    try:
        init(ctx)
        ctx.step_n(0, warmup, beta, beta, 1)
        stream = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        ctx.step_n(warmup, steps, beta, beta, 1)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps
    finally:
        ctx.close()


def tune_scorer(make_cfg: Callable[[str, int], object], init: Callable[[object], None], beta: float = 1.0,
                steps: int = 20, warmup: int = 3, options: Sequence = SCORER_OPTIONS,
                cache_path: Optional[str] = None, device: Optional[str] = None, timer=time_steps,
                retune: bool = False) -> Dict:
    """The fastest (scorer, tile width) for make_cfg (a function of (scorer, tile_cols)
    returning a Config or BatchConfig), over the options the library accepts for it
    (tile widths only for split-BF16 pair sums).

    Returns {"scorer", "tile_cols", "ms" (per "scorer:width"), "key", "cached"}."""
    if device is None:
        import torch
        device = torch.cuda.get_device_name(0)
    base = make_cfg("gemm", 0)
    key = "scorer|" + config_key(base, device) + f"|beta={beta!r}"
    table = _load(cache_path)
    if not retune and key in table:
        hit = table[key]
        return {"scorer": hit["scorer"], "tile_cols": int(hit["tile_cols"]), "ms": dict(hit["ms"]), "key": key,
                "cached": True}
    ms = {}
    for scorer, width in options:
        if width and base.precision != native.MC3_SPLIT_BF16:
            continue
        try:
            native.workspace_size(make_cfg(scorer, width))
        except native.MC3Error:
            continue   # outside this scorer's limits
        ms[f"{scorer}:{width}"] = float(timer(make_cfg, init, scorer, width, steps, warmup, beta))
    if not ms:
        raise ValueError("no scorer accepts this configuration")
    best = min(ms, key=lambda k: (ms[k], k))
    scorer, width = best.split(":")
    table[key] = {"scorer": scorer, "tile_cols": int(width), "ms": ms}
    _store(cache_path, table)
    return {"scorer": scorer, "tile_cols": int(width), "ms": ms, "key": key, "cached": False}
