"""Tile-width autotuner for the split-BF16 scoring launch.

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
