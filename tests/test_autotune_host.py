"""The tile-width autotuner's host logic (choice, cache) with a stand-in timer, and
the library's validation of the tile width: no GPU needed."""
import json

import pytest

from paper_2102_05613_amd import autotune, native


def _make(N=300, M=120, chains=9):
    return lambda w: native.make_config(N, M, chains, 1, 16, precision="split_bf16", tile_cols=w)


def _timer(times, calls):
    def t(make_cfg, init, width, launches, warmup):
        calls.append(width)
        assert make_cfg(width).tile_cols == width
        return times[width]
    return t


def test_picks_the_fastest_width_and_caches_it(tmp_path):
    calls = []
    path = str(tmp_path / "tiles.json")
    r = autotune.tune_tile_cols(_make(), None, cache_path=path, device="dev",
                                timer=_timer({0: 1.6, 128: 3.0, 256: 1.5, 512: 2.0}, calls))
    assert r["tile_cols"] == 256 and not r["cached"]
    assert sorted(calls) == [0, 128, 256, 512]
    with open(path, encoding="utf-8") as f:
        table = json.load(f)
    assert table[r["key"]]["tile_cols"] == 256
    # the same configuration: from the cache, no timing
    again = autotune.tune_tile_cols(_make(), None, cache_path=path, device="dev",
                                    timer=_timer({0: 9.0, 128: 0.1, 256: 9.0, 512: 9.0}, calls))
    assert again["cached"] and again["tile_cols"] == 256 and len(calls) == 4
    # retune times again and replaces the entry
    new = autotune.tune_tile_cols(_make(), None, cache_path=path, device="dev", retune=True,
                                  timer=_timer({0: 9.0, 128: 0.1, 256: 9.0, 512: 9.0}, calls))
    assert new["tile_cols"] == 128 and not new["cached"]


def test_ties_go_to_the_wider_tile_and_the_default_last():
    r = autotune.tune_tile_cols(_make(), None, device="dev",
                                timer=_timer({0: 1.0, 128: 1.0, 256: 1.0, 512: 1.0}, []))
    assert r["tile_cols"] == 512
    r = autotune.tune_tile_cols(_make(), None, device="dev",
                                timer=_timer({0: 1.0, 128: 2.0, 256: 1.0, 512: 3.0}, []))
    assert r["tile_cols"] == 256
    r = autotune.tune_tile_cols(_make(), None, device="dev",
                                timer=_timer({0: 0.5, 128: 2.0, 256: 1.0, 512: 3.0}, []))
    assert r["tile_cols"] == 0


def test_key_separates_devices_and_shapes():
    a = autotune.config_key(_make()(0), "dev0")
    assert a == autotune.config_key(_make()(512), "dev0")     # the width is not part of the key
    assert a != autotune.config_key(_make()(0), "dev1")
    assert a != autotune.config_key(_make(M=121)(0), "dev0")
    b = native.make_batch_config([(64, 8, 4, 1, 4), (128, 16, 4, 1, 4)], tile_cols=0)
    c = native.make_batch_config([(64, 8, 4, 1, 4), (128, 17, 4, 1, 4)], tile_cols=0)
    assert autotune.config_key(b, "dev0") != autotune.config_key(c, "dev0")


@pytest.mark.parametrize("width", [0, 128, 256, 512])
def test_library_accepts_the_tile_widths(width):
    assert native.workspace_size(_make()(width)) > 0


@pytest.mark.parametrize("width", [-1, 64, 100, 1024])
def test_library_rejects_other_tile_widths(width):
    with pytest.raises(native.MC3Error) as e:
        native.workspace_size(_make()(width))
    assert e.value.status == native.MC3_E_ARG
    with pytest.raises(native.MC3Error):
        native.workspace_size(native.make_batch_config([(64, 8, 4, 1, 4)], tile_cols=width))


def _make2(N=128, M=16, chains=4, kmax=4, precision="split_bf16"):
    return lambda scorer, w: native.make_config(N, M, chains, 1, kmax, precision=precision, scorer=scorer,
                                                tile_cols=w)


def _step_timer(times, calls):
    def t(make_cfg, init, scorer, width, steps, warmup, beta):
        cfg = make_cfg(scorer, width)
        assert cfg.tile_cols == width and cfg.scorer == native.SCORERS[scorer]
        calls.append((scorer, width))
        return times[(scorer, width)]
    return t


def test_scorer_choice_times_every_accepted_option(tmp_path):
    calls = []
    times = {("gemm", 0): 0.05, ("gemm", 128): 0.06, ("gemm", 256): 0.04, ("gemm", 512): 0.07, ("delta", 0): 0.01}
    path = str(tmp_path / "sc.json")
    r = autotune.tune_scorer(_make2(), None, cache_path=path, device="dev", timer=_step_timer(times, calls))
    assert (r["scorer"], r["tile_cols"]) == ("delta", 0) and len(calls) == 5
    again = autotune.tune_scorer(_make2(), None, cache_path=path, device="dev", timer=_step_timer(times, calls))
    assert again["cached"] and again["scorer"] == "delta" and len(calls) == 5
    # FP64 pair sums have no tile widths to time
    calls.clear()
    r = autotune.tune_scorer(_make2(precision="fp64"), None, device="dev", timer=_step_timer(times, calls))
    assert sorted(calls) == [("delta", 0), ("gemm", 0)] and r["scorer"] == "delta"


def test_scorer_choice_skips_what_the_library_refuses():
    # a tree with large flip sets: the field-update scorers refuse it
    make = lambda scorer, w: native.make_config(64, 14, 2, 1, 17, precision="split_bf16", scorer=scorer, tile_cols=w,
                                                arity=2)
    calls = []
    times = {("gemm", 0): 0.05, ("gemm", 128): 0.06, ("gemm", 256): 0.04, ("gemm", 512): 0.07, ("delta", 0): 0.0}
    r = autotune.tune_scorer(make, None, device="dev", timer=_step_timer(times, calls))
    assert ("delta", 0) not in calls and (r["scorer"], r["tile_cols"]) == ("gemm", 256)
