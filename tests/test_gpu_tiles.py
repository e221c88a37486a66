"""Split scoring tile widths (tile_cols 128, 256, 512 and the default by column count)
give the same energies and the same trajectories bit for bit, one instance and a
batch; the autotuner times every width on the device and caches its choice."""
import numpy as np
import pytest

from gpu_helpers import announce
from paper_2102_05613_amd import autotune, inputs, native

pytestmark = pytest.mark.gpu

WIDTHS = (0, 128, 256, 512)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()


def _energies_and_steps(cfg, couplings, steps=12):
    import torch
    ctx = native.Context(cfg)
    for i, (J, scale) in enumerate(couplings):
        ctx.init_couplings(J, scale, instance=i)
    ctx.init_chains()
    ctx.propose(0)
    E = torch.zeros(sum(d[2] * d[1] for d in ctx.instances), dtype=torch.float64, device="cuda")
    ctx.score_candidates(E)
    e = E.cpu().numpy()
    ctx.close()
    ctx = native.Context(cfg)
    for i, (J, scale) in enumerate(couplings):
        ctx.init_couplings(J, scale, instance=i)
    ctx.init_chains()
    ctx.step_n(0, steps, 1.5, 1.5, 1)
    ecur, bits, summ = ctx.measure()
    ctx.close()
    return e, ecur, bits, summ["moves"]


@pytest.mark.parametrize("N,M,chains,kmax", [(300, 120, 9, 16), (1024, 128, 24, 128), (160, 1500, 2, 4)])
def test_widths_agree_single_instance(N, M, chains, kmax):
    announce(f"tile widths N={N} M={M} chains={chains}")
    J, scale = inputs.couplings_gauss(N, 11 + N)
    runs = [_energies_and_steps(native.make_config(N, M, chains, 1, kmax, precision="split_bf16", seed=5,
                                                   tile_cols=w), [(J, scale)]) for w in WIDTHS]
    for w, r in zip(WIDTHS[1:], runs[1:]):
        for a, b in zip(runs[0], r):
            assert np.array_equal(a, b), w
    assert np.all(np.isfinite(runs[0][0]))


def test_widths_agree_batch():
    descs = [(64, 8, 4, 1, 4), (300, 120, 3, 1, 16), (1000, 17, 9, 1, 100), (200, 40, 7, 1, 8)]
    announce("tile widths batch")
    couplings = [inputs.couplings_gauss(d[0], 70 + i) for i, d in enumerate(descs)]
    runs = [_energies_and_steps(native.make_batch_config(descs, precision="split_bf16", seed=9, tile_cols=w),
                                couplings) for w in WIDTHS]
    for w, r in zip(WIDTHS[1:], runs[1:]):
        for a, b in zip(runs[0], r):
            assert np.array_equal(a, b), w


def test_autotuner_on_the_device(tmp_path):
    N, M, chains = 1024, 128, 64
    announce("autotune N=1024 M=128 chains=64")
    J, scale = inputs.couplings_gauss(N, 0x5EED0003)

    def make(w):
        return native.make_config(N, M, chains, 1, 128, precision="split_bf16", seed=3, tile_cols=w)

    def init(ctx):
        ctx.init_couplings(J, scale)
        ctx.init_chains()

    path = str(tmp_path / "tiles.json")
    r = autotune.tune_tile_cols(make, init, launches=8, warmup=2, cache_path=path)
    assert r["tile_cols"] in autotune.WIDTHS and not r["cached"]
    assert set(r["ms"]) == set(autotune.WIDTHS) and all(v > 0 for v in r["ms"].values())
    assert r["ms"][r["tile_cols"]] == min(r["ms"].values())
    assert autotune.tune_tile_cols(make, init, cache_path=path)["cached"]


def test_scorer_tuner_on_the_device(tmp_path):
    """tune_scorer times every scorer the library accepts (split pair sums at each width,
    the field update) and picks one whose timing it reports."""
    N, M, chains = 256, 16, 32
    announce("scorer tuner N=256 M=16")
    J, scale = inputs.couplings_gauss(N, 71)
    make = lambda scorer, w: native.make_config(N, M, chains, 1, 4, precision="split_bf16", seed=2, scorer=scorer,
                                                tile_cols=w)

    def init(ctx):
        ctx.init_couplings(J, scale)
        ctx.init_chains()

    path = str(tmp_path / "scorers.json")
    r = autotune.tune_scorer(make, init, beta=1.0, steps=10, warmup=2, cache_path=path)
    assert set(r["ms"]) == {"gemm:0", "gemm:128", "gemm:256", "gemm:512", "delta:0"}
    assert all(v > 0 for v in r["ms"].values())
    assert r["ms"][f"{r['scorer']}:{r['tile_cols']}"] == min(r["ms"].values())
    assert autotune.tune_scorer(make, init, beta=1.0, cache_path=path)["cached"]
