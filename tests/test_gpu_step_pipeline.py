"""mc3_step_n (flip sets drawn up to 16 steps ahead into a ring, one scoring and one
selection launch per step, the selection forming the next step's base words) against
the single-step calls (mc3_propose / mc3_score_candidates / mc3_select) and the oracle.

Both paths read the same partial sums in the same order and apply the same rule, so
their records, states, means and counters agree bit for bit.  The shapes cover one
chain in a scoring tile, many chains in one tile, chains straddling tile edges, chains
spanning several tiles of each width, a tree, the line law and Metropolis; each run is
split over two mc3_step_n calls.
"""
import numpy as np
import pytest

from gpu_helpers import announce, compare_trajectory, eps_energy, gpu_spins
from paper_2102_05613_amd import inputs, native

pytestmark = pytest.mark.gpu

# (N, M, chains, kmax, rule, arity, law, oracle): arity 0 = the star
CASES = [
    (40, 1, 20, 2, "metropolis", 0, "uniform", True),    # 20 chains in one 128-column tile
    (64, 1, 32, 3, "mcmcmc", 0, "uniform", True),        # 32 chains of two nodes
    (300, 120, 9, 16, "mcmcmc", 0, "uniform", True),     # 256-column tiles, chains straddle edges
    (256, 600, 3, 8, "mcmcmc", 0, "uniform", True),      # each chain spans 3-4 tiles
    (160, 1500, 2, 4, "mcmcmc", 0, "uniform", True),     # 512-column tiles, 1501 nodes
    (200, 62, 10, 4, "mcmcmc", 2, "uniform", True),      # binary tree
    (128, 40, 8, 3, "mcmcmc", 1, "line", True),          # line graph, binomial root, log-prior
    (96, 1, 200, 2, "metropolis", 0, "uniform", True),   # 200 chains per tile
]


def _ctx(N, M, chains, kmax, rule, arity, law, J, scale, steps, seed):
    cfg = native.make_config(N, M, chains, 1, kmax, precision="split_bf16", rule=rule, trace_steps=steps,
                             seed=seed, mean_steps=steps, arity=arity, law=law)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    return ctx


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()


@pytest.mark.parametrize("N,M,chains,kmax,rule,arity,law,with_oracle", CASES)
def test_step_n_matches_single_step_calls(N, M, chains, kmax, rule, arity, law, with_oracle):
    steps, seed = 24, 41
    beta = 1.3
    announce(f"step_n vs single steps N={N} M={M} chains={chains} {rule} arity={arity} {law}")
    J, scale = inputs.couplings_gauss(N, 900 + N + M)
    # one step_n call per half: the second starts from the first's carried state
    a = _ctx(N, M, chains, kmax, rule, arity, law, J, scale, steps, seed)
    a.step_n(0, steps // 2, beta, beta, 1)
    a.step_n(steps // 2, steps - steps // 2, beta, beta, 1)
    b = _ctx(N, M, chains, kmax, rule, arity, law, J, scale, steps, seed)
    for t in range(steps):
        b.propose(t)
        b.score_candidates()
        b.select(t, beta)
    ra, rb = a.read_records(0, steps), b.read_records(0, steps)
    for f in ("r", "vstar", "e_cur", "e_bar", "margin", "flags", "step"):
        assert np.array_equal(ra[f], rb[f]), f
    assert np.array_equal(a.read_means(0, steps), b.read_means(0, steps))
    ea, bits_a, sa = a.measure()
    eb, bits_b, sb = b.measure()
    assert np.array_equal(ea, eb)
    assert np.array_equal(bits_a, bits_b)
    for k in ("moves", "near_ties", "min_margin", "steps_done"):
        assert sa[k] == sb[k], k
    assert sa["moves"] > 0
    if with_oracle:
        compare_trajectory(ra, J, scale, N, M, chains, 1, kmax, seed, np.full(steps, beta), rule, 1e-4,
                           arity=arity if arity else None, law=law, eps_e=eps_energy("split_bf16", N),
                           max_forced=3, ecur_rtol=1e-9)
    a.close()
    b.close()


def test_step_n_headline_shape_repeatable():
    """Headline shape (N=1024, 256 chains x M=128): two runs of 20 steps of mc3_step_n
    agree bit for bit, and agree with the single-step calls."""
    N, M, chains, steps = 1024, 128, 256, 20
    announce("step_n headline shape")
    J, scale = inputs.couplings_gauss(N, 0x5EED0003)
    runs = []
    for rep in range(2):
        cfg = native.make_config(N, M, chains, 1, 128, precision="split_bf16", trace_steps=steps, seed=3)
        ctx = native.Context(cfg)
        ctx.init_couplings(J, scale)
        ctx.init_chains()
        ctx.step_n(0, steps, 2.0, 2.0, 1)
        runs.append((ctx.read_records(0, steps), gpu_spins(ctx)))
        ctx.close()
    cfg = native.make_config(N, M, chains, 1, 128, precision="split_bf16", trace_steps=steps, seed=3)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    for t in range(steps):
        ctx.propose(t)
        ctx.score_candidates()
        ctx.select(t, 2.0)
    runs.append((ctx.read_records(0, steps), gpu_spins(ctx)))
    for rec, s in runs[1:]:
        for f in ("r", "vstar", "e_cur", "e_bar", "margin", "flags"):
            assert np.array_equal(rec[f], runs[0][0][f]), f
        assert np.array_equal(s, runs[0][1])


def test_timing_every_kth_launch():
    """mc3_timing_enable(k): events around the first and then every k-th scoring
    launch; k < 0 is an argument error."""
    N, M, chains = 256, 16, 8
    J, scale = inputs.couplings_gauss(N, 77)
    cfg = native.make_config(N, M, chains, 1, 4, precision="split_bf16", seed=1)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    for every, steps, expect in ((1, 5, 5), (4, 10, 3), (16, 16, 1), (16, 17, 2)):
        ctx.timing_enable(True, every=every)
        ctx.step_n(0, steps, 1.0, 1.0, 1)
        ms, launches = ctx.timing_read()
        assert launches == expect, (every, steps)
        assert ms > 0.0
    ctx.timing_enable(False)
    assert native.lib().mc3_timing_enable(ctx.h, -1) == native.MC3_E_ARG
    ctx.close()
