"""Trees populated from a root drawn from a caller's table (App. 'General graph
populating process': the root law p_r is free), on the GPU against the oracle: the
three-configuration process with p != 1/2, the line-graph addition process with a
bias toward node 0, a star and a binary tree with skewed weights (some zero).

Bars: roots and candidate bitsets bit-exact; +-1 couplings give the oracle's
trajectories bit for bit on every scorer; Gaussian couplings at N=1024 give the
oracle's selections except at flagged near ties; a batch with a table per instance
runs each instance as its own context would; mc3_step_n equals the single-step calls.
"""
import math

import numpy as np
import pytest

from gpu_helpers import announce, compare_trajectory, eps_energy, gpu_spins, oracle_candidates
from paper_2102_05613_amd import inputs, native

pytestmark = pytest.mark.gpu


def biased_line(M, p):
    """Root weights of the line-graph addition process adding at node 0's end with
    probability p: C(M, v) p^v (1-p)^(M-v)."""
    return [math.comb(M, v) * p ** v * (1 - p) ** (M - v) for v in range(M + 1)]


SHAPES = [  # (M, arity, table, kmin, kmax)
    (2, 1, [0.4, 0.2, 0.4], 1, 1),                      # three-configuration process, p = 0.2
    (2, 1, [0.1, 0.8, 0.1], 1, 2),                      # three-configuration process, p = 0.8
    (15, 1, biased_line(15, 0.3), 1, 1),                # biased line addition
    (12, 12, [3.0] + [0.0, 1.0] * 6, 1, 2),             # star: hub favoured, odd leaves never the root
    (14, 2, [float(v % 4) for v in range(15)], 1, 1)]   # binary tree, every fourth node weight 0


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()


def _ctx(N, M, chains, kmin, kmax, J, scale, arity, table, prec="fp64", scorer="gemm", steps=0, seed=0):
    cfg = native.make_config(N, M, chains, kmin, kmax, precision=prec, trace_steps=steps, seed=seed, scorer=scorer,
                             arity=arity, law="table", law_table=table, mean_steps=steps)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    return ctx


@pytest.mark.parametrize("M,arity,table,kmin,kmax", SHAPES)
def test_table_candidates_bit_exact(M, arity, table, kmin, kmax):
    N, chains = 70, 6
    announce(f"table propose M={M} a={arity}")
    J, scale = inputs.couplings_pm1(N, 5)
    ctx = _ctx(N, M, chains, kmin, kmax, J, scale, arity, table, seed=41)
    s = gpu_spins(ctx)
    roots_seen = set()
    for step in (0, 9, 77, 2 ** 31 + 3):
        ctx.propose(step)
        bits, roots = ctx.read_candidates()
        cand = native.bits_to_spins(bits, N)
        for c in range(chains):
            r, cols = oracle_candidates(41, c, step, N, M, kmin, kmax, s[c], arity=arity, law="table", table=table)
            assert roots[c] == r
            assert table[r] > 0
            assert np.array_equal(cand[c], cols)
            roots_seen.add(int(r))
    assert len(roots_seen) > 1


@pytest.mark.parametrize("M,arity,table,kmin,kmax", SHAPES)
@pytest.mark.parametrize("prec,scorer", [("fp64", "gemm"), ("split_bf16", "gemm"), ("fp64", "delta")])
def test_table_pm1_trajectory_bit_exact(M, arity, table, kmin, kmax, prec, scorer):
    N, chains, steps = 48, 3, 1200
    announce(f"table pm1 trajectory M={M} a={arity} {prec} {scorer}")
    J, scale = inputs.couplings_pm1(N, 0x5EED0001)
    ctx = _ctx(N, M, chains, kmin, kmax, J, scale, arity, table, prec=prec, scorer=scorer, steps=steps, seed=9)
    ctx.step_n(0, steps, 1.0, 1.0, 1)
    rec = ctx.read_records(0, steps)
    compare_trajectory(rec, J, scale, N, M, chains, kmin, kmax, 9, np.ones(steps), "mcmcmc", 0.0, exact=True,
                       arity=arity, law="table", table=table)
    assert ctx.measure()[2]["moves"] > 0


def test_biased_line_gauss_guided():
    """Line of 2^7 nodes grown with probability 0.3 of adding at node 0's end, L = 1024,
    single-spin-flip edges, T = 1, split BF16: 15 steps of 4 chains match the oracle
    (guided at flagged ties)."""
    N, M, chains, steps = 1024, 127, 4, 15
    announce("biased line N=1024")
    table = biased_line(M, 0.3)
    J, scale = inputs.couplings_gauss(N, 0x5EED0003)
    ctx = _ctx(N, M, chains, 1, 1, J, scale, 1, table, prec="split_bf16", steps=steps, seed=12)
    ctx.step_n(0, steps, 1.0, 1.0, 1)
    rec = ctx.read_records(0, steps)
    compare_trajectory(rec, J, scale, N, M, chains, 1, 1, 12, np.ones(steps), "mcmcmc", 1e-4, arity=1, law="table",
                       table=table, eps_e=eps_energy("split_bf16", N), max_forced=3, ecur_rtol=1e-9)


def test_table_batch_matches_single_contexts():
    """A batch with one table per instance (concatenated in instance order) runs each
    instance bit for bit as a single-instance context with the matching chain_base."""
    descs = [(96, 2, 3, 1, 1), (64, 15, 2, 1, 2), (128, 12, 4, 1, 1)]
    tables = [[0.45, 0.1, 0.45], biased_line(15, 0.7), [3.0] + [0.0, 1.0] * 6]
    arities = [1, 1, 1]
    steps = 30
    announce("table batch")
    Js = [inputs.couplings_pm1(d[0], 100 + i) for i, d in enumerate(descs)]
    cfg = native.make_batch_config(descs, precision="fp64", trace_steps=steps, seed=4, arity=1, law="table",
                                   law_table=np.concatenate([np.asarray(t, dtype=np.float64) for t in tables]))
    batch = native.Context(cfg)
    for i, (J, scale) in enumerate(Js):
        batch.init_couplings(J, scale, instance=i)
    batch.init_chains()
    batch.step_n(0, steps, 1.3, 1.3, 1)
    rb = batch.read_records(0, steps)
    g0 = 0
    for i, d in enumerate(descs):
        N, M, chains, kmin, kmax = d
        one = native.make_config(N, M, chains, kmin, kmax, precision="fp64", trace_steps=steps, seed=4,
                                 chain_base=g0, arity=arities[i], law="table", law_table=tables[i])
        ctx = native.Context(one)
        ctx.init_couplings(*Js[i])
        ctx.init_chains()
        ctx.step_n(0, steps, 1.3, 1.3, 1)
        r1 = ctx.read_records(0, steps)
        for f in ("r", "vstar", "e_cur", "e_bar", "margin", "flags"):
            assert np.array_equal(rb[f][:, g0:g0 + chains], r1[f]), (i, f)
        ctx.close()
        g0 += chains
    batch.close()


def test_table_step_n_matches_single_step_calls():
    N, M, chains, steps = 200, 15, 6, 24
    announce("table step_n vs single steps")
    table = biased_line(M, 0.25)
    J, scale = inputs.couplings_gauss(N, 505)
    a = _ctx(N, M, chains, 1, 3, J, scale, 1, table, prec="split_bf16", steps=steps, seed=15)
    a.step_n(0, steps, 1.1, 1.1, 1)
    b = _ctx(N, M, chains, 1, 3, J, scale, 1, table, prec="split_bf16", steps=steps, seed=15)
    for t in range(steps):
        b.propose(t)
        b.score_candidates()
        b.select(t, 1.1)
    ra, rb = a.read_records(0, steps), b.read_records(0, steps)
    for f in ("r", "vstar", "e_cur", "e_bar", "margin", "flags", "step"):
        assert np.array_equal(ra[f], rb[f]), f
    assert np.array_equal(gpu_spins(a), gpu_spins(b))
    compare_trajectory(ra, J, scale, N, M, chains, 1, 3, 15, np.full(steps, 1.1), "mcmcmc", 1e-4,
                       arity=1, law="table", table=table, eps_e=eps_energy("split_bf16", N), max_forced=2,
                       ecur_rtol=1e-9)
