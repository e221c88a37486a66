"""mc3_step_n_graph (the launches of mc3_step_n captured once into a HIP graph and
replayed, a step clock in the workspace giving the replayed kernels their step and
beta) against mc3_step_n: states, energies and counters agree bit for bit after every
call, and so do the records and means of every step.

The calls of a run are chosen so that one captures the body and replays it twice, the
next starts at another step residue and captures again, the next reuses that capture,
and a short one runs below the replay threshold; the eager context makes the same
calls, with synchronising reads between them.  Beta anneals over the whole run, so a
replay that gave its selections the wrong step would also use the wrong beta.
"""
import numpy as np
import pytest

from gpu_helpers import announce
from paper_2102_05613_amd import inputs, native

pytestmark = pytest.mark.gpu

# (N, M, chains, kmax, rule, arity, law, precision, couplings)
CASES = [
    (32, 4, 1, 1, "mcmcmc", 0, "uniform", "fp64", "pm1"),            # the small-instance workload
    (32, 1, 1, 1, "metropolis", 0, "uniform", "split_bf16", "pm1"),   # M = 1 Metropolis
    (256, 16, 64, 4, "mcmcmc", 0, "uniform", "split_bf16", "gauss"),  # the anneal workload's shape
    (200, 62, 10, 4, "mcmcmc", 2, "uniform", "fp64", "gauss"),        # binary tree
    (128, 40, 8, 3, "mcmcmc", 1, "line", "split_bf16", "gauss"),      # line graph, log-prior
]

# call lengths: 600 = two replays of a 272-step body and a 56-step tail; 544 from
# step 600 (another residue: captured again, one replay); 544 from step 1144 (the same
# residue: the capture is reused); 100 (no replay)
CALLS = [600, 544, 544, 100]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()


def _ctx(N, M, chains, kmax, rule, arity, law, precision, J, scale, steps, seed):
    cfg = native.make_config(N, M, chains, 1, kmax, precision=precision, rule=rule, trace_steps=steps,
                             seed=seed, mean_steps=steps, arity=arity, law=law)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    return ctx


def _same_state(a, b, where):
    ea, bits_a, sa = a.measure()
    eb, bits_b, sb = b.measure()
    assert np.array_equal(ea, eb), where
    assert np.array_equal(bits_a, bits_b), where
    for k in ("moves", "near_ties", "min_margin", "steps_done"):
        assert sa[k] == sb[k], (where, k)
    return sa


@pytest.mark.parametrize("N,M,chains,kmax,rule,arity,law,precision,couplings", CASES)
def test_graph_replay_matches_step_n(N, M, chains, kmax, rule, arity, law, precision, couplings):
    total = sum(CALLS)
    beta0, beta1, seed = 0.2, 2.5, 17
    announce(f"step_n_graph vs step_n N={N} M={M} chains={chains} {rule} arity={arity} {law} {precision}")
    J, scale = (inputs.couplings_pm1 if couplings == "pm1" else inputs.couplings_gauss)(N, 300 + N + M)
    a = _ctx(N, M, chains, kmax, rule, arity, law, precision, J, scale, total, seed)
    b = _ctx(N, M, chains, kmax, rule, arity, law, precision, J, scale, total, seed)
    t = 0
    for n in CALLS:
        a.step_n(t, n, beta0, beta1, total)
        b.step_n_graph(t, n, beta0, beta1, total)
        t += n
        s = _same_state(a, b, f"after steps 0..{t - 1}")
    assert s["steps_done"] == total
    assert s["moves"] > 0
    ra, rb = a.read_records(0, total), b.read_records(0, total)
    for f in ("r", "vstar", "e_cur", "e_bar", "margin", "flags", "step"):
        assert np.array_equal(ra[f], rb[f]), f
    assert np.array_equal(a.read_means(0, total), b.read_means(0, total))
    a.close()
    b.close()


def test_graph_replay_headline_shape():
    """N=1024, 256 chains x M=128, split BF16: 600 steps through the graph equal 600
    steps of mc3_step_n."""
    N, M, chains, steps = 1024, 128, 256, 600
    announce("step_n_graph headline shape")
    J, scale = inputs.couplings_gauss(N, 0x5EED0003)
    a = _ctx(N, M, chains, 128, "mcmcmc", 0, "uniform", "split_bf16", J, scale, steps, 3)
    b = _ctx(N, M, chains, 128, "mcmcmc", 0, "uniform", "split_bf16", J, scale, steps, 3)
    a.step_n(0, steps, 2.0, 2.0, 1)
    b.step_n_graph(0, steps, 2.0, 2.0, 1)
    _same_state(a, b, "headline")
    ra, rb = a.read_records(0, steps), b.read_records(0, steps)
    for f in ("r", "vstar", "e_cur", "e_bar", "margin", "flags", "step"):
        assert np.array_equal(ra[f], rb[f]), f
    a.close()
    b.close()
