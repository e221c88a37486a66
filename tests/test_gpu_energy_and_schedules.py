"""The carried energy, the periodic FP64 recompute, per-instance schedules, the coupling
mirror, the automatic scorer choice, graph replay on a batch and selections over 1025
nodes.

Bars: the exact energy update keeps the carried energy within FP64 rounding of the
oracle's pair sums on the split path; a drift planted in a checkpoint is counted and
repaired by the next periodic recompute; per-instance schedules give, instance by
instance, the single-instance contexts' records bit for bit; couplings given only
above the diagonal (garbage below) give the trajectory of the full symmetric matrix bit
for bit on every scorer; the automatic scorer equals the scorer its rule names bit for
bit; graph replay on a batch equals mc3_step_n bit for bit; M = 1024 and M = 4000 (the
largest) selections match the oracle (guided at flagged near ties); at N = 8192 the
carried energy equals the oracle's pair sums to FP64 rounding."""
import numpy as np
import pytest

import oracle
from gpu_helpers import announce, compare_trajectory, eps_energy, gpu_spins, make_ctx
from paper_2102_05613_amd import inputs, native

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
@pytest.mark.parametrize("update", ["exact", "scored"])
def test_recompute_and_carried_energy(prec, update):
    """After 50 steps: the explicit recompute equals the oracle's pair sums; the carried
    energy is within FP64 rounding of them with the exact update (both precisions), and
    within the path's node-energy bound with the scored one."""
    N, M, chains = 512, 32, 8
    announce(f"recompute {prec} {update}")
    J, scale = inputs.couplings_gauss(N, 12)
    ctx = make_ctx(N, M, chains, 1, 8, prec, J, scale, seed=1, energy_update=update)
    ctx.step_n(0, 50, 0.5, 0.5, 1)
    e_before, bits, s0 = ctx.measure()
    assert s0["moves"] > 0 and s0["recomputes"] == 0
    ctx.recompute()
    e_after, _, summ = ctx.measure()
    s = native.bits_to_spins(bits, N)
    eo = np.array([oracle.energy(J, scale, s[c]) for c in range(chains)])
    np.testing.assert_allclose(e_after, eo, rtol=1e-12, atol=1e-12)
    assert summ["recomputes"] == 1
    if update == "exact":
        np.testing.assert_allclose(e_before, eo, rtol=1e-10, atol=1e-10)
        assert summ["max_drift"] < 1e-10 and summ["drift_events"] == 0
    else:
        bound = 2 * eps_energy(prec, N)
        assert summ["max_drift"] <= bound
        np.testing.assert_allclose(e_before, eo, rtol=0, atol=bound)


def _find_f64(blob: bytes, value: float) -> int:
    """Byte offset of the one occurrence of an FP64 value in a checkpoint."""
    pat = np.float64(value).tobytes()
    at = blob.find(pat)
    assert at >= 0 and blob.find(pat, at + 1) < 0, "value not unique in the checkpoint"
    return at


@pytest.mark.parametrize("prec", ["split_bf16", "fp64"])
def test_periodic_recompute_detects_and_repairs_drift(prec):
    """recompute_every = 10: a clean run records no drift event over 30 steps (three
    recomputes); a checkpoint whose carried pair sum of chain 3 is off by 0.5 resumes,
    and the recompute after step 29 counts one drift event of 0.5 and carries the
    oracle's energy again."""
    N, M, chains, K = 256, 16, 8, 10
    announce(f"periodic recompute {prec}")
    J, scale = inputs.couplings_gauss(N, 0x5EED0002)
    a = make_ctx(N, M, chains, 1, 4, prec, J, scale, seed=2, recompute_every=K, trace_steps=30)
    a.step_n(0, 20, 0.7, 0.7, 1)
    e20, bits20, s20 = a.measure()
    assert s20["recomputes"] == 2 and s20["drift_events"] == 0 and s20["max_drift"] < 1e-10
    blob = bytearray(a.checkpoint_save())
    a.step_n(20, 10, 0.7, 0.7, 1)
    ea, bits_a, sa = a.measure()
    assert sa["recomputes"] == 3 and sa["drift_events"] == 0
    # chain 3's carried pair sum U = -E / scale, planted off by 0.5
    at = _find_f64(bytes(blob), -e20[3] / scale)
    blob[at:at + 8] = np.float64(-e20[3] / scale + 0.5).tobytes()
    b = make_ctx(N, M, chains, 1, 4, prec, J, scale, seed=2, recompute_every=K, trace_steps=30)
    b.checkpoint_load(bytes(blob))
    b.step_n(20, 10, 0.7, 0.7, 1)
    eb, bits_b, sb = b.measure()
    assert sb["recomputes"] == 3
    assert sb["drift_events"] == 1
    assert abs(sb["max_drift"] - 0.5 * scale) < 1e-6
    s = native.bits_to_spins(bits_b, N)
    eo = np.array([oracle.energy(J, scale, s[c]) for c in range(chains)])
    np.testing.assert_allclose(eb, eo, rtol=1e-12, atol=1e-12)
    # the other chains never saw the planted error
    keep = [c for c in range(chains) if c != 3]
    assert np.array_equal(bits_a[keep], bits_b[keep])


def test_schedules_per_instance_equal_single_contexts():
    """A batch of three instances stepped with a different anneal each (and then one
    selection with a beta per instance) gives each instance's single-instance records
    bit for bit; +-1 couplings follow the oracle exactly."""
    descs = [(64, 4, 2, 1, 2), (96, 8, 3, 1, 3), (40, 1, 2, 1, 1)]
    scheds = [(0.2, 1.8, 40), (1.0, 1.0, 1), (2.5, 0.5, 40)]
    steps, seed, base = 30, 21, 3
    announce("schedules per instance")
    Js = [inputs.couplings_pm1(d[0], 300 + i) for i, d in enumerate(descs)]
    cfg = native.make_batch_config(descs, precision="split_bf16", trace_steps=steps + 1, seed=seed,
                                   chain_base=base)
    bat = native.Context(cfg)
    for i, (J, sc) in enumerate(Js):
        bat.init_couplings(J, sc, instance=i)
    bat.init_chains()
    bat.step_n_schedules(0, steps, scheds)
    betas_last = [2.0, 0.3, 1.1]
    bat.propose(steps)
    bat.score_candidates()
    bat.select_betas(steps, betas_last)
    rec = bat.read_records(0, steps + 1)
    g0 = 0
    for i, (d, (J, sc)) in enumerate(zip(descs, Js)):
        N, M, chains, kmin, kmax = d
        one = make_ctx(N, M, chains, kmin, kmax, "split_bf16", J, sc, trace_steps=steps + 1, seed=seed,
                       chain_base=base + g0)
        one.step_n(0, steps, *scheds[i])
        one.propose(steps)
        one.score_candidates()
        one.select(steps, betas_last[i])
        r1 = one.read_records(0, steps + 1)
        assert np.array_equal(rec[:, g0:g0 + chains], r1), f"instance {i}"
        betas = list(inputs.beta_schedule(scheds[i][0], scheds[i][1], scheds[i][2], 0, steps)) + [betas_last[i]]
        compare_trajectory(r1, J, sc, N, M, chains, kmin, kmax, seed, np.array(betas), "mcmcmc", 0.0, exact=True,
                           chain_base=base + g0)
        one.close()
        g0 += chains
    with pytest.raises(native.MC3Error) as ei:
        bat.step_n_schedules(steps + 1, 1, [(0.1, -1.0, 3), (1.0, 1.0, 1), (1.0, 1.0, 1)])
    assert ei.value.status == native.MC3_E_ARG
    bat.close()


@pytest.mark.parametrize("scorer,prec", [("delta", "fp64"), ("auto", "fp64"), ("gemm", "split_bf16"),
                                         ("gemm", "fp64")])
def test_upper_triangle_only_couplings(scorer, prec):
    """Couplings given above the diagonal only, with NaN, a nonzero diagonal and other
    garbage below it, run exactly as the full symmetric matrix."""
    N, M, chains, steps = 100, 6, 4, 80
    announce(f"upper-triangle couplings {scorer} {prec}")
    J, scale = inputs.couplings_gauss(N, 404)
    Ju = np.triu(J, 1)
    rng = np.random.Generator(np.random.PCG64(5))
    Ju += np.tril(rng.normal(size=(N, N)) * 7.0)
    Ju[10, 3] = np.nan
    Ju[50, 50] = np.inf
    runs = []
    for Jx in (J, Ju):
        ctx = make_ctx(N, M, chains, 1, 3, prec, Jx, scale, seed=4, trace_steps=steps, scorer=scorer)
        ctx.step_n(0, steps, 1.2, 1.2, 1)
        runs.append((ctx.read_records(0, steps), ctx.measure()[1]))
        ctx.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("kmax,arity,expect", [(4, 0, "delta"), (8, 0, "delta"), (9, 0, "gemm"),
                                               (1, 2, "delta"), (3, 2, "gemm")])
def test_auto_scorer_follows_its_rule(kmax, arity, expect):
    """AUTO is the field-update scorer while kmax times the longest path is at most 16
    (star: path 2; binary tree of 15 nodes: path 6), else the pair sum; its records
    equal the named scorer's bit for bit."""
    N, M, chains, steps = 128, 14, 3, 40
    announce(f"auto scorer kmax={kmax} arity={arity}")
    J, scale = inputs.couplings_gauss(N, 55)
    out = []
    for scorer in ("auto", expect):
        ctx = make_ctx(N, M, chains, 1, kmax, "fp64", J, scale, seed=6, trace_steps=steps, scorer=scorer,
                       arity=arity)
        ctx.step_n(0, steps, 1.0, 1.0, 1)
        out.append((ctx.read_records(0, steps), ctx.measure()[1]))
        if expect == "gemm":   # the single-step calls exist on the pair-sum path only
            ctx.propose(steps)
        else:
            with pytest.raises(native.MC3Error):
                ctx.propose(steps)
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_graph_replay_on_a_batch():
    """mc3_step_n_graph on a batch of uneven instances (two tile widths) equals
    mc3_step_n bit for bit: records, means, states and counters."""
    descs = [(64, 4, 2, 1, 2), (200, 9, 3, 1, 5), (129, 40, 5, 1, 3), (64, 1, 4, 1, 2)]
    steps = 600
    announce("graph replay on a batch")
    res = []
    for graph in (False, True):
        cfg = native.make_batch_config(descs, precision="split_bf16", trace_steps=steps, seed=7, mean_steps=steps)
        ctx = native.Context(cfg)
        for i, d in enumerate(descs):
            J, sc = inputs.couplings_gauss(d[0], 70 + i)
            ctx.init_couplings(J, sc, instance=i)
        ctx.init_chains()
        (ctx.step_n_graph if graph else ctx.step_n)(0, steps, 0.3, 2.0, steps)
        e, bits, summ = ctx.measure()
        res.append((ctx.read_records(0, steps), ctx.read_means(0, steps), e, bits, summ))
        ctx.close()
    (ra, ma, ea, ba, sa), (rb, mb, eb, bb, sb) = res
    assert np.array_equal(ra, rb)
    assert np.array_equal(ma, mb)
    assert np.array_equal(ea, eb) and np.array_equal(ba, bb)
    for k in ("moves", "near_ties", "min_margin", "steps_done"):
        assert sa[k] == sb[k], k


@pytest.mark.parametrize("prec", ["split_bf16", "fp64"])
def test_selection_over_1025_nodes_guided(prec):
    """M = 1024 (the large workload's graph size) at small N: selections over 1025
    nodes match the oracle, guided only at flagged near ties."""
    N, M, chains, steps = 96, 1024, 2, 12
    announce(f"M=1024 guided {prec}")
    J, scale = inputs.couplings_gauss(N, 1024)
    ctx = make_ctx(N, M, chains, 1, 6, prec, J, scale, seed=31, trace_steps=steps)
    ctx.step_n(0, steps, 0.8, 0.8, 1)
    rec = ctx.read_records(0, steps)
    assert (rec["flags"] & 2).any()
    compare_trajectory(rec, J, scale, N, M, chains, 1, 6, 31, np.full(steps, 0.8), "mcmcmc",
                       1e-4 if prec == "split_bf16" else 1e-6, eps_e=eps_energy(prec, N), max_forced=2,
                       ecur_rtol=1e-9)


def test_selection_over_the_most_nodes_guided():
    """M = 4000, the largest graph a context accepts, at small N: selections over 4001
    nodes (64 KiB of node energies and weights in LDS) match the oracle, guided only
    at flagged near ties."""
    N, M, chains, steps = 64, 4000, 2, 10
    announce("M=4000 guided")
    J, scale = inputs.couplings_gauss(N, 4000)
    ctx = make_ctx(N, M, chains, 1, 4, "split_bf16", J, scale, seed=37, trace_steps=steps)
    ctx.step_n(0, steps, 0.9, 0.9, 1)
    rec = ctx.read_records(0, steps)
    assert (rec["flags"] & 2).any()
    compare_trajectory(rec, J, scale, N, M, chains, 1, 4, 37, np.full(steps, 0.9), "mcmcmc", 1e-4,
                       eps_e=eps_energy("split_bf16", N), max_forced=2, ecur_rtol=1e-9)


def test_exact_update_at_the_largest_size():
    """N = 8192 (the largest instance) with flip sets of up to 256 sites at a low beta,
    where most chains move: the carried energy after 12 steps (each move's difference
    summed from up to 512 coupling rows of 64 KiB) equals the oracle's pair sums of the
    final states to FP64 rounding, and the FP64 recompute agrees."""
    N, M, chains, steps = 8192, 16, 4, 12
    announce("exact update N=8192")
    J, scale = inputs.couplings_gauss(N, 0x5EED0005)
    ctx = make_ctx(N, M, chains, 1, 256, "split_bf16", J, scale, seed=5)
    ctx.step_n(0, steps, 0.05, 0.05, 1)
    e_carried, bits, summ = ctx.measure()
    assert summ["moves"] >= chains * steps // 2
    s = native.bits_to_spins(bits, N)
    eo = np.array([oracle.energy(J, scale, s[c]) for c in range(chains)])
    np.testing.assert_allclose(e_carried, eo, rtol=1e-10, atol=1e-10)
    ctx.recompute()
    e_rec, _, summ = ctx.measure()
    np.testing.assert_allclose(e_rec, eo, rtol=1e-12, atol=1e-12)
    assert summ["max_drift"] < 1e-9 * (np.abs(eo).max() + 1)
