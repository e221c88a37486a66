"""Batches of SK instances in one context (one set of launches for all instances).

Bars: a batched instance runs bit for bit as a single-instance context over the same
Philox chains; the instance-by-instance launches give the batched result bit for bit;
+-1 couplings give the oracle's trajectory exactly; sampled candidate energies of the
batching workload (2000 instances, N = 64..2048, M = 8..256, 4 chains each) agree with
the oracle within the path's tolerance."""
import numpy as np
import pytest

import oracle
from gpu_helpers import announce, compare_trajectory, eps_energy, oracle_candidates
from paper_2102_05613_amd import inputs, native

pytestmark = pytest.mark.gpu

# (N, M, chains, kmin, kmax): ragged sizes, a one-block instance, M = 1, one chain
DESCS = [(32, 4, 2, 1, 1), (200, 9, 3, 1, 5), (129, 16, 1, 1, 3), (64, 1, 4, 1, 2), (300, 70, 2, 2, 19)]
SEED, BASE = 9, 5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()


def _couplings(kind, i, N):
    return (inputs.couplings_pm1 if kind == "pm1" else inputs.couplings_gauss)(N, 1000 + 17 * i + N)


def _batch(prec, kind, steps, descs=DESCS, beta=(0.5, 2.0)):
    cfg = native.make_batch_config(descs, precision=prec, trace_steps=steps, seed=SEED, chain_base=BASE,
                                   mean_steps=steps)
    ctx = native.Context(cfg)
    for i, d in enumerate(descs):
        J, scale = _couplings(kind, i, d[0])
        ctx.init_couplings(J, scale, instance=i)
    ctx.init_chains()
    return ctx


def _first_chains(descs):
    return np.cumsum([0] + [d[2] for d in descs])[:-1]


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_batch_equals_single_instance_contexts(prec):
    steps = 60
    announce(f"batch vs single contexts {prec}")
    ctx = _batch(prec, "gauss", steps)
    ctx.step_n(0, steps, 0.5, 2.0, steps)
    rec = ctx.read_records(0, steps)
    e, bits, summ = ctx.measure()
    assert summ["steps_done"] == steps
    for i, (d, g0) in enumerate(zip(DESCS, _first_chains(DESCS))):
        N, M, chains, kmin, kmax = d
        J, scale = _couplings("gauss", i, N)
        cfg = native.make_config(N, M, chains, kmin, kmax, precision=prec, trace_steps=steps, seed=SEED,
                                 chain_base=BASE + int(g0))
        one = native.Context(cfg)
        one.init_couplings(J, scale)
        one.init_chains()
        one.step_n(0, steps, 0.5, 2.0, steps)
        r1 = one.read_records(0, steps)
        e1, b1, _ = one.measure()
        one.close()
        sl = slice(int(g0), int(g0) + chains)
        assert np.array_equal(rec[:, sl], r1), f"instance {i}"
        assert np.array_equal(e[sl], e1)
        assert np.array_equal(bits[sl, :b1.shape[1]], b1)
        assert not bits[sl, b1.shape[1]:].any()


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_per_instance_launches_equal_batched(prec):
    steps = 30
    announce(f"per-instance launches vs batched {prec}")
    out = []
    for per_instance in (False, True):
        ctx = _batch(prec, "gauss", steps)
        (ctx.step_n_per_instance if per_instance else ctx.step_n)(0, steps, 0.5, 2.0, steps)
        rec = ctx.read_records(0, steps)
        e, bits, summ = ctx.measure()
        means = ctx.read_means(0, steps)
        ctx.close()
        out.append((rec, e, bits, summ, means))
    (ra, ea, ba, sa, ma), (rb, eb, bb, sb, mb) = out
    assert np.array_equal(ra, rb)
    assert np.array_equal(ea, eb) and np.array_equal(ba, bb)
    assert np.array_equal(ma, mb)
    assert sa == sb


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_batch_pm1_trajectories_match_oracle_exactly(prec):
    steps = 200
    announce(f"batch pm1 vs oracle {prec}")
    ctx = _batch(prec, "pm1", steps)
    ctx.step_n(0, steps, 1.0, 1.0, 1)
    rec = ctx.read_records(0, steps)
    for i, (d, g0) in enumerate(zip(DESCS, _first_chains(DESCS))):
        N, M, chains, kmin, kmax = d
        J, scale = _couplings("pm1", i, N)
        compare_trajectory(rec[:, int(g0):int(g0) + chains], J, scale, N, M, chains, kmin, kmax, SEED,
                           np.ones(steps), "mcmcmc", 0.0, exact=True, chain_base=BASE + int(g0))


def _sampled_energy_check(ctx, descs, prec, step, instances, chains_per, seed, base, coupling):
    import torch
    s_all = ctx.measure()[1]
    ctx.propose(step)
    total = sum(d[1] * d[2] for d in descs)
    E = torch.zeros(total, dtype=torch.float64, device="cuda")
    ctx.score_candidates(E)
    Eg = E.cpu().numpy()
    assert np.all(np.isfinite(Eg))
    g0s = _first_chains(descs)
    col0 = np.cumsum([0] + [d[1] * d[2] for d in descs])[:-1]
    worst = 0.0
    for i in instances:
        N, M, chains, kmin, kmax = descs[i]
        J, scale = coupling(i, N)
        for c in range(min(chains, chains_per)):
            g = int(g0s[i]) + c
            s = native.bits_to_spins(s_all[g], N)
            _, cols = oracle_candidates(seed, base + g, step, N, M, kmin, kmax, s)
            Eo = np.array([oracle.energy(J, scale, x) for x in cols])
            Ec = Eg[int(col0[i]) + c * M:int(col0[i]) + (c + 1) * M]
            np.testing.assert_allclose(Ec, Eo, rtol=0, atol=eps_energy(prec, N))
            worst = max(worst, float(np.max(np.abs(Ec - Eo) / np.maximum(np.abs(Eo), 1e-300))))
    return worst


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_batch_energies_small(prec):
    announce(f"batch energies small {prec}")
    ctx = _batch(prec, "gauss", 0)
    ctx.step_n(0, 3, 1.0, 1.0, 1)
    _sampled_energy_check(ctx, DESCS, prec, 3, range(len(DESCS)), 4, SEED, BASE,
                          lambda i, N: _couplings("gauss", i, N))


def test_batching_workload_full_size_sampled():
    """The batching workload at full size (2000 instances) in the launch configuration
    the benchmark times: two batched steps, then sampled energies of the third step's
    candidates (12 instances spanning the N range, 2 chains each) against the oracle."""
    prec = "split_bf16"
    descs = inputs.batch_descs()
    announce(f"batching workload: {len(descs)} instances, loading couplings")
    w = inputs.workload("sk_batch_rep_n1024_m128")
    cfg = native.make_batch_config(descs, precision=prec, seed=w.seed)
    ctx = native.Context(cfg)
    for i, J, scale in inputs.iter_batch_couplings(descs):
        ctx.init_couplings(J, scale, instance=i)
    ctx.init_chains()
    announce("batching workload: stepping")
    ctx.step_n(0, 2, inputs.BATCH_BETA, inputs.BATCH_BETA, 1)
    Ns = np.array([d[0] for d in descs])
    picks = sorted({int(np.argmin(Ns)), int(np.argmax(Ns))} | set(range(0, 2000, 200)))
    worst = _sampled_energy_check(ctx, descs, prec, 2, picks, 2, w.seed, 0, inputs.batch_couplings)
    print(f"max rel energy error over sampled batch columns: {worst:.3e}")
