"""The field-update scorer (energies as differences from the current state, one
persistent workgroup per chain) against the oracle.

Bars: +-1 couplings give the oracle's trajectories bit for bit (integer pair sums
and fields); Gaussian couplings give the oracle's selections except at flagged near
ties, energies within 1e-9 relative; batches equal single-instance contexts bit for
bit; the means trace equals the per-chain records' means."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_helpers import announce, compare_trajectory, eps_energy
from paper_2102_05613_amd import inputs, native

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()


def _ctx(N, M, chains, kmin, kmax, J, scale, rule="mcmcmc", steps=0, seed=0, chain_base=0, mean_steps=0):
    cfg = native.make_config(N, M, chains, kmin, kmax, precision="fp64", rule=rule, trace_steps=steps, seed=seed,
                             chain_base=chain_base, mean_steps=mean_steps, scorer="delta")
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    return ctx


@pytest.mark.parametrize("M,rule,kmax", [(4, "mcmcmc", 1), (1, "mcmcmc", 1), (1, "metropolis", 1),
                                         (16, "mcmcmc", 4), (7, "mcmcmc", 16)])
def test_pm1_trajectory_bit_exact(M, rule, kmax):
    N, chains, steps = 32, 3, 3000
    announce(f"delta pm1 trajectory M={M} {rule} k<={kmax}")
    J, scale = inputs.couplings_pm1(N, 0x5EED0001)
    ctx = _ctx(N, M, chains, 1, kmax, J, scale, rule=rule, steps=steps, seed=4)
    ctx.step_n(0, steps, 1.0, 1.0, 1)
    rec = ctx.read_records(0, steps)
    compare_trajectory(rec, J, scale, N, M, chains, 1, kmax, 4, np.ones(steps), rule, 0.0, exact=True)
    e, bits, summ = ctx.measure()
    assert summ["steps_done"] == steps and summ["moves"] > 0
    s = native.bits_to_spins(bits, N)
    for c in range(chains):
        assert e[c] == oracle.energy(J, scale, s[c])


def test_pm1_anneal_n256_bit_exact_across_launches():
    """N=256, M=16, flip sets 1..4, beta 0.1 -> 3: 2500 steps in two calls (the second
    spans the 2048-step launch split) equal the oracle's records."""
    N, M, chains, steps = 256, 16, 8, 2500
    announce("delta pm1 anneal N=256")
    J, scale = inputs.couplings_pm1(N, 77)
    ctx = _ctx(N, M, chains, 1, 4, J, scale, steps=steps, seed=2)
    ctx.step_n(0, 100, 0.1, 3.0, steps)
    ctx.step_n(100, steps - 100, 0.1, 3.0, steps)
    rec = ctx.read_records(0, steps)
    betas = inputs.beta_schedule(0.1, 3.0, steps, 0, steps)
    compare_trajectory(rec, J, scale, N, M, chains, 1, 4, 2, betas, "mcmcmc", 0.0, exact=True)


def test_gauss_anneal_guided_and_means():
    """The anneal workload's law (N=256, M=16, k 1..4, Gaussian J, beta 0.1 -> 3) on 16
    chains: selections equal the oracle's except at flagged near ties; the means trace
    equals the means of the records."""
    N, M, chains, steps = 256, 16, 16, 600
    announce("delta gauss anneal")
    J, scale = inputs.couplings_gauss(N, 0x5EED0002)
    ctx = _ctx(N, M, chains, 1, 4, J, scale, steps=steps, seed=2, mean_steps=steps)
    ctx.step_n(0, steps, 0.1, 3.0, steps)
    rec = ctx.read_records(0, steps)
    betas = inputs.beta_schedule(0.1, 3.0, steps, 0, steps)
    ro, nforced = compare_trajectory(rec, J, scale, N, M, chains, 1, 4, 2, betas, "mcmcmc", 1e-9,
                                     eps_e=eps_energy("fp64", N), max_forced=2)
    means = ctx.read_means(0, steps)
    np.testing.assert_allclose(means[:, 0], rec["e_cur"].mean(axis=1), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(means[:, 1], rec["e_bar"].mean(axis=1), rtol=1e-12, atol=1e-12)
    # field and pair sum carried over 600 steps: FP64 recompute differs by rounding only
    e_before, bits, _ = ctx.measure()
    ctx.recompute()
    _, _, summ = ctx.measure()
    assert summ["max_drift"] < 1e-10
    s = native.bits_to_spins(bits, N)
    for c in range(chains):
        assert e_before[c] == pytest.approx(oracle.energy(J, scale, s[c]), rel=1e-12, abs=1e-12)


def test_delta_batch_equals_single_contexts():
    descs = [(32, 4, 2, 1, 1), (200, 9, 3, 1, 5), (129, 16, 1, 2, 3), (64, 1, 4, 1, 2)]
    steps = 300
    announce("delta batch vs single contexts")
    cfg = native.make_batch_config(descs, precision="fp64", trace_steps=steps, seed=9, chain_base=5,
                                   scorer="delta")
    ctx = native.Context(cfg)
    Js = [inputs.couplings_gauss(d[0], 500 + i) for i, d in enumerate(descs)]
    for i, (J, scale) in enumerate(Js):
        ctx.init_couplings(J, scale, instance=i)
    ctx.init_chains()
    ctx.step_n(0, steps, 0.5, 2.0, steps)
    rec = ctx.read_records(0, steps)
    g0 = 0
    for d, (J, scale) in zip(descs, Js):
        N, M, chains, kmin, kmax = d
        one = _ctx(N, M, chains, kmin, kmax, J, scale, steps=steps, seed=9, chain_base=5 + g0)
        one.step_n(0, steps, 0.5, 2.0, steps)
        assert np.array_equal(rec[:, g0:g0 + chains], one.read_records(0, steps))
        one.close()
        g0 += chains


def test_delta_rejects_stepwise_calls():
    J, scale = inputs.couplings_gauss(64, 1)
    ctx = _ctx(64, 4, 2, 1, 2, J, scale)
    for call in (lambda: ctx.propose(0), lambda: ctx.score_candidates(), lambda: ctx.select(0, 1.0),
                 lambda: ctx.read_candidates(), lambda: ctx.step_n_per_instance(0, 1, 1.0, 1.0, 1)):
        with pytest.raises(native.MC3Error) as ei:
            call()
        assert ei.value.status == native.MC3_E_UNSUPPORTED
    ctx.step_n(0, 5, 1.0, 1.0, 1)
    assert ctx.measure()[2]["steps_done"] == 5


# ---------------------------------------------------------------- flip sets of any size (stars)

@pytest.mark.parametrize("N,M,chains,kmin,kmax", [(64, 8, 3, 1, 32), (256, 32, 2, 1, 64), (300, 5, 2, 40, 120)])
def test_star_any_flip_size_pm1_bit_exact(N, M, chains, kmin, kmax):
    """Stars whose flip sets are beyond the small-flip kernel: +-1 trajectories equal the
    oracle's and the matrix-core scorer's bit for bit."""
    steps = 400
    announce(f"delta star pm1 N={N} M={M} k={kmin}..{kmax}")
    J, scale = inputs.couplings_pm1(N, 1300 + N)
    recs = {}
    for scorer in ("delta", "gemm"):
        cfg = native.make_config(N, M, chains, kmin, kmax, precision="fp64", trace_steps=steps, seed=6,
                                 scorer=scorer)
        ctx = native.Context(cfg)
        ctx.init_couplings(J, scale)
        ctx.init_chains()
        ctx.step_n(0, steps, 0.9, 0.9, 1)
        recs[scorer] = (ctx.read_records(0, steps), ctx.measure()[1])
        ctx.close()
    for f in ("r", "vstar", "e_cur", "margin", "flags"):
        assert np.array_equal(recs["delta"][0][f], recs["gemm"][0][f]), f
    assert np.array_equal(recs["delta"][1], recs["gemm"][1])
    compare_trajectory(recs["delta"][0], J, scale, N, M, chains, kmin, kmax, 6, np.full(steps, 0.9), "mcmcmc", 0.0,
                       exact=True)


def test_star_headline_flip_sizes_gauss_guided():
    """The headline's shape of graph (N = 1024, M = 128, flip sets of 1..128 sites) with
    the field-update scorer: 20 steps of 4 chains match the oracle, guided at flagged
    near ties, energies within 1e-9."""
    N, M, chains, steps = 1024, 128, 4, 20
    announce("delta star headline flip sizes")
    J, scale = inputs.couplings_gauss(N, 0x5EED0003)
    cfg = native.make_config(N, M, chains, 1, 128, precision="fp64", trace_steps=steps, seed=3, scorer="delta")
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    ctx.step_n(0, steps, 1.0, 1.0, 1)
    rec = ctx.read_records(0, steps)
    assert (rec["flags"] & 2).any()
    compare_trajectory(rec, J, scale, N, M, chains, 1, 128, 3, np.ones(steps), "mcmcmc", 1e-9,
                       eps_e=eps_energy("fp64", N), max_forced=2, ecur_rtol=1e-9)


def test_star_batch_beyond_64k_lds_pm1_bit_exact():
    """A heterogeneous batch on the star field-update kernel whose per-chain state needs
    more than 64 KiB of LDS (N = 2048, M = 256, flip sets up to 128 sites: 106 KiB): +-1
    trajectories equal the FP64 matrix-core batch bit for bit, and the small instances'
    the oracle's."""
    descs = [(2048, 256, 1, 1, 128), (64, 8, 2, 1, 4), (200, 33, 2, 1, 12), (96, 5, 3, 4, 6)]
    steps = 30
    announce("delta star batch, 106 KiB of LDS")
    Js = [inputs.couplings_pm1(d[0], 1700 + i) for i, d in enumerate(descs)]
    recs = {}
    for scorer in ("delta", "gemm"):
        cfg = native.make_batch_config(descs, precision="fp64", trace_steps=steps, seed=8, chain_base=3,
                                       scorer=scorer)
        ctx = native.Context(cfg)
        for i, (J, scale) in enumerate(Js):
            ctx.init_couplings(J, scale, instance=i)
        ctx.init_chains()
        ctx.step_n(0, steps, 0.7, 0.7, 1)
        recs[scorer] = (ctx.read_records(0, steps), ctx.measure()[1])
        ctx.close()
    for f in ("r", "vstar", "e_cur", "margin", "flags"):
        assert np.array_equal(recs["delta"][0][f], recs["gemm"][0][f]), f
    assert np.array_equal(recs["delta"][1], recs["gemm"][1])
    g0 = descs[0][2]
    for d, (J, scale) in zip(descs[1:], Js[1:]):
        N, M, chains, kmin, kmax = d
        compare_trajectory(recs["delta"][0][:, g0:g0 + chains], J, scale, N, M, chains, kmin, kmax, 8,
                           np.full(steps, 0.7), "mcmcmc", 0.0, exact=True, chain_base=3 + g0)
        g0 += chains


def test_star_n8192_gauss_guided():
    """N = 8192 on the star field-update kernel (133 KiB of LDS per chain): 6 steps of
    2 chains match the oracle, guided at flagged near ties, energies within 1e-9."""
    N, M, chains, steps = 8192, 4, 2, 6
    announce("delta star N=8192")
    J, scale = inputs.couplings_gauss(N, 0x5EED0006)
    cfg = native.make_config(N, M, chains, 1, 3, precision="fp64", trace_steps=steps, seed=12, scorer="delta")
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    ctx.step_n(0, steps, 0.3, 0.3, 1)
    rec = ctx.read_records(0, steps)
    assert (rec["flags"] & 2).any()
    compare_trajectory(rec, J, scale, N, M, chains, 1, 3, 12, np.full(steps, 0.3), "mcmcmc", 1e-9,
                       eps_e=eps_energy("fp64", N), max_forced=2, ecur_rtol=1e-9)
