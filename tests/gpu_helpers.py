"""Shared helpers of the GPU parity tests (marshalling and comparison only)."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_2102_05613_amd import native


def announce(msg: str):
    sys.stdout.write(f"\n[gpu-case] {msg}\n")
    sys.stdout.flush()


def make_ctx(N, M, chains, kmin, kmax, precision, J, scale, rule="mcmcmc", trace_steps=0, seed=0,
             chain_base=0, spins=None, tol=-1.0, **kw):
    cfg = native.make_config(N, M, chains, kmin, kmax, precision=precision, rule=rule, trace_steps=trace_steps,
                             seed=seed, chain_base=chain_base, near_tie_tol=tol, **kw)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains(spins)
    return ctx


def gpu_spins(ctx) -> np.ndarray:
    _, bits, _ = ctx.measure()
    return native.bits_to_spins(bits, ctx.N)


def column_nodes(M, r):
    """Node held by each candidate column: column m is node m+1, except that for a
    root r >= 1 column r-1 holds the hub (node 0)."""
    return [0 if (r >= 1 and m == r - 1) else m + 1 for m in range(M)]


LAW_CODES = {"uniform": oracle.LAW_UNIFORM, "line": oracle.LAW_LINE, "table": oracle.LAW_TABLE,
             "biased": oracle.LAW_BIASED}


def oracle_candidates(seed, chain, step, N, M, kmin, kmax, s, rule="mcmcmc", arity=None, law="uniform",
                      table=None):
    """Root and the M non-current node configurations in column order."""
    r, nodes = oracle.propose_nodes(seed, chain, step, N, M, kmin, kmax, s,
                                    rule=oracle.RULE_METROPOLIS if rule == "metropolis" else oracle.RULE_MCMCMC,
                                    arity=arity, law=LAW_CODES[law], table=table)
    return r, nodes[column_nodes(M, r)]


def eps_energy(precision: str, N: int) -> float:
    """The library's bound on the rounding error of one node energy, eps_E: N 2^-24 for
    split-BF16 scores (FP32 accumulation of N terms of a field of order one), N 2^-40
    for FP64 scores."""
    return N * 2.0 ** -24 if precision == "split_bf16" else N * 2.0 ** -40


def compare_trajectory(gpu_rec, J, scale, N, M, chains, kmin, kmax, seed, betas, rule, energy_rtol,
                       exact=False, chain_base=0, arity=None, law="uniform", table=None, eps_e=None, tau=None,
                       max_forced=None, ecur_rtol=None, alpha=0.0):
    """Run the oracle over the same steps, taking the GPU's pick at the steps the GPU
    flagged as near ties (guided replay), and compare every record.

    exact: +-1 couplings, no guidance; margins equal bit for bit.  Otherwise:
      eps_e       the path's bound on a node energy's error;
      tau         the GPU's near-tie threshold per step (default 4 beta eps_e);
      max_forced  the most flagged steps the test accepts;
    and the checks are: the GPU flagged exactly the steps whose margin is below tau;
    every margin is within 2 beta eps_e of the oracle's (the largest change energy
    errors of eps_e can make to an interval edge, or to a Metropolis rate) -- so an
    unflagged step picks the node exact arithmetic picks; every forced step is also
    a near tie on the oracle's side (its margin below tau + 2 beta eps_e).
    energy_rtol bounds the node-weighted energies, ecur_rtol (default energy_rtol)
    the carried energies, each as |x - y| <= rtol (|y| + 1)."""
    steps = len(betas)
    betas = np.asarray(betas, dtype=np.float64)
    flagged = (gpu_rec["flags"] & 1) != 0
    forced = np.where(flagged, gpu_rec["vstar"], -1).astype(np.int32)
    if exact:
        forced[:] = -1
    else:
        assert eps_e is not None and max_forced is not None, "guided comparison needs eps_e and max_forced"
    ro = oracle.run(J, scale, N, M, chains, kmin, kmax, seed, betas,
                    rule=oracle.RULE_METROPOLIS if rule == "metropolis" else oracle.RULE_MCMCMC,
                    forced=forced, chain_base=chain_base, arity=arity, law=LAW_CODES[law], table=table, alpha=alpha)
    orec = ro["rec"]
    assert np.array_equal(gpu_rec["r"], orec["r"]), "roots differ"
    bad = np.argwhere(gpu_rec["vstar"] != orec["vstar"])
    assert len(bad) == 0, f"selections differ at (step, chain) {bad[:5].tolist()}"
    mg, mo = gpu_rec["margin"], orec["margin"]
    nforced = int((forced >= 0).sum())
    if exact:
        assert np.array_equal(gpu_rec["e_cur"], orec["e_cur"])
        same = (mg == mo) | (np.isinf(mg) & np.isinf(mo))
        assert np.all(same), f"margins differ at {np.argwhere(~same)[:5].tolist()}"
    else:
        if tau is None:
            tau = betas * (4.0 * eps_e)
        tau_t = np.broadcast_to(np.asarray(tau, dtype=np.float64).reshape(-1, 1), mg.shape) \
            if np.ndim(tau) else np.full(mg.shape, float(tau))
        # the GPU's flag is its own margin below the threshold
        assert np.array_equal(flagged, mg < tau_t), "near-tie flags do not follow the threshold"
        bound = (2.0 * betas * eps_e).reshape(-1, 1) + 1e-12
        fin = np.isfinite(mg) & np.isfinite(mo)
        dm = np.zeros(mg.shape)
        dm[fin] = np.abs(mg[fin] - mo[fin])
        assert np.all(dm <= bound), \
            f"margin differs beyond 2 beta eps_E: worst {float(np.max(dm - bound)):.3e} at {np.unravel_index(np.argmax(dm - bound), dm.shape)}"
        # an infinite margin (Metropolis, dE <= 0) on one side only: the other side
        # accepts too, with a margin that is no near tie
        one_inf = np.isfinite(mg) != np.isfinite(mo)
        assert not np.any(one_inf & flagged), "a flagged step has an infinite margin on one side"
        # forced steps are near ties on the oracle's side as well
        if nforced:
            assert np.all(mo[flagged] <= tau_t[flagged] + bound.repeat(mg.shape[1], axis=1)[flagged]), \
                "a forced step is no near tie on the oracle's side"
        assert nforced <= max_forced, f"{nforced} forced steps > {max_forced}"
        er = energy_rtol if ecur_rtol is None else ecur_rtol
        np.testing.assert_allclose(gpu_rec["e_cur"], orec["e_cur"], rtol=er, atol=er)
    # e_bar is a weighted mean of node energies that each carry the path's absolute
    # error, so it takes the same absolute tolerance as the node energies
    np.testing.assert_allclose(gpu_rec["e_bar"], orec["e_bar"], rtol=max(energy_rtol, 1e-12),
                               atol=max(energy_rtol, 1e-12))
    sys.stdout.write(f"[compare] steps={steps} chains={chains} forced={nforced}\n")
    return ro, nforced
