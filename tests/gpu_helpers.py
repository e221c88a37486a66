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
             chain_base=0, spins=None, tol=-1.0):
    cfg = native.make_config(N, M, chains, kmin, kmax, precision=precision, rule=rule, trace_steps=trace_steps,
                             seed=seed, chain_base=chain_base, near_tie_tol=tol)
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


LAW_CODES = {"uniform": oracle.LAW_UNIFORM, "line": oracle.LAW_LINE, "table": oracle.LAW_TABLE}


def oracle_candidates(seed, chain, step, N, M, kmin, kmax, s, rule="mcmcmc", arity=None, law="uniform",
                      table=None):
    """Root and the M non-current node configurations in column order."""
    r, nodes = oracle.propose_nodes(seed, chain, step, N, M, kmin, kmax, s,
                                    rule=oracle.RULE_METROPOLIS if rule == "metropolis" else oracle.RULE_MCMCMC,
                                    arity=arity, law=LAW_CODES[law], table=table)
    return r, nodes[column_nodes(M, r)]


def compare_trajectory(gpu_rec, J, scale, N, M, chains, kmin, kmax, seed, betas, rule, energy_rtol,
                       exact=False, chain_base=0, arity=None, law="uniform", table=None):
    """Run the oracle over the same steps, taking the GPU's pick at the steps the GPU
    flagged as near ties (guided replay), and compare every record."""
    steps = len(betas)
    forced = np.where((gpu_rec["flags"] & 1) != 0, gpu_rec["vstar"], -1).astype(np.int32)
    if exact:
        forced[:] = -1
    ro = oracle.run(J, scale, N, M, chains, kmin, kmax, seed, betas,
                    rule=oracle.RULE_METROPOLIS if rule == "metropolis" else oracle.RULE_MCMCMC,
                    forced=forced, chain_base=chain_base, arity=arity, law=LAW_CODES[law], table=table)
    orec = ro["rec"]
    assert np.array_equal(gpu_rec["r"], orec["r"]), "roots differ"
    bad = np.argwhere(gpu_rec["vstar"] != orec["vstar"])
    assert len(bad) == 0, f"selections differ at (step, chain) {bad[:5].tolist()}"
    if exact:
        assert np.array_equal(gpu_rec["e_cur"], orec["e_cur"])
    else:
        np.testing.assert_allclose(gpu_rec["e_cur"], orec["e_cur"], rtol=energy_rtol, atol=energy_rtol)
    # e_bar is a weighted mean of node energies that each carry the path's absolute
    # error, so it takes the same absolute tolerance as e_cur
    np.testing.assert_allclose(gpu_rec["e_bar"], orec["e_bar"], rtol=max(energy_rtol, 1e-12),
                               atol=max(energy_rtol, 1e-12))
    return ro, int((forced >= 0).sum())
