"""The oracle's chain against exact kernels: one-step transition frequencies from a
fixed state (chi-square against the exact row), and long-run averages against exact
Boltzmann enumeration."""
import numpy as np
import pytest

import oracle
from exact_tools import (all_energies, barker_kernel, boltzmann, metropolis_kernel,
                         spins_of, star_kernel)
from paper_2102_05613_amd import inputs


def _states_of(spins):
    bits = (spins < 0).astype(np.int64)
    return (bits << np.arange(spins.shape[1])[None, :]).sum(axis=1)


def _chi2_pass(counts, probs, n):
    """Pearson chi-square over bins with expected count >= 5 (the rest pooled);
    returns (statistic, dof).  Threshold: mean + 6 sd of chi2(dof)."""
    exp = probs * n
    big = exp >= 5
    obs_b = list(counts[big]) + [counts[~big].sum()]
    exp_b = list(exp[big]) + [exp[~big].sum()]
    obs_b, exp_b = np.array(obs_b, float), np.array(exp_b, float)
    keep = exp_b > 0
    stat = (((obs_b - exp_b) ** 2)[keep] / exp_b[keep]).sum()
    dof = keep.sum() - 1
    return stat, dof


@pytest.mark.parametrize("rule,M,kmin,kmax,beta,start", [
    (oracle.RULE_MCMCMC, 3, 1, 2, 1.0, 5),
    (oracle.RULE_MCMCMC, 2, 1, 1, 2.5, 17),
    (oracle.RULE_MCMCMC, 1, 1, 2, 0.7, 9),
    (oracle.RULE_METROPOLIS, 1, 1, 2, 1.2, 22),
])
def test_one_step_frequencies_match_exact_row(rule, M, kmin, kmax, beta, start):
    N, K = 5, 40000
    J, scale = inputs.couplings_gauss(N, 21)
    E = all_energies(J, scale)
    if rule == oracle.RULE_METROPOLIS:
        P = metropolis_kernel(E, beta, N, kmin, kmax)
    elif M == 1:
        P = barker_kernel(E, beta, N, kmin, kmax)
    else:
        P = star_kernel(E, beta, N, M, kmin, kmax)
    s0 = spins_of(np.array([start]), N)[0].astype(np.int8)
    spins = np.repeat(s0[None, :], K, axis=0)
    out = oracle.run(J, scale, N, M, K, kmin, kmax, seed=77, betas=[beta], spins=spins, rule=rule)
    counts = np.bincount(_states_of(out["spins"]), minlength=2 ** N)
    stat, dof = _chi2_pass(counts, P[start], K)
    assert stat < dof + 6 * np.sqrt(2 * dof), (stat, dof)
    # recorded energies are those of the new states
    Ef = np.array([oracle.energy(J, scale, s) for s in out["spins"][:50]])
    assert np.array_equal(Ef, out["rec"]["e_cur"][0, :50])


@pytest.mark.slow
@pytest.mark.parametrize("rule,M,beta", [(oracle.RULE_MCMCMC, 4, 1.0), (oracle.RULE_MCMCMC, 8, 2.0),
                                         (oracle.RULE_METROPOLIS, 1, 1.0)])
def test_long_run_matches_exact_boltzmann(rule, M, beta):
    N, chains, steps, burn = 10, 16, 4000, 400
    J, scale = inputs.couplings_gauss(N, 31)
    E = all_energies(J, scale)
    pi = boltzmann(E, beta)
    e_exact = float((pi * E).sum())
    out = oracle.run(J, scale, N, M, chains, 1, 2, seed=5, betas=np.full(steps, beta), rule=rule)
    rec = out["rec"][burn:]
    for key in ("e_cur", "e_bar"):
        per_chain = rec[key].mean(axis=0)
        m = per_chain.mean()
        se = per_chain.std(ddof=1) / np.sqrt(chains)
        assert abs(m - e_exact) < 5 * se + 1e-3, (key, m, e_exact, se)


def test_node_energies_recorded_and_nodes_follow_star_rule():
    N, M = 12, 5
    J, scale = inputs.couplings_gauss(N, 8)
    out = oracle.run(J, scale, N, M, 3, 1, 3, seed=9, betas=[0.5, 0.5], want_node_e=True)
    s = np.stack([oracle.init_spins(9, N, c) for c in range(3)])
    for c in range(3):
        r, nodes = oracle.propose_nodes(9, c, 0, N, M, 1, 3, s[c])
        assert out["rec"]["r"][0, c] == r
        assert np.array_equal(nodes[r], s[c])
        for v in range(M + 1):
            assert out["node_e"][0, c, v] == oracle.energy(J, scale, nodes[v])
