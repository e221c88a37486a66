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


# ---------------------------------------------------------------- trees and lines

from exact_tools import tree_kernel  # noqa: E402


def test_line_root_is_binomial():
    """The line process's root (number of left additions among M) is Binomial(M, 1/2)."""
    import math
    M, n = 9, 20000
    r = np.array([oracle.root(3, c % 64, c // 64, M, oracle.LAW_LINE) for c in range(n)])
    probs = np.array([math.comb(M, k) / 2 ** M for k in range(M + 1)])
    stat, dof = _chi2_pass(np.bincount(r, minlength=M + 1), probs, n)
    assert stat < dof + 6 * np.sqrt(2 * dof), (stat, dof)


def test_line_log_prior_is_log_binomial():
    import math
    for M in (1, 4, 127):
        lp = oracle.log_prior_line(M)
        exact = np.array([math.log(math.comb(M, v)) for v in range(M + 1)])
        np.testing.assert_allclose(lp, exact, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("M,arity,law,kmin,kmax,beta,start", [
    (3, 2, oracle.LAW_UNIFORM, 1, 1, 1.0, 5),
    (4, 2, oracle.LAW_UNIFORM, 1, 2, 0.8, 11),
    (3, 1, oracle.LAW_LINE, 1, 1, 1.5, 19),
    (3, 1, oracle.LAW_UNIFORM, 1, 1, 1.2, 2),
])
def test_tree_one_step_frequencies_match_exact_row(M, arity, law, kmin, kmax, beta, start):
    N, K = 5, 40000
    J, scale = inputs.couplings_gauss(N, 23)
    E = all_energies(J, scale)
    P = tree_kernel(E, beta, N, M, arity, kmin, kmax, law="line" if law == oracle.LAW_LINE else "uniform",
                    prior="comb" if law == oracle.LAW_LINE else "none")
    s0 = spins_of(np.array([start]), N)[0].astype(np.int8)
    spins = np.repeat(s0[None, :], K, axis=0)
    out = oracle.run(J, scale, N, M, K, kmin, kmax, seed=78, betas=[beta], spins=spins, arity=arity, law=law)
    counts = np.bincount(_states_of(out["spins"]), minlength=2 ** N)
    stat, dof = _chi2_pass(counts, P[start], K)
    assert stat < dof + 6 * np.sqrt(2 * dof), (stat, dof)


def test_tree_nodes_follow_path_rule():
    """Node v of the tree is the current state with the flip sets of the edges between
    the root position and v flipped (checked edge by edge on a binary tree)."""
    N, M, arity = 40, 9, 2
    s = oracle.init_spins(4, N, 0)
    for step in range(6):
        r, nodes = oracle.propose_nodes(4, 0, step, N, M, 1, 3, s, arity=arity)
        F = [None] + [oracle.edge_flips(4, 0, step, e, N, 1, 3)[1].astype(bool) for e in range(1, M + 1)]

        def up(v):
            out = []
            while v:
                out.append(v)
                v = (v - 1) // arity
            return out
        for v in range(M + 1):
            a, b = set(up(r)), set(up(v))
            flip = np.zeros(N, dtype=bool)
            for e in a ^ b:
                flip ^= F[e]
            assert np.array_equal(nodes[v], np.where(flip, -s, s)), (step, r, v)


def test_high_temperature_expansion_at_n64():
    """Beyond exhaustive enumeration: for H = sum_{i<j} J_ij s_i s_j the cumulants under
    the uniform measure are k2 = sum J^2 and k3 = 6 sum_{i<j<k} J_ij J_jk J_ik, so
    <E> = -scale <H> = -beta scale^2 k2 - (beta^2 scale^3 / 2) k3 + O(beta^3).  The
    oracle's long-run node-weighted energy at N = 64, beta = 0.1 agrees within its
    statistical error (chains as independent samples) plus the O(beta^3) term."""
    N, chains, steps, burn, beta = 64, 32, 3000, 300, 0.1
    J, scale = inputs.couplings_gauss(N, 61)
    iu = np.triu_indices(N, 1)
    k2 = float(np.sum(J[iu] ** 2))
    tri = float(np.einsum("ij,jk,ik->", np.triu(J, 1), np.triu(J, 1), np.triu(J, 1)))
    k3 = 6.0 * tri
    e_pred = -beta * scale ** 2 * k2 - 0.5 * beta ** 2 * scale ** 3 * k3
    out = oracle.run(J, scale, N, 8, chains, 1, 4, seed=17, betas=np.full(steps, beta))
    per_chain = out["rec"]["e_bar"][burn:].mean(axis=0)
    m = per_chain.mean()
    se = per_chain.std(ddof=1) / np.sqrt(chains)
    assert abs(m - e_pred) < 5 * se + 0.01, (m, e_pred, se)
    # the leading term alone is resolved: a dropped factor or sign fails
    assert abs(m - 2 * e_pred) > 10 * se and abs(m + e_pred) > 10 * se


# ---------------------------------------------------------------- table root law

@pytest.mark.parametrize("table", [[0.1, 0.5, 0.3, 0.1], [2.0, 0.0, 1.0, 5.0, 0.0, 2.0], [1.0] * 7])
def test_table_root_follows_its_weights(table):
    """Roots drawn under a table law have frequencies table[v] / sum (chi-square over
    20000 chain-steps); weight 0 is never drawn."""
    M, n = len(table) - 1, 20000
    r = np.array([oracle.root(5, c % 64, c // 64, M, oracle.LAW_TABLE, table) for c in range(n)])
    counts = np.bincount(r, minlength=M + 1)
    g = np.asarray(table, dtype=np.float64)
    assert np.all(counts[g == 0] == 0)
    stat, dof = _chi2_pass(counts, g / g.sum(), n)
    assert stat < dof + 6 * np.sqrt(2 * dof), (stat, dof)


def test_table_root_special_cases():
    """One nonzero weight: that node is always the root.  Weights that differ by a
    common factor give the same roots.  Invalid tables are rejected."""
    M = 5
    for v in range(M + 1):
        tab = np.zeros(M + 1)
        tab[v] = 3.0
        assert all(oracle.root(1, c, 7, M, oracle.LAW_TABLE, tab) == v for c in range(50))
    t1 = [1.0, 2.0, 3.0, 4.0, 5.0, 6.0]
    t2 = [x * 4.0 for x in t1]        # a power of two: the same fixed-point weights
    assert [oracle.root(2, c, 3, M, oracle.LAW_TABLE, t1) for c in range(200)] == \
           [oracle.root(2, c, 3, M, oracle.LAW_TABLE, t2) for c in range(200)]
    for bad in ([0.0] * 6, [1.0, -1.0, 1.0, 1.0, 1.0, 1.0], [1.0, float("nan"), 1, 1, 1, 1],
                [1.0, float("inf"), 1, 1, 1, 1]):
        with pytest.raises(ValueError):
            oracle.root_table_cdf(bad)


def test_table_log_prior_is_log_weight():
    """exp of the table law's log-prior is proportional to the weights (to the 2^-52
    resolution of the fixed point); a zero weight gives -infinity."""
    tab = np.array([0.3, 0.0, 1.7, 1e-3, 5.0])
    lp = oracle.log_prior_table(tab)
    assert lp[1] == -np.inf
    ok = tab > 0
    ratio = np.exp(lp[ok] - lp[ok].max())
    np.testing.assert_allclose(ratio, tab[ok] / tab[ok].max(), rtol=1e-12)


@pytest.mark.parametrize("M,arity,table,beta,start", [
    (3, 3, [0.1, 0.5, 0.3, 0.1], 1.0, 6),
    (3, 1, [0.05, 0.15, 0.3, 0.5], 1.4, 13),
    (2, 1, [0.4, 0.2, 0.4], 0.8, 27),          # three-configuration process, p = 0.2
])
def test_table_one_step_frequencies_match_exact_row(M, arity, table, beta, start):
    N, K = 5, 40000
    J, scale = inputs.couplings_gauss(N, 29)
    E = all_energies(J, scale)
    P = tree_kernel(E, beta, N, M, arity, 1, 1, law="table", prior="table", table=table)
    s0 = spins_of(np.array([start]), N)[0].astype(np.int8)
    spins = np.repeat(s0[None, :], K, axis=0)
    out = oracle.run(J, scale, N, M, K, 1, 1, seed=79, betas=[beta], spins=spins, arity=arity,
                     law=oracle.LAW_TABLE, table=table)
    counts = np.bincount(_states_of(out["spins"]), minlength=2 ** N)
    stat, dof = _chi2_pass(counts, P[start], K)
    assert stat < dof + 6 * np.sqrt(2 * dof), (stat, dof)
