"""Exact checks of the method itself (no oracle involved): the star graph with a
uniform root leaves the Boltzmann distribution invariant, the hub-always-current
reading does not, the paper's two- and three-configuration cases, and the reading of
the line-graph prior."""
import json
import math
import os

import numpy as np
import pytest

from exact_tools import (all_energies, barker_kernel, boltzmann, line_graph_generation,
                         metropolis_kernel, star_kernel, three_config_generation)
from paper_2102_05613_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("N,M,kmin,kmax,beta", [(4, 2, 1, 1, 1.0), (5, 3, 1, 2, 0.3),
                                                (5, 2, 1, 2, 3.0), (4, 3, 1, 2, 1.0)])
def test_star_uniform_root_is_stationary_and_reversible(N, M, kmin, kmax, beta):
    J, scale = inputs.couplings_gauss(N, 100 + N)
    E = all_energies(J, scale)
    pi = boltzmann(E, beta)
    P = star_kernel(E, beta, N, M, kmin, kmax)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
    assert np.max(np.abs(pi @ P - pi)) < 1e-12
    F = pi[:, None] * P
    assert np.max(np.abs(F - F.T)) < 1e-12


def test_star_m1_is_heat_bath():
    N, beta = 5, 0.8
    J, scale = inputs.couplings_gauss(N, 5)
    E = all_energies(J, scale)
    assert np.allclose(star_kernel(E, beta, N, 1, 1, 2), barker_kernel(E, beta, N, 1, 2), atol=1e-13)


def test_metropolis_kernel_is_stationary():
    N, beta = 5, 1.7
    J, scale = inputs.couplings_gauss(N, 6)
    E = all_energies(J, scale)
    pi = boltzmann(E, beta)
    P = metropolis_kernel(E, beta, N, 1, 2)
    assert np.max(np.abs(pi @ P - pi)) < 1e-12


def test_negative_control_hub_always_current_is_biased():
    """Keeping the current state at the hub and weighting nodes by exp(-beta E) is
    not the node rule (P_gen(T|leaf) differs from P_gen(T|hub)): it breaks
    stationarity for M >= 2."""
    N, beta = 5, 2.0
    J, scale = inputs.couplings_gauss(N, 7)
    E = all_energies(J, scale)
    pi = boltzmann(E, beta)
    for M in (2, 3):
        P = star_kernel(E, beta, N, M, 1, 2, root_mode="hub")
        assert np.max(np.abs(pi @ P - pi) / pi) > 1e-2
        # its own stationary law is measurably away from Boltzmann
        w, v = np.linalg.eig(P.T)
        st = np.real(v[:, np.argmin(np.abs(w - 1.0))])
        st = st / st.sum()
        assert 0.5 * np.abs(st - pi).sum() > 2e-3
    # M = 1 is the exception: a two-node graph is symmetric under re-rooting
    P1 = star_kernel(E, beta, N, 1, 1, 2, root_mode="hub")
    assert np.max(np.abs(pi @ P1 - pi)) < 1e-13


def _load_three():
    with open(os.path.join(GOLDEN, "three_configuration.json")) as f:
        return json.load(f)


def _eval_factor(fac, Pprp, p, lab):
    tot = 1.0
    for x in fac:
        if isinstance(x, (int, float)):
            tot *= x
        elif x == "p":
            tot *= p
        elif x == "q":
            tot *= 1 - p
        else:
            _, a, b = x
            tot *= Pprp[lab[b], lab[a]]
    return tot


@pytest.mark.parametrize("p", [0.2, 0.5, 0.8])
def test_three_configuration_generation_probabilities(p):
    """Brute-force enumeration of the three-configuration process reproduces the
    printed P_gen(T|c) for every labelling of a line c0-c1-c2 (middle node c1),
    including the factor 2 at the middle node, for an asymmetric proposal."""
    gold = _load_three()["P_gen_T_given"]
    n = 5
    rng = np.random.Generator(np.random.PCG64(3))
    Pprp = rng.random((n, n))
    np.fill_diagonal(Pprp, 0.0)
    Pprp /= Pprp.sum(axis=1, keepdims=True)
    gen = three_config_generation(Pprp, p)
    checked = 0
    for c0 in range(n):
        for c1 in range(n):
            for c2 in range(n):
                if len({c0, c1, c2}) < 3:
                    continue
                edges = tuple(sorted([tuple(sorted((c0, c1))), tuple(sorted((c1, c2)))]))
                lab = {"c0": c0, "c1": c1, "c2": c2}
                for node in ("c0", "c1", "c2"):
                    want = _eval_factor(gold[node], Pprp, p, lab)
                    got = gen.get((lab[node], edges), 0.0)
                    assert got == pytest.approx(want, rel=1e-12, abs=1e-15)
                    checked += 1
    assert checked == 3 * n * (n - 1) * (n - 2)


@pytest.mark.parametrize("p", [0.2, 0.5, 0.8])
def test_three_configuration_node_rule_is_stationary(p):
    """The graph chain with P_node proportional to P_eq(c) P_gen(T|c) leaves P_eq
    invariant; dropping the printed factor 2 breaks it (unless p makes it vanish)."""
    n = 5
    rng = np.random.Generator(np.random.PCG64(4))
    Pprp = rng.random((n, n))
    np.fill_diagonal(Pprp, 0.0)
    Pprp /= Pprp.sum(axis=1, keepdims=True)
    w = rng.random(n) + 0.1
    pi = w / w.sum()
    gen = three_config_generation(Pprp, p)
    graphs = {}
    for (x, edges), pr in gen.items():
        graphs.setdefault(edges, {})[x] = pr

    def kernel(drop_two):
        P = np.zeros((n, n))
        for (x, edges), pr in gen.items():
            g = dict(graphs[edges])
            if drop_two:
                # remove the factor 2 of the middle node of a line
                deg = {}
                for a, b in edges:
                    deg[a] = deg.get(a, 0) + 1
                    deg[b] = deg.get(b, 0) + 1
                for node in g:
                    if deg[node] == 2:
                        g[node] = g[node] / 2.0
            nodes = sorted({a for e in edges for a in e})
            z = sum(pi[c] * g.get(c, 0.0) for c in nodes)
            for c in nodes:
                P[x, c] += pr * pi[c] * g.get(c, 0.0) / z
        # generation paths that repeat a configuration are not enumerated above; the
        # chain stays put on them (a self-loop cannot affect stationarity)
        P[np.diag_indices(n)] += 1.0 - P.sum(axis=1)
        return P

    P = kernel(False)
    assert np.allclose(P.sum(axis=1), 1.0)
    assert np.max(np.abs(pi @ P - pi)) < 1e-13
    P_bad = kernel(True)
    assert np.max(np.abs(pi @ P_bad - pi)) > 1e-4


@pytest.mark.parametrize("L", [2, 3, 4, 6, 8])
def test_line_graph_prior_reading(L):
    """Line-graph addition process (App. 'Line-graph addition process'): the start
    node ends at position k with probability C(L-1, k) / 2^(L-1).  The printed
    C(L, k) / 2^L does not even normalise over k = 0..L-1, so the reading taken is
    C(L-1, k) / 2^(L-1)."""
    g = line_graph_generation(L)
    for k in range(L):
        assert g[k] == pytest.approx(math.comb(L - 1, k) / 2 ** (L - 1), rel=1e-14)
    printed = np.array([math.comb(L, k) / 2 ** L for k in range(L)])
    assert abs(printed.sum() - 1.0) > 1e-3


# ---------------------------------------------------------------- trees and lines

from exact_tools import tree_kernel  # noqa: E402


def _stationary_and_reversible(P, pi, tol=1e-12):
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-13)
    assert np.max(np.abs(pi @ P - pi)) < tol
    F = pi[:, None] * P
    assert np.max(np.abs(F - F.T)) < tol


@pytest.mark.parametrize("M,arity,kmin,kmax,beta", [(3, 2, 1, 1, 1.3), (4, 2, 1, 2, 0.8), (3, 1, 1, 1, 2.0),
                                                    (4, 3, 1, 1, 1.0)])
def test_tree_uniform_root_is_stationary_and_reversible(M, arity, kmin, kmax, beta):
    """Any tree populated from a uniformly drawn root with a symmetric two-body law
    is self-thermalising (App. 'General graph populating process'): the node rule with
    plain Boltzmann weights leaves the Boltzmann law invariant."""
    N = 3
    J, scale = inputs.couplings_gauss(N, 40 + M + arity)
    E = all_energies(J, scale)
    P = tree_kernel(E, beta, N, M, arity, kmin, kmax)
    _stationary_and_reversible(P, boltzmann(E, beta))
    # arity M is the star of the main path
    if arity == M:
        from exact_tools import star_kernel
        assert np.allclose(P, star_kernel(E, beta, N, M, kmin, kmax), atol=1e-14)


@pytest.mark.parametrize("M", [2, 3])
def test_line_addition_process_needs_its_prior(M):
    """Line-graph addition process (App. 'Line-graph addition process'): the starting
    node sits at position k ~ Binomial(M, 1/2) of a line of L = M+1 nodes, so
    P_gen(T|c_v) carries C(L-1, v) (reading of the garbled prefactor).  With that
    factor in the node weights the chain is stationary; without it, or with the
    printed C(L, v), it is not."""
    N, beta = 3, 1.5
    J, scale = inputs.couplings_gauss(N, 91 + M)
    E = all_energies(J, scale)
    pi = boltzmann(E, beta)
    good = tree_kernel(E, beta, N, M, 1, 1, 1, law="line", prior="comb")
    _stationary_and_reversible(good, pi)
    for bad in ("none", "printed"):
        P = tree_kernel(E, beta, N, M, 1, 1, 1, law="line", prior=bad)
        assert np.max(np.abs(pi @ P - pi)) > 1e-4, bad


@pytest.mark.parametrize("M,arity,table", [
    (3, 3, [0.1, 0.5, 0.3, 0.1]),            # star, hub favoured
    (3, 2, [0.4, 0.0, 0.35, 0.25]),          # binary tree, one node never the root
    (3, 1, [0.05, 0.15, 0.3, 0.5]),          # line, skewed toward the far end
    (4, 2, [1.0, 2.0, 0.5, 3.0, 1.5])])      # unnormalised weights
def test_table_root_law_needs_its_prior(M, arity, table):
    """A populating process with a free root law p_r (App. 'General graph populating
    process'): with symmetric flip sets P_gen(T|c_v) = p_v times a product common to
    the nodes, so node weights exp(-beta E_v) p_v make the chain stationary and
    reversible; plain Boltzmann node weights do not."""
    N, beta = 3, 1.2
    J, scale = inputs.couplings_gauss(N, 300 + M + arity)
    E = all_energies(J, scale)
    pi = boltzmann(E, beta)
    good = tree_kernel(E, beta, N, M, arity, 1, 1, law="table", prior="table", table=table)
    _stationary_and_reversible(good, pi)
    bad = tree_kernel(E, beta, N, M, arity, 1, 1, law="table", prior="none", table=table)
    assert np.max(np.abs(pi @ bad - pi)) > 1e-6   # six orders above the stationary kernel's 1e-12


@pytest.mark.parametrize("p", [0.2, 0.5, 0.8])
def test_three_configuration_process_is_a_table_law(p):
    """The three-configuration process of Sec. 'Generalization to three configurations
    per Monte Carlo step' with symmetric proposals: the printed P_gen(T|c) of the end,
    middle and end nodes are in the ratio q : 2p : q, which is the line of three
    nodes with root weights (q/2, p, q/2); that table law is stationary for every p,
    and p = 1/2 is the line-graph addition process of two additions."""
    gold = _load_three()["P_gen_T_given"]
    n = 4
    rng = np.random.Generator(np.random.PCG64(8))
    A = rng.random((n, n))
    Pprp = A + A.T
    np.fill_diagonal(Pprp, 0.0)
    Pprp /= Pprp.sum()                      # symmetric two-body law
    lab = {"c0": 0, "c1": 1, "c2": 2}       # c1 is the middle node of c0 - c1 - c2
    g = np.array([_eval_factor(gold[c], Pprp, p, lab) for c in ("c0", "c1", "c2")])
    q = 1.0 - p
    table = np.array([q / 2, p, q / 2])
    assert np.allclose(g / g.sum(), table / table.sum(), rtol=1e-12)
    N, beta = 3, 0.9
    J, scale = inputs.couplings_gauss(N, 77)
    E = all_energies(J, scale)
    P = tree_kernel(E, beta, N, 2, 1, 1, 2, law="table", prior="table", table=table)
    _stationary_and_reversible(P, boltzmann(E, beta))
    if p == 0.5:
        assert np.allclose(P, tree_kernel(E, beta, N, 2, 1, 1, 2, law="line", prior="comb"), atol=1e-14)
