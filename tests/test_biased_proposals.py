"""The state-dependent two-body proposal (single sites drawn with probability
proportional to exp(-alpha dE_i) from the state an edge is generated from) on the
star with a uniform root, on the CPU: the exact transition matrix and the oracle.

Pins: the exact matrix (all roots, all site draws) leaves the Boltzmann law invariant
and is reversible with the generation-probability ratio in the node rule, and is not
without it; at alpha = 0 it is the symmetric single-flip star; the oracle's
fixed-point site weights, site draws and ratio rule follow their definitions exactly;
its one-step transition frequencies match the exact rows."""
import math

import numpy as np
import pytest

import oracle
from exact_tools import all_energies, biased_star_kernel, boltzmann, site_probs, tree_kernel
from test_oracle_chain import _chi2_pass


def _instance(N, seed, pm1=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    if pm1:
        J = np.triu(rng.choice([-1.0, 1.0], size=(N, N)), 1)
    else:
        J = np.triu(rng.normal(size=(N, N)) / math.sqrt(N), 1)
    return J + J.T


@pytest.mark.parametrize("alpha,beta", [(0.5, 0.3), (1.0, 1.5), (3.0, 1.0), (-0.7, 2.0)])
def test_exact_kernel_stationary_and_reversible(alpha, beta):
    N, M = 3, 2
    J = _instance(N, 11)
    E = all_energies(J, 1.0)
    pi = boltzmann(E, beta)
    P = biased_star_kernel(E, beta, N, M, alpha)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(pi @ P, pi, atol=1e-13)
    F = pi[:, None] * P
    assert np.allclose(F, F.T, atol=1e-13)


def test_negative_control_without_the_ratio_is_biased():
    N, M, alpha, beta = 3, 2, 1.5, 1.0
    E = all_energies(_instance(N, 12), 1.0)
    pi = boltzmann(E, beta)
    P = biased_star_kernel(E, beta, N, M, alpha, ratio=False)
    assert np.max(np.abs(pi @ P - pi)) > 1e-3


def test_alpha_zero_is_the_symmetric_single_flip_star():
    N, M, beta = 3, 2, 0.8
    E = all_energies(_instance(N, 13), 1.0)
    P0 = biased_star_kernel(E, beta, N, M, 0.0)
    Ps = tree_kernel(E, beta, N, M, M, 1, 1)
    assert np.allclose(P0, Ps, atol=1e-14)


def test_oracle_site_weights_follow_their_definition():
    """q_i = floor(2^52 exp(a_i - max a)), a_i = -(alpha ((2 scale) (s_i h_i))), h = J s,
    rebuilt in Python (the oracle's exp is pinned to libm elsewhere)."""
    rng = np.random.Generator(np.random.PCG64(3))
    for N, pm1 in ((7, True), (12, False), (30, False)):
        J = _instance(N, 20 + N, pm1)
        scale = 1.0 / math.sqrt(N) if pm1 else 1.0
        for alpha in (0.0, 0.8, -2.0):
            s = rng.choice([-1, 1], size=N).astype(np.int8)
            q, W = oracle.site_weights(J, scale, alpha, s)
            h = [sum(J[i, j] * float(s[j]) for j in range(N)) for i in range(N)]
            a = [-(alpha * ((2.0 * scale) * (float(s[i]) * h[i]))) for i in range(N)]
            amax = max(a)
            qp = [math.floor(oracle.exp(x - amax) * 2.0 ** 52) for x in a]
            assert [int(x) for x in q] == qp
            assert W == sum(qp)


def test_oracle_site_draw_is_the_fixed_point_law():
    """Every draw lands in the site whose interval of [0, W) holds floor(u W / 2^53):
    checked at both edges of every interval; the interval counts give p_i within 2^-50."""
    N = 9
    J = _instance(N, 5)
    s = np.array([1, -1, 1, 1, -1, -1, 1, -1, 1], dtype=np.int8)
    q, W = oracle.site_weights(J, 1.0, 1.3, s)
    Q = list(np.cumsum(np.array([int(x) for x in q], dtype=object)))
    first = [-(-a * 2 ** 53 // W) for a in [0] + Q]
    E = all_energies(J, 1.0)
    c = sum(1 << i for i in range(N) if s[i] < 0)
    p = site_probs(E, N, c, 1.3)
    for i in range(N):
        count = first[i + 1] - first[i]
        assert abs(count / 2 ** 53 - p[i]) < 2.0 ** -50 + 1e-12 * p[i]
        if count:
            assert oracle.draw_site(q, W, first[i]) == i
            assert oracle.draw_site(q, W, first[i + 1] - 1) == i


def test_oracle_ratio_rule_probabilities():
    """The ratio rule picks node v with probability y_v / sum y within 2^-50,
    y_v = exp(-beta (E_v - Emin)) rho_v (checked by exact interval counts)."""
    rng = np.random.Generator(np.random.PCG64(8))
    for beta in (0.4, 2.0):
        E = rng.normal(size=7) * 2
        rho = np.exp(rng.normal(size=7))
        rho[0] = 1.0
        y = [oracle.exp(-(beta * (e - E.min()))) * r for e, r in zip(E, rho)]
        w = [x / max(y) for x in y]
        q = [math.floor(x * 2.0 ** 52) for x in w]
        Q = list(np.cumsum(np.array(q, dtype=object)))
        W = Q[-1]
        first = [-(-a * 2 ** 53 // W) for a in [0] + Q]
        ex = np.exp(-beta * (E - E.min())) * rho
        ex /= ex.sum()
        for v in range(7):
            assert abs((first[v + 1] - first[v]) / 2 ** 53 - ex[v]) < 2.0 ** -50 + 1e-12
            if first[v + 1] > first[v]:
                vs, _, _, Wo = oracle.select_ratio(E, rho, beta, first[v])
                assert vs == v and Wo == W


@pytest.mark.parametrize("alpha,beta", [(1.0, 1.0), (-0.8, 0.5)])
def test_oracle_one_step_frequencies_match_exact_rows(alpha, beta):
    """From each of the 8 states of N = 3 (M = 2), 20000 independent chains take one
    step: the frequencies of the next state agree with the exact row (chi-square)."""
    N, M, chains = 3, 2, 20000
    J = _instance(N, 31)
    E = all_energies(J, 1.0)
    P = biased_star_kernel(E, beta, N, M, alpha)
    for c in range(2 ** N):
        s0 = np.array([-1 if (c >> i) & 1 else 1 for i in range(N)], dtype=np.int8)
        out = oracle.run(J, 1.0, N, M, chains, 1, 1, 77 + c, [beta], spins=np.tile(s0, (chains, 1)),
                         law=oracle.LAW_BIASED, alpha=alpha)
        nxt = ((out["spins"] < 0).astype(np.int64) << np.arange(N)).sum(axis=1)
        counts = np.bincount(nxt, minlength=2 ** N)
        stat, dof = _chi2_pass(counts, P[c], chains)
        assert stat < dof + 6 * np.sqrt(2 * dof), (c, stat, dof)


def test_oracle_records_energies_of_the_chosen_node():
    N, M = 10, 5
    J = _instance(N, 41, pm1=True)
    scale = 1.0 / math.sqrt(N)
    out = oracle.run(J, scale, N, M, 4, 1, 1, 3, np.full(30, 0.9), law=oracle.LAW_BIASED, alpha=0.6)
    for c in range(4):
        assert out["rec"]["e_cur"][-1, c] == oracle.energy(J, scale, out["spins"][c])
    moved = (out["rec"]["vstar"] != out["rec"]["r"]).sum()
    assert moved > 0
