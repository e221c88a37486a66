"""Pins of the oracle's exp, SK energy and node-selection rule."""
import math

import numpy as np
import pytest

import oracle
from exact_tools import all_energies, spins_of
from paper_2102_05613_amd import inputs


def _ulp_diff(a, b):
    ia = np.array([a], dtype=np.float64).view(np.int64)[0]
    ib = np.array([b], dtype=np.float64).view(np.int64)[0]
    return abs(int(ia) - int(ib))


def test_exp_within_two_ulp_of_libm():
    rng = np.random.Generator(np.random.PCG64(1))
    xs = np.concatenate([-rng.random(20000) * 708.0, -rng.random(5000) * 2.0,
                         np.linspace(-1e-12, 0, 50), -np.arange(0, 700, 0.5)])
    worst = 0
    for x in xs:
        got = oracle.exp(float(x))
        ref = math.exp(float(x))
        worst = max(worst, _ulp_diff(got, ref))
    assert worst <= 2


def test_exp_special_values():
    assert oracle.exp(0.0) == 1.0
    assert oracle.exp(-0.0) == 1.0
    assert oracle.exp(-709.0) == 0.0
    assert oracle.exp(-1e300) == 0.0
    xs = -np.linspace(0, 50, 2001)
    ys = [oracle.exp(float(x)) for x in xs]
    assert all(a >= b for a, b in zip(ys, ys[1:]))


@pytest.mark.parametrize("N,kind", [(2, "gauss"), (7, "gauss"), (12, "pm1"), (33, "gauss")])
def test_energy_invariants(N, kind):
    J, scale = (inputs.couplings_gauss if kind == "gauss" else inputs.couplings_pm1)(N, 3)
    rng = np.random.Generator(np.random.PCG64(N))
    for _ in range(5):
        s = np.where(rng.random(N) < 0.5, -1, 1).astype(np.int8)
        E = oracle.energy(J, scale, s)
        # global spin flip symmetry
        assert oracle.energy(J, scale, -s) == E
        # quadratic-form identity  E = -scale/2 s^T J s
        sf = s.astype(np.float64)
        assert E == pytest.approx(-scale * 0.5 * sf @ J @ sf, rel=1e-13, abs=1e-13)
        # single-flip difference 2 s_i h_i with h = scale * J s
        h = scale * (J @ sf)
        i = int(rng.integers(N))
        s2 = s.copy()
        s2[i] = -s2[i]
        assert oracle.energy(J, scale, s2) - E == pytest.approx(2 * sf[i] * h[i], rel=1e-12, abs=1e-12)
        # multi-flip difference 2 s_F.h - 2 sum_{i,j in F} J_ij s_i s_j
        F = rng.choice(N, size=min(N, 3), replace=False)
        s3 = s.copy()
        s3[F] = -s3[F]
        quad = scale * sf[F] @ J[np.ix_(F, F)] @ sf[F]
        dE = 2 * (sf[F] @ h[F]) - 2 * quad
        assert oracle.energy(J, scale, s3) - E == pytest.approx(dE, rel=1e-12, abs=1e-12)


def test_pm1_energy_is_integer_times_scale():
    N = 32
    J, scale = inputs.couplings_pm1(N, 0x5EED0001)
    assert scale == 1.0 / math.sqrt(32.0)
    rng = np.random.Generator(np.random.PCG64(0))
    for _ in range(20):
        s = np.where(rng.random(N) < 0.5, -1, 1).astype(np.int8)
        sf = s.astype(np.float64)
        n_int = int(round(0.5 * sf @ J @ sf))
        assert oracle.energy(J, scale, s) == -(scale * float(n_int))


def test_energy_ground_state_brute_force():
    N = 10
    J, scale = inputs.couplings_gauss(N, 9)
    E = all_energies(J, scale)
    g = int(np.argmin(E))
    s = spins_of(np.array([g]), N)[0].astype(np.int8)
    assert oracle.energy(J, scale, s) == pytest.approx(E[g], rel=1e-13)
    rng = np.random.Generator(np.random.PCG64(2))
    for st in rng.integers(0, 2 ** N, size=30):
        s = spins_of(np.array([st]), N)[0].astype(np.int8)
        assert oracle.energy(J, scale, s) >= E[g] - 1e-12


# ------------------------------------------------------------------ selection


def _pick_counts(Q, W):
    """Exact number of u53 in [0, 2^53) whose threshold floor(u W / 2^53) lands in
    [Q_{v-1}, Q_v): the smallest u with threshold >= a is ceil(a 2^53 / W)."""
    first = [-(-a * 2 ** 53 // W) for a in [0] + list(Q)]
    return [first[v + 1] - first[v] for v in range(len(Q))]


@pytest.mark.parametrize("beta", [0.0, 0.7, 2.0, 30.0])
def test_select_probabilities_are_the_node_rule(beta):
    """P(v*) = q_v / W with q_v = floor(2^52 exp(-beta (E_v - Emin))): equal to the
    normalised Boltzmann weights of the nodes to within 2^-50 relative."""
    rng = np.random.Generator(np.random.PCG64(4))
    E = rng.normal(size=9) * 2.0
    w = np.exp(-beta * (E - E.min()))
    q = [math.floor(float(x) * 2.0 ** 52) for x in w]
    Q = list(np.cumsum(np.array(q, dtype=object)))
    W = Q[-1]
    counts = _pick_counts(Q, W)
    p_exact = w / w.sum()
    for v in range(len(E)):
        assert abs(counts[v] / 2 ** 53 - p_exact[v]) <= 2.0 ** -50 + 1e-15 * p_exact[v]
    # the oracle's draw at each interval edge and just inside it
    first = [-(-a * 2 ** 53 // W) for a in [0] + Q]
    for v in range(len(E)):
        if counts[v] == 0:
            continue
        for u in (first[v], first[v + 1] - 1):
            vs, _, _, ws = oracle.select_mcmcmc(E, beta, int(u))
            assert vs == v and ws == W


def test_select_two_nodes_is_heat_bath():
    """Two-configuration case (Sec. 'MCMC in the language of graphs'): the node rule
    is the heat-bath rate w1 / (w0 + w1)."""
    for dE in [-3.0, -0.5, 0.0, 0.25, 1.0, 4.0]:
        E = np.array([0.0, dE])
        q = [math.floor(math.exp(-1.3 * (e - E.min())) * 2.0 ** 52) for e in E]
        Q = [q[0], q[0] + q[1]]
        counts = _pick_counts(Q, Q[1])
        hb = 1.0 / (1.0 + math.exp(1.3 * dE))
        assert abs(counts[1] / 2 ** 53 - hb) < 1e-14


def test_metropolis_rule_closed_form():
    for dE in [-1.0, 0.0, 0.3, 2.0]:
        w = math.exp(-0.9 * dE) if dE > 0 else 1.0
        for u in [0, 2 ** 52, 2 ** 53 - 1, int(w * 2 ** 53) - 1, int(w * 2 ** 53) + 1]:
            u = max(0, min(2 ** 53 - 1, u))
            acc, _ = oracle.accept_metropolis(5.0, 5.0 + dE, 0.9, u)
            assert acc == (dE <= 0 or u / 2 ** 53 < w)


def test_select_margin_and_ebar():
    E = np.array([1.0, 0.5, 0.75])
    vs, ebar, margin, W = oracle.select_mcmcmc(E, 1.0, 2 ** 52)
    w = np.exp(-(E - E.min()))
    assert ebar == pytest.approx((w * E).sum() / w.sum(), rel=1e-15)
    assert 0.0 <= margin <= 0.5


@pytest.mark.parametrize("beta", [0.3, 1.7, 9.0])
def test_select_margin_is_the_integer_distance(beta):
    """The selected node and its margin, rebuilt in Python integers from the definition:
    fixed-point weights q_v = floor(2^52 exp(l_v - max l)) with l_v = -(beta (E_v - Emin))
    (the oracle's own exp, pinned to libm above), Q_v their running sums, W = Q_M,
    t = floor(u W / 2^53), v* = the first v with Q_v > t, and margin
    min(t - Q_{v*-1}, Q_{v*} - t) / W.  An off-by-one in either distance, a wrong
    interval edge or a threshold taken in floating point fails."""
    rng = np.random.Generator(np.random.PCG64(7))
    hit_lo = hit_hi = 0
    for trial in range(400):
        nodes = int(rng.integers(2, 40))
        E = rng.normal(size=nodes) * 3.0
        emin = float(E.min())
        ls = [-(beta * (float(e) - emin)) for e in E]
        lmax = max(ls)
        q = [math.floor(oracle.exp(l - lmax) * 2.0 ** 52) for l in ls]
        Q = list(np.cumsum(np.array(q, dtype=object)))
        W = Q[-1]
        # draws near interval edges as well as anywhere
        if trial % 2:
            v = int(rng.integers(0, nodes))
            edge = Q[v - 1] if v else 0
            u = max(0, min(2 ** 53 - 1, -(-edge * 2 ** 53 // W) + int(rng.integers(-3, 4))))
        else:
            u = int(rng.integers(0, 2 ** 53))
        t = (u * W) >> 53
        vs = next(v for v in range(nodes) if Q[v] > t)
        lo = Q[vs - 1] if vs else 0
        d1, d2 = t - lo, Q[vs] - t
        hit_lo += d1 < d2
        hit_hi += d2 < d1
        margin = float(min(d1, d2)) / float(W)
        v_o, _, m_o, W_o = oracle.select_mcmcmc(E, beta, u)
        assert (v_o, W_o) == (vs, W)
        assert m_o == margin, (trial, m_o, margin)
    assert hit_lo > 20 and hit_hi > 20   # both distances decided some margins
