"""The set variant's generation probability (Sec. 'Stochastic generation of the set';
Sec. 'Recursive exponential formula for the generation probability'): the oracle's
sum over insertion orders against closed forms and against a direct simulation of
the process, and the reading of the recursion's garbled prefactor."""
import itertools

import numpy as np
import pytest

import oracle


def _random_G(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    G = rng.random((n, n))
    np.fill_diagonal(G, 0.0)
    return G / G.sum(axis=0, keepdims=True) * 0.9   # column p: law of the new element given parent p


def test_closed_forms():
    G = _random_G(3, 1)
    assert oracle.set_gen_brute(G[:2, :2], 0b01) == pytest.approx(G[1, 0], rel=1e-15)
    assert oracle.set_gen_brute(G[:2, :2], 0b11) == 1.0
    # n = 3 from {0}: add 1 then 2 (parents {0}, then {0, 1}), or 2 then 1
    want = G[1, 0] * (G[2, 0] + G[2, 1]) / 2 + G[2, 0] * (G[1, 0] + G[1, 2]) / 2
    assert oracle.set_gen_brute(G, 0b001) == pytest.approx(want, rel=1e-15)
    # from {0, 1}: the new element 2 from a uniform parent
    assert oracle.set_gen_brute(G, 0b011) == pytest.approx((G[2, 0] + G[2, 1]) / 2, rel=1e-15)
    with pytest.raises(ValueError):
        oracle.set_gen_brute(G, 0)


@pytest.mark.parametrize("X", [0b0001, 0b0101, 0b1110])
def test_brute_force_matches_simulated_process(X):
    """Simulate the process itself on a universe of 6 elements (S = {0..3} plus two
    elements outside S; a new element may repeat one already present): the frequency
    of ending at exactly S matches the oracle's P_gen(S | X) within 5 standard
    deviations over 200000 runs."""
    u, n, runs = 6, 4, 200000
    rng = np.random.Generator(np.random.PCG64(11 + X))
    Gu = rng.random((u, u))
    Gu /= Gu.sum(axis=0, keepdims=True)            # every column a law over the universe
    p = oracle.set_gen_brute(Gu[:n, :n], X)
    start = [e for e in range(n) if (X >> e) & 1]
    adds = n - len(start)
    cum = np.cumsum(Gu, axis=0)
    cur = np.zeros((runs, u), dtype=bool)
    cur[:, start] = True
    size = np.full(runs, len(start))
    for _ in range(adds):
        # a uniform parent among the current elements of each run
        k = (rng.random(runs) * size).astype(np.int64)
        order = np.cumsum(cur, axis=1) - 1
        parent = np.argmax((order == k[:, None]) & cur, axis=1)
        e = (rng.random(runs)[:, None] > cum[:, parent].T).sum(axis=1)
        new = ~cur[np.arange(runs), e]
        cur[np.arange(runs), e] = True
        size = size + new
    # at most n elements are ever present, so holding all of S means being exactly S
    at_S = np.all(cur[:, :n], axis=1)
    assert not np.any(cur[at_S][:, n:])
    hits = int(at_S.sum())
    sd = np.sqrt(p * (1 - p) / runs)
    assert abs(hits / runs - p) < 5 * sd + 1e-12, (hits / runs, p, sd)


def _recursion(G, prefactor):
    """P~_S(S') = P_gen(S | S minus S') by the recursion over the added elements S' with
    the given prefactor(|S'|, |S minus S'|) (test-side transcription of the printed
    formula and of the first-step reading)."""
    n = G.shape[0]
    full = (1 << n) - 1
    P = {0: 1.0}
    for size in range(1, n):
        for Sp in (sum(1 << e for e in c) for c in itertools.combinations(range(n), size)):
            rest = full & ~Sp
            tot = 0.0
            for e1 in range(n):
                if not (Sp >> e1) & 1:
                    continue
                for e2 in range(n):
                    if (rest >> e2) & 1:
                        tot += G[e1, e2] * P[Sp & ~(1 << e1)]
            P[Sp] = prefactor(size, n - size) * tot
    return P


def test_recursion_reading():
    """The recursion's prefactor: conditioning on the first addition gives
    1/|S minus S'| (the size of the set the parent is chosen from), which reproduces the
    sum over insertion orders for every subset; the printed 1/(|S'| |S minus S'|)
    agrees only where |S'| = 1, and the printed one-element case 1/|S| not at all."""
    n = 5
    G = _random_G(n, 7)
    full = (1 << n) - 1
    good = _recursion(G, lambda a, b: 1.0 / b)
    printed = _recursion(G, lambda a, b: 1.0 / (a * b))
    for Sp, v in good.items():
        if Sp == 0:
            continue
        want = oracle.set_gen_brute(G, full & ~Sp)
        assert v == pytest.approx(want, rel=1e-12)
        if bin(Sp).count("1") == 1:
            assert printed[Sp] == pytest.approx(want, rel=1e-12)
            e = Sp.bit_length() - 1
            one = sum(G[e, p] for p in range(n) if p != e) / n      # printed 1/|S|
            assert abs(one - want) > 1e-3 * want
        else:
            assert abs(printed[Sp] - want) > 1e-3 * want
