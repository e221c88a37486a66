"""Exact, brute-force checks of the MCMCMC method (numpy; shares no code with the
oracle or the GPU library).

Everything here enumerates: all 2^N spin states, every flip-set realisation of every
edge, every root position.  These are the independent facts the oracle is pinned to.

States are integers s in [0, 2^N); bit i set means spin i is -1.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, List, Tuple

import numpy as np


def spins_of(states: np.ndarray, N: int) -> np.ndarray:
    """[len(states), N] array of +-1 spins."""
    bits = (states[:, None] >> np.arange(N)[None, :]) & 1
    return (1 - 2 * bits).astype(np.float64)


def all_energies(J: np.ndarray, scale: float) -> np.ndarray:
    """E(s) = -scale * sum_{i<j} J_ij s_i s_j for all 2^N states, via -scale/2 s^T J s
    (J symmetric, zero diagonal)."""
    N = J.shape[0]
    S = spins_of(np.arange(2 ** N), N)
    return -scale * 0.5 * np.einsum("si,ij,sj->s", S, J, S)


def boltzmann(E: np.ndarray, beta: float) -> np.ndarray:
    lw = -beta * (E - E.min())
    w = np.exp(lw)
    return w / w.sum()


def flip_sets(N: int, kmin: int, kmax: int) -> Tuple[np.ndarray, np.ndarray]:
    """All flip sets with kmin <= |F| <= kmax as bitmasks, and their probabilities
    under k ~ U{kmin..kmax}, F uniform among k-subsets."""
    masks, probs = [], []
    nk = kmax - kmin + 1
    for k in range(kmin, kmax + 1):
        c = math.comb(N, k)
        for sub in itertools.combinations(range(N), k):
            masks.append(sum(1 << i for i in sub))
            probs.append(1.0 / (nk * c))
    return np.array(masks, dtype=np.int64), np.array(probs, dtype=np.float64)


def star_kernel(E: np.ndarray, beta: float, N: int, M: int, kmin: int, kmax: int,
                root_mode: str = "uniform", weights: str = "node") -> np.ndarray:
    """Exact transition matrix of one MCMCMC step with the M-ary star, over all root
    positions and all flip-set realisations.

    root_mode "uniform": the current state sits at position r ~ U{0..M} (the
    populating process with uniform root).  root_mode "hub": the current state is
    always the hub (the invalid construction, kept as a negative control).
    weights "node": P_node proportional to exp(-beta E_v) over all M+1 nodes.
    """
    S = 2 ** N
    masks, probs = flip_sets(N, kmin, kmax)
    nF = len(masks)
    P = np.zeros((S, S))
    combos = np.array(list(itertools.product(range(nF), repeat=M)), dtype=np.int64)  # [C, M]
    cprob = np.prod(probs[combos], axis=1)                                          # [C]
    fm = masks[combos]                                                              # [C, M]
    roots = range(M + 1) if root_mode == "uniform" else [0]
    for s in range(S):
        for r in roots:
            pr = 1.0 / len(roots)
            nodes = np.zeros((len(combos), M + 1), dtype=np.int64)
            if r == 0:
                nodes[:, 0] = s
                nodes[:, 1:] = s ^ fm
            else:
                hub = s ^ fm[:, r - 1]
                nodes[:, 0] = hub
                nodes[:, 1:] = hub[:, None] ^ fm
                nodes[:, r] = s
            En = E[nodes]
            lw = -beta * (En - En.min(axis=1, keepdims=True))
            w = np.exp(lw)
            pn = w / w.sum(axis=1, keepdims=True)
            np.add.at(P, (np.full(nodes.shape, s), nodes), pr * cprob[:, None] * pn)
    return P


def barker_kernel(E: np.ndarray, beta: float, N: int, kmin: int, kmax: int) -> np.ndarray:
    """Single-proposal heat-bath (Barker) rate: w'/(w + w')."""
    S = 2 ** N
    masks, probs = flip_sets(N, kmin, kmax)
    P = np.zeros((S, S))
    for s in range(S):
        for m, p in zip(masks, probs):
            t = s ^ m
            a = 1.0 / (1.0 + math.exp(beta * (E[t] - E[s])))
            P[s, t] += p * a
            P[s, s] += p * (1 - a)
    return P


def metropolis_kernel(E: np.ndarray, beta: float, N: int, kmin: int, kmax: int) -> np.ndarray:
    """Single-proposal Metropolis rate min(1, exp(-beta dE))."""
    S = 2 ** N
    masks, probs = flip_sets(N, kmin, kmax)
    P = np.zeros((S, S))
    for s in range(S):
        for m, p in zip(masks, probs):
            t = s ^ m
            a = min(1.0, math.exp(-beta * (E[t] - E[s])))
            P[s, t] += p * a
            P[s, s] += p * (1 - a)
    return P


# ---------------------------------------------------------------- worked examples

def three_config_generation(Pprp: np.ndarray, p: float) -> Dict[Tuple[int, Tuple], float]:
    """Enumerate the three-configuration generation process from every start x:
    draw y1 ~ Pprp[x]; with probability p draw y2 ~ Pprp[x] (both attached to x),
    otherwise y2 ~ Pprp[y1] (attached to y1).  Returns the probability of each
    (start, undirected edge set) with three distinct configurations."""
    n = Pprp.shape[0]
    out: Dict[Tuple[int, Tuple], float] = {}
    for x in range(n):
        for y1 in range(n):
            p1 = Pprp[x, y1]
            for y2 in range(n):
                if len({x, y1, y2}) < 3:
                    continue
                for branch, pb, src in (("star", p, x), ("line", 1 - p, y1)):
                    pr = p1 * pb * Pprp[src, y2]
                    if pr == 0:
                        continue
                    edges = tuple(sorted([tuple(sorted((x, y1))), tuple(sorted((src, y2)))]))
                    key = (x, edges)
                    out[key] = out.get(key, 0.0) + pr
    return out


def line_graph_generation(L: int) -> np.ndarray:
    """Line-graph addition process with a symmetric two-body law, counting only the
    combinatorial factor: starting from one node, add L-1 nodes, each at the left
    or right end with probability 1/2.  Returns g[k] = probability that the starting
    node ends at position k of the line (positions 0..L-1)."""
    g = np.zeros(L)
    for bits in itertools.product((0, 1), repeat=L - 1):
        left = sum(1 for b in bits if b == 0)
        g[left] += 0.5 ** (L - 1)
    return g


# ---------------------------------------------------------------- trees and lines

def tree_parent(v: int, arity: int) -> int:
    """Parent of node v >= 1 in the breadth-first labelling of an arity-ary tree
    (node 0 on top; arity 1 is a line, arity M the M-ary star)."""
    return (v - 1) // arity


def tree_kernel(E: np.ndarray, beta: float, N: int, M: int, arity: int, kmin: int, kmax: int,
                law: str = "uniform", prior: str = "none", table=None) -> np.ndarray:
    """Exact transition matrix of one MCMCMC step on the tree with M+1 nodes
    (breadth-first labelling, parent(v) = (v-1) // arity), every edge populated with an
    independent flip set, over all root positions and all flip-set realisations.

    law "uniform": the current state sits at node r ~ U{0..M} (populating process
    with a uniform root).  law "line" (arity 1): r ~ Binomial(M, 1/2), the position of
    the starting node after M additions at either end of a line.  law "table":
    P(r = v) = table[v] / sum(table), any arity (the populating process with a free
    root law).
    prior: "none" (weights exp(-beta E_v)), "comb" (times C(M, v), the line process's
    generation probability of the graph from node v), or "printed" (times C(M+1, v),
    the printed form) -- the last two for the line law -- or "table" (times table[v],
    the table law's generation probability of the graph from node v).
    Node v's configuration is the current state with the flip sets of every edge on
    the path from r to v flipped."""
    S = 2 ** N
    masks, probs = flip_sets(N, kmin, kmax)
    nF = len(masks)
    V = M + 1
    P = np.zeros((S, S))
    combos = np.array(list(itertools.product(range(nF), repeat=M)), dtype=np.int64)  # edge e = column e-1
    cprob = np.prod(probs[combos], axis=1)
    fm = masks[combos]                                                                # [C, M]
    # path masks from node 0: Ppath[:, v] = xor of the flip sets on the path 0 -> v
    Ppath = np.zeros((len(combos), V), dtype=np.int64)
    for v in range(1, V):
        Ppath[:, v] = Ppath[:, tree_parent(v, arity)] ^ fm[:, v - 1]
    if law == "uniform":
        roots = [(r, 1.0 / V) for r in range(V)]
    elif law == "table":
        tab = np.asarray(table, dtype=np.float64)
        roots = [(r, tab[r] / tab.sum()) for r in range(V) if tab[r] > 0]
    else:
        roots = [(r, math.comb(M, r) / 2 ** M) for r in range(V)]
    if prior == "comb":
        g = np.array([math.comb(M, v) for v in range(V)], dtype=np.float64)
    elif prior == "printed":
        g = np.array([math.comb(M + 1, v) for v in range(V)], dtype=np.float64)
    elif prior == "table":
        g = np.asarray(table, dtype=np.float64)
    else:
        g = np.ones(V)
    for s in range(S):
        for r, pr in roots:
            nodes = s ^ Ppath[:, r:r + 1] ^ Ppath
            En = E[nodes]
            w = np.exp(-beta * (En - En.min(axis=1, keepdims=True))) * g[None, :]
            pn = w / w.sum(axis=1, keepdims=True)
            np.add.at(P, (np.full(nodes.shape, s), nodes), pr * cprob[:, None] * pn)
    return P


# ---------------------------------------------------------------- state-dependent proposals

def site_probs(E: np.ndarray, N: int, c: int, alpha: float) -> np.ndarray:
    """p_i(c) proportional to exp(-alpha (E(c with site i flipped) - E(c))), i = 0..N-1."""
    dE = np.array([E[c ^ (1 << i)] - E[c] for i in range(N)])
    w = np.exp(-alpha * (dE - dE.min()))
    return w / w.sum()


def biased_star_kernel(E: np.ndarray, beta: float, N: int, M: int, alpha: float, ratio: bool = True) -> np.ndarray:
    """Exact transition matrix of one step on the M-ary star with the state-dependent
    single-site proposal: the current state sits at r ~ U{0..M}; r = 0: the hub is the
    current state; r >= 1: the hub is the current state with site i_r flipped,
    i_r ~ p(.|current); every other leaf e is the hub with site i_e ~ p(.|hub)
    flipped.  Node weights exp(-beta E_v) G_v with G_hub = 1 and, for leaf v,
    G_v = p_{i_v}(c_v) / p_{i_v}(hub) -- the graph's generation probability from c_v
    relative to the hub's (ratio=False drops it: the negative control)."""
    S = 2 ** N
    P = np.zeros((S, S))
    probs = {c: site_probs(E, N, c, alpha) for c in range(S)}
    combos = list(itertools.product(range(N), repeat=M))
    for s in range(S):
        for r in range(M + 1):
            for sites in combos:   # sites[e-1] = i_e
                if r == 0:
                    hub = s
                    pr = np.prod([probs[hub][i] for i in sites])
                else:
                    hub = s ^ (1 << sites[r - 1])
                    pr = probs[s][sites[r - 1]] * np.prod([probs[hub][i] for e, i in enumerate(sites, 1) if e != r])
                nodes = [hub] + [hub ^ (1 << i) for i in sites]
                G = [1.0] + [probs[nodes[v]][sites[v - 1]] / probs[hub][sites[v - 1]] for v in range(1, M + 1)]
                if not ratio:
                    G = [1.0] * (M + 1)
                En = E[nodes]
                w = np.exp(-beta * (En - En.min())) * np.array(G)
                pn = w / w.sum()
                for v in range(M + 1):
                    P[s, nodes[v]] += pr / (M + 1) * pn[v]
    return P
