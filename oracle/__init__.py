"""CPU oracle for many-configuration MCMC (MCMCMC) on the SK spin glass.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path (the HIP library under
``paper_2102_05613_amd``) never imports this package, and this package never imports
the product.  The arithmetic lives in ``mc3_oracle.c`` (plain FP64 C, compiled with
``-O2 -ffp-contract=off``); this module only marshals arguments with ctypes.

Every function cites the passage of the paper it follows (see ``mc3_oracle.c``):
SK energy (Sec. "The Sherrington-Kirkpatrick model"), node rule of the graph chain
(App. "Markov chain of graphs of configurations", Eq. eq_det_balance_graph_solution),
populating process with a uniform root or a root law given as a table, and the
line-graph addition process (App. "Generating graphs of configurations"), Metropolis
rate (Sec. "Problem statement").

Parity pins (tests/test_oracle_*.py): Philox known-answer vectors and an independent
Philox implementation; Floyd by exhaustive enumeration; exp against libm within 2 ulp;
energy invariants and brute force; exact transition matrices (stationarity, detailed
balance, heat-bath at M=1, Metropolis closed form) against the oracle's one-step
frequencies; long-run Boltzmann averages by exhaustive enumeration.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mc3_oracle.c")
_LIB = os.path.join(_HERE, "libmc3_oracle.so")

TAG_INIT, TAG_ROOT, TAG_EDGE, TAG_SELECT = 1, 2, 3, 4
RULE_MCMCMC, RULE_METROPOLIS = 0, 1
LAW_UNIFORM, LAW_LINE, LAW_TABLE, LAW_BIASED = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Rec(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("vstar", ctypes.c_int32), ("e_cur", ctypes.c_double),
                ("e_bar", ctypes.c_double), ("margin", ctypes.c_double), ("wsum", ctypes.c_uint64)]


class Cfg(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("chains", ctypes.c_int32),
                ("kmin", ctypes.c_int32), ("kmax", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("chain_base", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("scale", ctypes.c_double), ("arity", ctypes.c_int32),
                ("law", ctypes.c_int32), ("pad2", ctypes.c_int32), ("table", ctypes.POINTER(ctypes.c_double)),
                ("alpha", ctypes.c_double)]


REC_DTYPE = np.dtype([("r", np.int32), ("vstar", np.int32), ("e_cur", np.float64),
                      ("e_bar", np.float64), ("margin", np.float64), ("wsum", np.uint64)])

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.POINTER
        u32, u64, i32, dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        L.mc3o_philox.argtypes = [P(u32), P(u32), P(u32)]
        L.mc3o_word.argtypes = [u64, u32, u32, u32, u32, u32]
        L.mc3o_word.restype = u32
        L.mc3o_randint.argtypes = [u32, u32]
        L.mc3o_randint.restype = u32
        L.mc3o_u53.argtypes = [u32, u32]
        L.mc3o_u53.restype = u64
        L.mc3o_exp.argtypes = [dbl]
        L.mc3o_exp.restype = dbl
        L.mc3o_floyd_words.argtypes = [i32, i32, P(u32), P(ctypes.c_uint8)]
        L.mc3o_energy.argtypes = [i32, P(dbl), dbl, P(ctypes.c_int8)]
        L.mc3o_energy.restype = dbl
        L.mc3o_init_spins.argtypes = [u64, i32, u32, P(ctypes.c_int8)]
        L.mc3o_edge_flips.argtypes = [u64, u32, u32, u32, i32, i32, i32, P(ctypes.c_uint8)]
        L.mc3o_edge_flips.restype = i32
        L.mc3o_root.argtypes = [u64, u32, u32, i32]
        L.mc3o_root.restype = i32
        L.mc3o_root_line.argtypes = [u64, u32, u32, i32]
        L.mc3o_root_line.restype = i32
        L.mc3o_log_prior_line.argtypes = [i32, P(dbl)]
        L.mc3o_root_table_prepare.argtypes = [i32, P(dbl), P(u64)]
        L.mc3o_root_table_prepare.restype = i32
        L.mc3o_root_table.argtypes = [u64, u32, u32, i32, P(u64)]
        L.mc3o_root_table.restype = i32
        L.mc3o_log_prior_table.argtypes = [i32, P(u64), P(dbl)]
        L.mc3o_set_gen_brute.argtypes = [i32, P(dbl), u32, P(i32)]
        L.mc3o_couplings.argtypes = [i32, i32, u64, P(dbl)]
        L.mc3o_couplings.restype = ctypes.c_int
        L.mc3o_set_gen_brute.restype = dbl
        L.mc3o_build_nodes.argtypes = [i32, i32, i32, i32, P(ctypes.c_int8), P(ctypes.c_uint8), P(ctypes.c_int8)]
        L.mc3o_select_mcmcmc.argtypes = [i32, P(dbl), P(dbl), dbl, u64, P(dbl), P(dbl), P(u64)]
        L.mc3o_select_mcmcmc.restype = i32
        L.mc3o_accept_metropolis.argtypes = [dbl, dbl, dbl, u64, P(dbl)]
        L.mc3o_accept_metropolis.restype = i32
        L.mc3o_site_weights.argtypes = [i32, P(dbl), dbl, dbl, P(ctypes.c_int8), P(u64)]
        L.mc3o_site_weights.restype = u64
        L.mc3o_draw_site.argtypes = [i32, P(u64), u64, u64]
        L.mc3o_draw_site.restype = i32
        L.mc3o_select_ratio.argtypes = [i32, P(dbl), P(dbl), dbl, u64, P(dbl), P(dbl), P(u64)]
        L.mc3o_select_ratio.restype = i32
        L.mc3o_biased_step.argtypes = [i32, i32, P(dbl), dbl, dbl, dbl, u64, u32, u32, P(ctypes.c_int8),
                                       P(ctypes.c_int8), P(dbl), P(dbl), P(i32), P(dbl), P(dbl)]
        L.mc3o_biased_step.restype = i32
        L.mc3o_run.argtypes = [P(Cfg), P(dbl), P(ctypes.c_int8), P(dbl), u64, ctypes.c_int64,
                               P(dbl), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.mc3o_run.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().mc3o_philox(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def word(seed: int, tag: int, chain: int, step: int, edge: int, n: int) -> int:
    return int(lib().mc3o_word(seed, tag, chain, step, edge, n))


def randint(w: int, n: int) -> int:
    return int(lib().mc3o_randint(w, n))


def u53(w0: int, w1: int) -> int:
    return int(lib().mc3o_u53(w0, w1))


def exp(x: float) -> float:
    return float(lib().mc3o_exp(float(x)))


def floyd_words(N: int, k: int, words) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint32)
    m = np.zeros(N, dtype=np.uint8)
    lib().mc3o_floyd_words(N, k, _ptr(w, ctypes.c_uint32), _ptr(m, ctypes.c_uint8))
    return m


COUPLINGS_PM1, COUPLINGS_GAUSS = 0, 1


def couplings(N: int, kind: int, seed: int):
    """(J, scale) of the seeded instance generator: kind 0 +-1 couplings with scale
    1/sqrt(N), kind 1 Gaussian couplings of variance 1/N with scale 1."""
    J = np.zeros((N, N), dtype=np.float64)
    if lib().mc3o_couplings(N, kind, seed, _ptr(J, ctypes.c_double)) != 0:
        raise ValueError("unknown coupling kind")
    return J, (1.0 / math.sqrt(N) if kind == COUPLINGS_PM1 else 1.0)


def energy(J: np.ndarray, scale: float, s: np.ndarray) -> float:
    J = np.ascontiguousarray(J, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return float(lib().mc3o_energy(J.shape[0], _ptr(J, ctypes.c_double), scale, _ptr(s, ctypes.c_int8)))


def init_spins(seed: int, N: int, chain: int) -> np.ndarray:
    s = np.zeros(N, dtype=np.int8)
    lib().mc3o_init_spins(seed, N, chain, _ptr(s, ctypes.c_int8))
    return s


def edge_flips(seed, chain, step, edge, N, kmin, kmax):
    m = np.zeros(N, dtype=np.uint8)
    k = lib().mc3o_edge_flips(seed, chain, step, edge, N, kmin, kmax, _ptr(m, ctypes.c_uint8))
    return int(k), m


def root_table_cdf(table) -> np.ndarray:
    """Fixed-point cumulative root weights Q_0..Q_M of a table law (mc3o_root_table_prepare)."""
    g = np.ascontiguousarray(table, dtype=np.float64)
    Q = np.zeros(len(g), dtype=np.uint64)
    if lib().mc3o_root_table_prepare(len(g) - 1, _ptr(g, ctypes.c_double), _ptr(Q, ctypes.c_uint64)) != 0:
        raise ValueError("root table needs nonnegative finite weights with a positive fixed-point total")
    return Q


def log_prior_table(table) -> np.ndarray:
    """log q_v of a table law: the node rule's log-prior."""
    Q = root_table_cdf(table)
    out = np.zeros(len(Q), dtype=np.float64)
    lib().mc3o_log_prior_table(len(Q) - 1, _ptr(Q, ctypes.c_uint64), _ptr(out, ctypes.c_double))
    return out


def root(seed, chain, step, M, law: int = LAW_UNIFORM, table=None) -> int:
    """Root position: uniform over the M+1 nodes, the line process's left count, or a
    draw from a table law."""
    if law == LAW_LINE:
        return int(lib().mc3o_root_line(seed, chain, step, M))
    if law == LAW_TABLE:
        Q = root_table_cdf(table)
        assert len(Q) == M + 1
        return int(lib().mc3o_root_table(seed, chain, step, M, _ptr(Q, ctypes.c_uint64)))
    return int(lib().mc3o_root(seed, chain, step, M))


def log_prior_line(M: int) -> np.ndarray:
    """log C(M, v), v = 0..M: the line-graph addition process's log-prior."""
    out = np.zeros(M + 1, dtype=np.float64)
    lib().mc3o_log_prior_line(M, _ptr(out, ctypes.c_double))
    return out


def propose_nodes(seed, chain, step, N, M, kmin, kmax, s, rule=RULE_MCMCMC, arity: Optional[int] = None,
                  law: int = LAW_UNIFORM, table=None):
    """Root and node configurations [(M+1), N] of the tree (arity a, default the star
    a = M) generated from s."""
    arity = M if arity is None else arity
    r = 0 if rule == RULE_METROPOLIS else root(seed, chain, step, M, law, table)
    flips = np.zeros((M + 1, N), dtype=np.uint8)
    for e in range(1, M + 1):
        flips[e] = edge_flips(seed, chain, step, e, N, kmin, kmax)[1]
    nodes = np.zeros((M + 1, N), dtype=np.int8)
    s = np.ascontiguousarray(s, dtype=np.int8)
    lib().mc3o_build_nodes(N, M, arity, r, _ptr(s, ctypes.c_int8), _ptr(flips, ctypes.c_uint8),
                           _ptr(nodes, ctypes.c_int8))
    return r, nodes


def select_mcmcmc(E, beta: float, u53_value: int, log_prior=None):
    """Returns (vstar, e_bar, margin, W)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    lp = None if log_prior is None else np.ascontiguousarray(log_prior, dtype=np.float64)
    eb, mg, ws = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint64()
    v = lib().mc3o_select_mcmcmc(len(E), _ptr(E, ctypes.c_double),
                                 None if lp is None else _ptr(lp, ctypes.c_double),
                                 beta, u53_value, ctypes.byref(eb), ctypes.byref(mg), ctypes.byref(ws))
    return int(v), eb.value, mg.value, int(ws.value)


def accept_metropolis(e_cur: float, e_new: float, beta: float, u53_value: int):
    mg = ctypes.c_double()
    a = lib().mc3o_accept_metropolis(e_cur, e_new, beta, u53_value, ctypes.byref(mg))
    return bool(a), mg.value


def site_weights(J: np.ndarray, scale: float, alpha: float, s: np.ndarray):
    """Fixed-point site weights q [N] (uint64) and their total W of the biased
    single-site proposal from state s."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.int8)
    q = np.zeros(J.shape[0], dtype=np.uint64)
    W = lib().mc3o_site_weights(J.shape[0], _ptr(J, ctypes.c_double), scale, alpha, _ptr(s, ctypes.c_int8),
                                _ptr(q, ctypes.c_uint64))
    return q, int(W)


def draw_site(q: np.ndarray, W: int, u53_value: int) -> int:
    q = np.ascontiguousarray(q, dtype=np.uint64)
    return int(lib().mc3o_draw_site(len(q), _ptr(q, ctypes.c_uint64), W, u53_value))


def select_ratio(E, rho, beta: float, u53_value: int):
    """Node rule with generation-probability ratios rho; returns (vstar, e_bar, margin, W)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    eb, mg, ws = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint64()
    v = lib().mc3o_select_ratio(len(E), _ptr(E, ctypes.c_double), _ptr(rho, ctypes.c_double), beta, u53_value,
                                ctypes.byref(eb), ctypes.byref(mg), ctypes.byref(ws))
    return int(v), eb.value, mg.value, int(ws.value)


def biased_step(J, scale, alpha, beta, seed, chain, step, s, M):
    """One step of the biased single-site star from state s: dict(r, vstar, nodes
    [(M+1), N], E, rho, e_bar, margin)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    N = J.shape[0]
    s = np.ascontiguousarray(s, dtype=np.int8)
    nodes = np.zeros((M + 1, N), dtype=np.int8)
    E = np.zeros(M + 1)
    rho = np.zeros(M + 1)
    r, eb, mg = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
    v = lib().mc3o_biased_step(N, M, _ptr(J, ctypes.c_double), scale, alpha, beta, seed, chain, step,
                               _ptr(s, ctypes.c_int8), _ptr(nodes, ctypes.c_int8), _ptr(E, ctypes.c_double),
                               _ptr(rho, ctypes.c_double), ctypes.byref(r), ctypes.byref(eb), ctypes.byref(mg))
    return {"r": r.value, "vstar": int(v), "nodes": nodes, "E": E, "rho": rho, "e_bar": eb.value,
            "margin": mg.value}


def run(J: np.ndarray, scale: float, N: int, M: int, chains: int, kmin: int, kmax: int, seed: int,
        betas, spins: Optional[np.ndarray] = None, step0: int = 0, rule: int = RULE_MCMCMC,
        chain_base: int = 0, want_node_e: bool = False, forced: Optional[np.ndarray] = None,
        arity: Optional[int] = None, law: int = LAW_UNIFORM, table=None, alpha: float = 0.0):
    """Run len(betas) steps.  Returns dict(spins, e_cur, rec[, node_e]).

    Initial spins default to the INIT stream of each chain; energies are recomputed
    from the configurations at every step."""
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    nsteps = len(betas)
    J = np.ascontiguousarray(J, dtype=np.float64)
    if spins is None:
        spins = np.stack([init_spins(seed, N, chain_base + c) for c in range(chains)])
    spins = np.ascontiguousarray(spins, dtype=np.int8).copy()
    e_cur = np.array([energy(J, scale, spins[c]) for c in range(chains)], dtype=np.float64)
    rec = np.zeros((nsteps, chains), dtype=REC_DTYPE)
    node_e = np.zeros((nsteps, chains, M + 1), dtype=np.float64) if want_node_e else None
    f = None
    if forced is not None:
        f = np.ascontiguousarray(forced, dtype=np.int32)
        assert f.shape == (nsteps, chains)
    tab = None
    if law == LAW_TABLE:
        tab = np.ascontiguousarray(table, dtype=np.float64)
        assert tab.shape == (M + 1,)
    cfg = Cfg(N, M, chains, kmin, kmax, rule, chain_base, 0, seed, scale, M if arity is None else arity, law, 0,
              None if tab is None else _ptr(tab, ctypes.c_double), alpha)
    rc = lib().mc3o_run(ctypes.byref(cfg), _ptr(J, ctypes.c_double), _ptr(spins, ctypes.c_int8),
                        _ptr(e_cur, ctypes.c_double), step0, nsteps, _ptr(betas, ctypes.c_double),
                        rec.ctypes.data, None if node_e is None else node_e.ctypes.data,
                        None if f is None else f.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the configuration")
    out = {"spins": spins, "e_cur": e_cur, "rec": rec}
    if node_e is not None:
        out["node_e"] = node_e
    return out


def set_gen_brute(G, X: int) -> float:
    """P_gen(S | X) of the set variant (S = {0..n-1}, X a nonempty bitmask), summed over
    every order of the added elements (at most 10 of them); G[e][p] = P_gen(e | p)."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    n = G.shape[0]
    st = ctypes.c_int32()
    v = lib().mc3o_set_gen_brute(n, _ptr(G, ctypes.c_double), int(X), ctypes.byref(st))
    if st.value != 0:
        raise ValueError("set_gen_brute: empty X, more than 10 additions or n > 30")
    return float(v)
