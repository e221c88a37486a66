"""Seeded synthetic inputs for the SK MCMCMC hot path.

This module holds no arithmetic of the method: it only draws coupling matrices and
names workloads.  Both the GPU path and the CPU oracle take their couplings from
here, so neither ever reads the other's data.

Couplings follow the SK definition (paper, Sec. "The Sherrington-Kirkpatrick model"):
a dense symmetric matrix of independent zero-mean Gaussian couplings.  The energy
convention used throughout is E(s) = -scale * sum_{i<j} J_ij s_i s_j, which equals the
paper's (1/sqrt(L)) sum J S S in law (the Gaussian law is symmetric, so the sign and
the 1/sqrt(L) factor fold into J ~ N(0, 1/N)).  The paper's own disorder realisation
is not published; seeded draws of the same law stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np


def couplings_gauss(N: int, seed: int) -> Tuple[np.ndarray, float]:
    """J_ij ~ N(0, 1/N) for i<j, symmetric, zero diagonal; energy scale 1.0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((N, N)) * (1.0 / math.sqrt(N))
    J = np.triu(g, 1)
    J = J + J.T
    return np.ascontiguousarray(J, dtype=np.float64), 1.0


def couplings_pm1(N: int, seed: int) -> Tuple[np.ndarray, float]:
    """J_ij = +-1 fair signs for i<j, symmetric, zero diagonal; energy scale 1/sqrt(N).

    Energies are exact integers times the scale, so any summation order gives the
    same value: trajectories can be compared bit for bit."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sg = np.where(rng.integers(0, 2, size=(N, N)) == 1, 1.0, -1.0)
    J = np.triu(sg, 1)
    J = J + J.T
    return np.ascontiguousarray(J, dtype=np.float64), 1.0 / math.sqrt(N)


@dataclass
class Workload:
    """One SK MCMCMC workload: instance shape, proposal law, schedule and precision."""
    name: str
    N: int
    M: int
    chains: int
    kmin: int
    kmax: int
    couplings: str            # "pm1" | "gauss"
    precision: str            # "fp64" | "split_bf16"
    rule: str = "mcmcmc"      # "mcmcmc" | "metropolis"
    beta0: float = 1.0
    beta1: float = 1.0
    steps: int = 1000
    seed: int = 0             # RNG key of the chain streams
    coupling_seed: int = 0

    def couplings_matrix(self) -> Tuple[np.ndarray, float]:
        if self.couplings == "pm1":
            return couplings_pm1(self.N, self.coupling_seed)
        return couplings_gauss(self.N, self.coupling_seed)

    @property
    def candidates_per_step(self) -> int:
        return self.chains * self.M


def workloads() -> List[Workload]:
    """The five SK workloads: small exact (PM1), anneal, headline precision, batching
    (one representative instance; the batch list is drawn separately), large."""
    return [
        Workload("sk_n32_pm1_m4", N=32, M=4, chains=1, kmin=1, kmax=1, couplings="pm1",
                 precision="fp64", beta0=1.0, beta1=1.0, steps=10000, seed=0, coupling_seed=0x5EED0001),
        Workload("sk_n256_anneal_m16", N=256, M=16, chains=64, kmin=1, kmax=4, couplings="gauss",
                 precision="fp64", beta0=0.1, beta1=3.0, steps=100000, seed=2, coupling_seed=0x5EED0002),
        Workload("sk_n1024_m128_split", N=1024, M=128, chains=256, kmin=1, kmax=128, couplings="gauss",
                 precision="split_bf16", beta0=2.0, beta1=2.0, steps=20000, seed=3, coupling_seed=0x5EED0003),
        Workload("sk_batch_rep_n1024_m128", N=1024, M=128, chains=4, kmin=1, kmax=64, couplings="gauss",
                 precision="split_bf16", beta0=1.5, beta1=1.5, steps=5000, seed=4, coupling_seed=0x5EED0004),
        Workload("sk_n8192_m1024_split", N=8192, M=1024, chains=32, kmin=256, kmax=256, couplings="gauss",
                 precision="split_bf16", beta0=0.2, beta1=2.5, steps=20000, seed=5, coupling_seed=0x5EED0005),
    ]


def workload(name: str) -> Workload:
    for w in workloads():
        if w.name == name:
            return w
    raise KeyError(name)


def batch_instances(n_instances: int = 2000, seed: int = 0x5EED0004) -> List[Tuple[int, int, int]]:
    """Instance list of the batching workload: N = 64*U{1..32}, M ~ U{8..256},
    flip sizes up to N/16.  Returns [(N, M, kmax)]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ns = 64 * rng.integers(1, 33, size=n_instances)
    Ms = rng.integers(8, 257, size=n_instances)
    return [(int(n), int(m), int(max(1, n // 16))) for n, m in zip(Ns, Ms)]


BATCH_CHAINS = 4       # chains per instance of the batching workload
BATCH_BETA = 1.5
BATCH_SEED = 0x5EED0004


def batch_descs(n_instances: int = 2000, seed: int = BATCH_SEED, chains: int = BATCH_CHAINS):
    """(N, M, chains, kmin, kmax) per instance of the batching workload: N = 64*U{1..32},
    M ~ U{8..256}, `chains` chains, flip-set sizes U{1..N/16}."""
    return [(N, M, chains, 1, kmax) for N, M, kmax in batch_instances(n_instances, seed)]


def batch_couplings(i: int, N: int, seed: int = BATCH_SEED) -> Tuple[np.ndarray, float]:
    """Gaussian couplings of instance i of the batching workload (its own stream)."""
    return couplings_gauss(N, (seed << 20) + i)


def iter_batch_couplings(descs, seed: int = BATCH_SEED, threads: int = 8):
    """Yield (i, J, scale) for every instance in order; matrices are drawn on a small
    thread pool (numpy's generators release the GIL while filling)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as pool:
        pending = {}
        nxt = 0
        for i in range(len(descs)):
            while nxt < len(descs) and nxt < i + 2 * threads:
                pending[nxt] = pool.submit(batch_couplings, nxt, descs[nxt][0], seed)
                nxt += 1
            J, scale = pending.pop(i).result()
            yield i, J, scale


def beta_schedule(beta0: float, beta1: float, total: int, t0: int, n: int) -> np.ndarray:
    """Linear anneal beta_t = beta0 + (beta1 - beta0) * t / (total - 1), t = t0..t0+n-1."""
    t = np.arange(t0, t0 + n, dtype=np.float64)
    if total <= 1:
        return np.full(n, beta0, dtype=np.float64)
    return beta0 + (beta1 - beta0) * (t / float(total - 1))
