"""Pins of the oracle's random-number layer: Philox4x32-10, randint, the 53-bit
uniform and Floyd's distinct-subset draw."""
import itertools
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert list(oracle.philox(ctr, key)) == out


_TORCH_PROBE = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t sub = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t off = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::philox_engine e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
  return 0;
}
"""


def test_philox_matches_independent_implementation():
    """PyTorch's ATen Philox4x32-10 header (an implementation written by others from
    the same SC'11 definition) must give identical blocks on random counters/keys."""
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if shutil.which("g++") is None or not os.path.exists(os.path.join(inc, "ATen/core/PhiloxRNGEngine.h")):
        pytest.skip("g++ or the ATen header is missing")
    rng = np.random.Generator(np.random.PCG64(7))
    vals = rng.integers(0, 2 ** 32, size=(200, 6), dtype=np.uint64)
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.cpp")
        exe = os.path.join(d, "p")
        with open(src, "w") as f:
            f.write(_TORCH_PROBE)
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", inc, src, "-o", exe])
        inp = "\n".join(" ".join("%x" % int(x) for x in row) for row in vals)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for row, line in zip(vals, out):
        got = oracle.philox(row[:4], row[4:6])
        assert ["%08x" % int(x) for x in got] == line.split()


def test_word_stream_layout():
    """Word n of a stream is element n%4 of the block at counter (n/4, edge, step,
    tag<<28 | chain) under key (seed lo, seed hi)."""
    seed = 0x0123456789ABCDEF
    for (tag, chain, step, edge, n) in [(1, 0, 0, 0, 0), (3, 17, 99, 5, 13), (4, 2 ** 27 + 3, 2 ** 31, 0, 1)]:
        blk = oracle.philox([n // 4, edge, step, (tag << 28) | (chain & 0x0FFFFFFF)],
                            [seed & 0xFFFFFFFF, seed >> 32])
        assert oracle.word(seed, tag, chain, step, edge, n) == int(blk[n % 4])


def test_randint_closed_form():
    for w in [0, 1, 2 ** 31, 2 ** 32 - 1, 123456789]:
        for n in [1, 2, 3, 7, 1025, 2 ** 31 + 5]:
            assert oracle.randint(w, n) == (w * n) >> 32
            assert 0 <= oracle.randint(w, n) < n


def test_u53_closed_form():
    assert oracle.u53(0xFFFFFFFF, 0xFFFFFFFF) == 2 ** 53 - 1
    assert oracle.u53(0, 0) == 0
    assert oracle.u53(1 << 5, 0) == 1 << 26
    assert oracle.u53(0, 1 << 6) == 1


def _word_for(t, n):
    """Smallest 32-bit word w with floor(w n / 2^32) == t."""
    return -((-t * 2 ** 32) // n)


@pytest.mark.parametrize("N,k", [(1, 1), (4, 2), (5, 3), (6, 1), (6, 6), (7, 3)])
def test_floyd_exhaustive_uniformity(N, k):
    """Drive Floyd with every sequence of exact uniform integers: each k-subset must
    come out exactly k! times (N!/(N-k)! equally likely sequences)."""
    counts = {}
    ranges = [range(N - k + idx + 1) for idx in range(k)]
    for ts in itertools.product(*ranges):
        words = [_word_for(t, N - k + idx + 1) for idx, t in enumerate(ts)]
        m = oracle.floyd_words(N, k, words)
        assert m.sum() == k
        key = tuple(np.nonzero(m)[0])
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == math.comb(N, k)
    assert set(counts.values()) == {math.factorial(k)}


def test_edge_flip_sizes_in_range_and_chi2():
    """k_e = kmin + randint(w0, kmax-kmin+1): sizes spread uniformly over the range."""
    N, kmin, kmax = 64, 3, 10
    sizes = []
    for step in range(400):
        for e in range(1, 6):
            k, m = oracle.edge_flips(11, 0, step, e, N, kmin, kmax)
            assert m.sum() == k and kmin <= k <= kmax
            sizes.append(k)
    hist = np.bincount(sizes, minlength=kmax + 1)[kmin:]
    exp = len(sizes) / (kmax - kmin + 1)
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 30.0  # 7 dof: P(chi2 > 30) < 1e-4


def test_init_spins_are_stream_bits():
    s = oracle.init_spins(5, 70, 3)
    for i in range(70):
        w = oracle.word(5, oracle.TAG_INIT, 3, 0, 0, i // 32)
        assert s[i] == (-1 if (w >> (i % 32)) & 1 else 1)
