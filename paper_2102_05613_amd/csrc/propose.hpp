// propose.hpp -- initial spins and the star-graph proposal (flip sets, roots, base words).
#pragma once
#include "common.hpp"

namespace mc3 {

// ------------------------------------------------------------------- init spins

// Spins of every chain from the init stream: word w of the chain's bitset is word w
// of stream (init, chain_base + global chain, step 0, edge 0); bits at and beyond N
// are cleared.  Grid: x over words (up to the largest W), y over global chains.
__global__ void k_init_spins(char* __restrict__ ws, const Inst* __restrict__ insts,
                             const int32_t* __restrict__ chain_inst, int total_chains, Key key, uint32_t chain_base) {
  const int g = blockIdx.y;
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_chains) return;
  const Inst& in = insts[chain_inst[g]];
  if (w >= in.W) return;
  const int c = g - in.chain0;
  uint32_t v = 0;
  if (w * 32 < in.N) {
    uint4 b = stream_block(key, kTagInit, chain_base + (uint32_t)g, 0u, 0u, (uint32_t)w / 4u);
    v = pick(b, (uint32_t)w % 4u);
    int rem = in.N - w * 32;
    if (rem < 32) v &= (1u << rem) - 1u;
  }
  ws_at<uint32_t>(ws, in.spins)[(size_t)c * in.W + w] = v;
}

// ------------------------------------------------------------------- propose

// Root position r of chain gc at `step`: randint(ROOT word 0, M+1), 0 for Metropolis.
__device__ __forceinline__ int root_of(Key key, uint32_t gc, uint32_t step, int M, int metropolis) {
  if (metropolis) return 0;
  uint4 rb = stream_block(key, kTagRoot, gc, step, 0u, 0u);
  return (int)randint(rb.x, (uint32_t)(M + 1));
}

// Flip sets and roots do not depend on the chains' states, so several steps are
// drawn in one launch: grid (proposal blocks, steps), step = step0 + blockIdx.y, its
// results in ring slot step % nslots.  One thread per (chain, edge) of one instance
// (block table): k_e and Floyd's k-of-N draw into the thread's own LDS bitset (row
// stride `stride` >= W words; W+1 where it fits, so the final copy does not collide
// on banks), then every word written to flipsT[w][chain*M + e-1] (consecutive
// threads, consecutive addresses).  Thread (chain, edge 1) stores the chain's root in
// roots_ring[slot][global chain].  With write_base, for the first step only, the
// thread of edge r (edge 1 if r = 0) also writes base = s ^ F_r from the chain's
// current spins.  Dynamic LDS: blockDim.x * stride words.
__global__ void k_propose(char* __restrict__ ws, const Inst* __restrict__ insts, const PBlock* __restrict__ blocks,
                          int32_t* __restrict__ roots_ring, int total_chains, uint32_t nslots, int write_base,
                          int stride, int metropolis, Key key, uint32_t chain_base, uint32_t step0) {
  extern __shared__ uint32_t lds_bits[];
  const int T = blockDim.x;
  const uint32_t step = step0 + blockIdx.y;
  const uint32_t slot = step % nslots;
  const PBlock blk0 = blocks[blockIdx.x];
  const Inst& in = insts[blk0.inst];
  const int N = in.N, M = in.M, W = in.W, Bp = in.Bp;
  const long long total = (long long)in.chains * M;
  for (int i = threadIdx.x; i < T * stride; i += T) lds_bits[i] = 0u;
  __syncthreads();
  const long long g = (long long)blk0.edge0 + threadIdx.x;
  if (g >= total) return;
  const int c = (int)(g / M);
  const uint32_t e = (uint32_t)(g % M) + 1u;
  const uint32_t gc = chain_base + (uint32_t)(in.chain0 + c);
  uint32_t* mine = lds_bits + (size_t)threadIdx.x * stride;
  uint4 blk = stream_block(key, kTagEdge, gc, step, e, 0u);
  const int k = in.kmin + (int)randint(blk.x, (uint32_t)(in.kmax - in.kmin + 1));
  for (int idx = 0; idx < k; ++idx) {
    const uint32_t n = 1u + (uint32_t)idx;
    if ((n & 3u) == 0u) blk = stream_block(key, kTagEdge, gc, step, e, n >> 2);
    const uint32_t j = (uint32_t)(N - k + idx);
    const uint32_t t = randint(pick(blk, n & 3u), j + 1u);
    const uint32_t bt = mine[t >> 5] >> (t & 31u) & 1u;
    const uint32_t pos = bt ? j : t;
    mine[pos >> 5] |= 1u << (pos & 31u);
  }
  const int r = root_of(key, gc, step, M, metropolis);
  if (e == 1u) roots_ring[(size_t)slot * total_chains + in.chain0 + c] = (int32_t)r;
  uint32_t* flipsT = flips_at(ws, in, slot);
  for (int w = 0; w < W; ++w) flipsT[(size_t)w * Bp + g] = mine[w];
  if (write_base && blockIdx.y == 0 && (int)e == (r == 0 ? 1 : r)) {
    uint32_t* base = ws_at<uint32_t>(ws, in.base[step & 1u]);
    const uint32_t* spins = ws_at<const uint32_t>(ws, in.spins);
    for (int w = 0; w < W; ++w) base[(size_t)c * W + w] = spins[(size_t)c * W + w] ^ (r ? mine[w] : 0u);
  }
}

// Bit word w of candidate column `col` (see the layout note at the top).
__device__ __forceinline__ uint32_t column_word(const uint32_t* __restrict__ flipsT, const uint32_t* __restrict__ base,
                                                const int32_t* __restrict__ roots, int M, int W, int Bp, int B,
                                                int col, int w) {
  if (col >= B) return 0u;
  const int c = col / M, m = col - c * M;
  const int r = roots[c];
  const uint32_t b = base[(size_t)c * W + w];
  return (r >= 1 && m == r - 1) ? b : (b ^ flipsT[(size_t)w * Bp + col]);
}

// Materialise the candidate bitsets candT[w][col] (inspection only; the hot path
// scores straight from flipsT and base).  Grid: x over columns, y over words.
__global__ void k_build_candidates(uint32_t* __restrict__ candT, const uint32_t* __restrict__ flipsT,
                                   const uint32_t* __restrict__ base, const int32_t* __restrict__ roots, int chains,
                                   int M, int W, int Bp) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = blockIdx.y;
  if (col >= Bp || w >= W) return;
  candT[(size_t)w * Bp + col] = column_word(flipsT, base, roots, M, W, Bp, chains * M, col, w);
}

}  // namespace mc3
