// propose.hpp -- initial spins and the star-graph proposal (flip sets, roots, base words).
#pragma once
#include "common.hpp"

namespace mc3 {

// ------------------------------------------------------------------- init spins

// Spins of every chain from the init stream: site 32w + k is bit k of word w of
// stream (init, chain_base + global chain, step 0, edge 0), stored at bit site_bit(k);
// sites at and beyond N are cleared.  Grid: x over words (up to the largest W), y over global chains.
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
    v = stored_word(v);
  }
  ws_at<uint32_t>(ws, in.spins)[(size_t)c * in.W + w] = v;
}

// ------------------------------------------------------------------- propose

// Root position r of chain gc at `step` (the node the current state sits at).
// Uniform law: randint(ROOT word 0, M+1).  Line law: the number of the M additions
// that went to the left end, addition j going left iff bit j%32 of ROOT word j/32 is
// set.  0 for Metropolis.
__device__ __forceinline__ int root_of(Key key, uint32_t gc, uint32_t step, int M, int metropolis, int law) {
  if (metropolis) return 0;
  if (law == 0) {
    const uint4 rb = stream_block(key, kTagRoot, gc, step, 0u, 0u);
    return (int)randint(rb.x, (uint32_t)(M + 1));
  }
  int k = 0;
  for (int j0 = 0; j0 < M; j0 += 128) {
    const uint4 rb = stream_block(key, kTagRoot, gc, step, 0u, (uint32_t)(j0 >> 7));
    for (int q = 0; q < 4 && j0 + 32 * q < M; ++q) {
      const int nb = M - (j0 + 32 * q);
      const uint32_t word = pick(rb, (uint32_t)q);
      k += __popc(nb >= 32 ? word : (word & ((1u << nb) - 1u)));
    }
  }
  return k;
}

// Floyd's k-of-N draw of the flip set of edge e into the bitset `set` (all zero on
// entry): k_e = kmin + randint(word 0, kmax-kmin+1), then for idx = 0..k-1 a
// uniform t in [0, N-k+idx], taking N-k+idx instead when t is already in the set.
__device__ __forceinline__ void draw_flip_set(uint32_t* set, Key key, uint32_t gc, uint32_t step, uint32_t e, int N,
                                              int kmin, int kmax) {
  uint4 blk = stream_block(key, kTagEdge, gc, step, e, 0u);
  const int k = kmin + (int)randint(blk.x, (uint32_t)(kmax - kmin + 1));
  for (int idx = 0; idx < k; ++idx) {
    const uint32_t n = 1u + (uint32_t)idx;
    if ((n & 3u) == 0u) blk = stream_block(key, kTagEdge, gc, step, e, n >> 2);
    const uint32_t j = (uint32_t)(N - k + idx);
    const uint32_t t = randint(pick(blk, n & 3u), j + 1u);
    const uint32_t bt = set[t >> 5] >> site_bit(t & 31u) & 1u;
    const uint32_t pos = bt ? j : t;
    set[pos >> 5] |= 1u << site_bit(pos & 31u);
  }
}

// Flip sets and roots do not depend on the chains' states, so several steps are
// drawn in one launch: grid (proposal blocks, steps), step = step0 + blockIdx.y, its
// results in ring slot step % nslots.  One thread per (chain, node v = 1..M) of one
// instance (block table) forms the path set P(v): the XOR of the flip sets of the
// edges from node 0 down to v (edge u joins node u to its parent), each drawn by
// Floyd into the thread's LDS scratch row and folded into its accumulator row (for
// the star the path is the one edge and the two rows are one).  Rows have stride
// `stride` >= W words (W+1 where it fits, so the final copy does not collide on
// banks); every word goes to flipsT[w][chain*M + v-1] (consecutive threads,
// consecutive addresses).  Thread (chain, node 1) stores the chain's root in
// roots_ring[slot][global chain].  With write_base, for the first step only, the
// thread of node r (node 1 if r = 0) also writes base = s ^ P(r) from the chain's
// current spins.  Dynamic LDS: rows * blockDim.x * stride words.
__global__ void k_propose(char* __restrict__ ws, const Inst* __restrict__ insts, const PBlock* __restrict__ blocks,
                          int32_t* __restrict__ roots_ring, int total_chains, uint32_t nslots, int write_base,
                          int stride, int rows, int metropolis, Key key, uint32_t chain_base, uint32_t step0) {
  extern __shared__ uint32_t lds_bits[];
  const int T = blockDim.x;
  const uint32_t step = step0 + blockIdx.y;
  const uint32_t slot = step % nslots;
  const PBlock blk0 = blocks[blockIdx.x];
  const Inst& in = insts[blk0.inst];
  const int N = in.N, M = in.M, W = in.W, Bp = in.Bp;
  const long long total = (long long)in.chains * M;
  for (int i = threadIdx.x; i < rows * T * stride; i += T) lds_bits[i] = 0u;
  __syncthreads();
  const long long g = (long long)blk0.edge0 + threadIdx.x;
  if (g >= total) return;
  const int c = (int)(g / M);
  const uint32_t e = (uint32_t)(g % M) + 1u;
  const uint32_t gc = chain_base + (uint32_t)(in.chain0 + c);
  uint32_t* mine = lds_bits + (size_t)threadIdx.x * stride;
  if (in.arity >= M) {
    draw_flip_set(mine, key, gc, step, e, N, in.kmin, in.kmax);
  } else {
    uint32_t* tmp = lds_bits + (size_t)(T + threadIdx.x) * stride;
    for (uint32_t u = e; u >= 1u; u = (u - 1u) / (uint32_t)in.arity) {
      draw_flip_set(tmp, key, gc, step, u, N, in.kmin, in.kmax);
      for (int w = 0; w < W; ++w) {
        mine[w] ^= tmp[w];
        tmp[w] = 0u;
      }
    }
  }
  const int r = root_of(key, gc, step, M, metropolis, in.law);
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
