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
// set.  Table law: t = floor(u53 W / 2^53) (u53 from ROOT words 0 and 1, W = Q_M),
// r = min { v : Q_v > t } over the cumulative fixed-point weights Qcum.  0 for
// Metropolis.
__device__ __forceinline__ int root_of(Key key, uint32_t gc, uint32_t step, int M, int metropolis, int law,
                                       const uint64_t* __restrict__ Qcum) {
  if (metropolis) return 0;
  if (law == 0) {
    const uint4 rb = stream_block(key, kTagRoot, gc, step, 0u, 0u);
    return (int)randint(rb.x, (uint32_t)(M + 1));
  }
  if (law == 2) {
    const uint4 rb = stream_block(key, kTagRoot, gc, step, 0u, 0u);
    const unsigned long long u53 = u53_of(rb.x, rb.y), W = Qcum[M];
    const unsigned long long lo = u53 * W, hi = __umul64hi(u53, W);
    const unsigned long long t = (hi << 11) | (lo >> 53);
    int a = 0, b = M;   // the first v with Qcum[v] > t lies in [a, b]
    while (a < b) {
      const int mid = (a + b) >> 1;
      if (Qcum[mid] > t)
        b = mid;
      else
        a = mid + 1;
    }
    return a;
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

// One insertion of Floyd's k-of-N: t = randint(word, j+1), then t if it is not in the
// set yet, else j (never in the set before this insertion).  The words of t and j are
// read together, and the chosen one is written back with its bit set.
__device__ __forceinline__ void floyd_insert(uint32_t* set, uint32_t word, uint32_t j) {
  const uint32_t t = randint(word, j + 1u);
  const uint32_t wt = set[t >> 5], wj = set[j >> 5];
  const bool taken = ((wt >> site_bit(t & 31u)) & 1u) != 0u;
  const uint32_t pos = taken ? j : t;
  set[pos >> 5] = (taken ? wj : wt) | (1u << site_bit(pos & 31u));
}

// Floyd's k-of-N draw of the flip set of edge e into the bitset `set` (all zero on
// entry): k_e = kmin + randint(word 0, kmax-kmin+1), then for idx = 0..k-1 a
// uniform t in [0, N-k+idx] from word idx+1, taking N-k+idx instead when t is already
// in the set.  Words 1..3 are the rest of block 0; block b >= 1 holds words 4b..4b+3.
__device__ __forceinline__ void draw_flip_set(uint32_t* set, Key key, uint32_t gc, uint32_t step, uint32_t e, int N,
                                              int kmin, int kmax) {
  uint4 blk = stream_block(key, kTagEdge, gc, step, e, 0u);
  const int k = kmin + (int)randint(blk.x, (uint32_t)(kmax - kmin + 1));
  const uint32_t j0 = (uint32_t)(N - k);
  floyd_insert(set, blk.y, j0);   // k >= 1
  if (k > 1) floyd_insert(set, blk.z, j0 + 1u);
  if (k > 2) floyd_insert(set, blk.w, j0 + 2u);
  for (int idx = 3; idx < k; idx += 4) {
    blk = stream_block(key, kTagEdge, gc, step, e, (uint32_t)(idx + 1) >> 2);
    floyd_insert(set, blk.x, j0 + (uint32_t)idx);
    if (idx + 1 < k) floyd_insert(set, blk.y, j0 + (uint32_t)idx + 1u);
    if (idx + 2 < k) floyd_insert(set, blk.z, j0 + (uint32_t)idx + 2u);
    if (idx + 3 < k) floyd_insert(set, blk.w, j0 + (uint32_t)idx + 3u);
  }
}

// The flip-set size k_e of edge e (word 0 of its stream).
__device__ __forceinline__ int flip_count(Key key, uint32_t gc, uint32_t step, uint32_t e, int kmin, int kmax) {
  const uint4 blk = stream_block(key, kTagEdge, gc, step, e, 0u);
  return kmin + (int)randint(blk.x, (uint32_t)(kmax - kmin + 1));
}

// Flip sets and roots do not depend on the chains' states, so several steps are
// drawn in one launch: grid (proposal blocks, steps), step = step0 + blockIdx.y, its
// results in ring slot step % nslots.  Each (chain, node v = 1..M) of one instance
// (block table) gets the path set P(v): the XOR of the flip sets of the edges from
// node 0 down to v (edge u joins node u to its parent), each drawn by Floyd into an
// LDS scratch row and folded into an accumulator row (for the star the path is the
// one edge and the two rows are one).  A wave runs as long as its longest draw, so the
// block first orders its paths by their number of insertions (the sum of k_u along
// the path, in 16 buckets of 1/16 of the largest possible sum, kmax times the depth of
// node M; ties in any order): thread i draws the path of rank i into row i.  Then
// thread i writes the path of its own column, (chain, v) = edge0 + i, from the row
// that holds it: every word to flipsT[w][chain*M + v-1]
// (consecutive threads, consecutive addresses).  Rows have stride `stride` >= W
// words (W+1 where it fits, against bank collisions).  The thread of node 1 stores the
// chain's root in roots_ring[slot][global chain].  With write_base, for the first step
// only, the thread of node r (node 1 if r = 0) also writes base = s ^ P(r) from the
// chain's current spins.
// Trees other than the star whose chains fit a block (M <= blockDim.x; the host then
// lays blocks on whole chains) instead draw every edge once: thread v-1 of a chain
// draws F_v into its row, and the path sets follow by pointer jumping, P(v) ^= P(a(v))
// and a(v) <- a(a(v)) starting from a(v) = parent(v), over ceil(log2(depth)) rounds
// between the two row sets (no ordering by size there: each thread draws one set).
// With a step clock (clk non-null, replayed graphs) the steps start at *clk + step0.
// Dynamic LDS: rows * blockDim.x * stride words.
__global__ void k_propose(char* __restrict__ ws, const Inst* __restrict__ insts, const PBlock* __restrict__ blocks,
                          int32_t* __restrict__ roots_ring, int total_chains, uint32_t nslots, int write_base,
                          int stride, int rows, int metropolis, Key key, uint32_t chain_base, uint32_t step0,
                          const uint32_t* __restrict__ clk) {
  extern __shared__ uint32_t lds_bits[];
  __shared__ int bucket_n[16], bucket_at[16];
  __shared__ int order[256];
  __shared__ int anc_row[256];
  const int T = blockDim.x, tid = threadIdx.x;
  const uint32_t step = (clk ? *clk : 0u) + step0 + blockIdx.y;
  const uint32_t slot = step % nslots;
  const PBlock blk0 = blocks[blockIdx.x];
  const Inst& in = insts[blk0.inst];
  const int N = in.N, M = in.M, W = in.W, Bp = in.Bp;
  const long long total = (long long)in.chains * M;
  const bool star = in.arity >= M;
  for (int i = tid; i < rows * T * stride; i += T) lds_bits[i] = 0u;
  if (tid < 16) bucket_n[tid] = 0;
  __syncthreads();
  const long long g = (long long)blk0.edge0 + tid;
  const bool real = tid < blk0.count && g < total;
  if (!star && M <= T) {
    // each edge once, then path sets by pointer jumping within the chain
    const int c = real ? (int)(g / M) : 0;
    const uint32_t e = real ? (uint32_t)(g % M) + 1u : 0u;
    const uint32_t gc = chain_base + (uint32_t)(in.chain0 + c);
    const int row0 = tid - (int)e + 1;   // row of node 1 of this chain
    if (real) draw_flip_set(lds_bits + (size_t)tid * stride, key, gc, step, e, N, in.kmin, in.kmax);
    int a = real ? (int)((e - 1u) / (uint32_t)in.arity) : 0;   // ancestor node, 0 = node 0
    int depth = 0;
    for (uint32_t u = (uint32_t)M; u >= 1u; u = (u - 1u) / (uint32_t)in.arity) ++depth;
    int rounds = 0;
    while ((1 << rounds) < depth) ++rounds;
    anc_row[tid] = a;
    __syncthreads();
    uint32_t* src = lds_bits;
    uint32_t* dst = lds_bits + (size_t)T * stride;
    for (int rd = 0; rd < rounds; ++rd) {
      int a_next = 0;
      if (real) {
        const uint32_t* me = src + (size_t)tid * stride;
        uint32_t* out = dst + (size_t)tid * stride;
        if (a >= 1) {
          const int ra = row0 + a - 1;
          const uint32_t* up = src + (size_t)ra * stride;
          for (int w = 0; w < W; ++w) out[w] = me[w] ^ up[w];
          a_next = anc_row[ra];
        } else {
          for (int w = 0; w < W; ++w) out[w] = me[w];
        }
      }
      __syncthreads();
      a = a_next;
      anc_row[tid] = a;
      uint32_t* t = src;
      src = dst;
      dst = t;
      __syncthreads();
    }
    if (!real) return;
    const uint32_t* path = src + (size_t)tid * stride;
    const int r = root_of(key, gc, step, M, metropolis, in.law,
                          in.root_q ? ws_at<const uint64_t>(ws, in.root_q) : nullptr);
    if (e == 1u) roots_ring[(size_t)slot * total_chains + in.chain0 + c] = (int32_t)r;
    uint32_t* flipsT = flips_at(ws, in, slot);
    for (int w = 0; w < W; ++w) flipsT[(size_t)w * Bp + g] = path[w];
    if (write_base && blockIdx.y == 0 && (int)e == (r == 0 ? 1 : r)) {
      uint32_t* base = ws_at<uint32_t>(ws, in.base[step & 1u]);
      const uint32_t* spins = ws_at<const uint32_t>(ws, in.spins);
      for (int w = 0; w < W; ++w) base[(size_t)c * W + w] = spins[(size_t)c * W + w] ^ (r ? path[w] : 0u);
    }
    return;
  }
  // 1. rank of this thread's own path by its number of insertions
  const int c = real ? (int)(g / M) : 0;
  const uint32_t e = real ? (uint32_t)(g % M) + 1u : 0u;
  const uint32_t gc = chain_base + (uint32_t)(in.chain0 + c);
  int work = 0;
  if (real)
    for (uint32_t u = e; u >= 1u; u = star ? 0u : (u - 1u) / (uint32_t)in.arity)
      work += flip_count(key, gc, step, u, in.kmin, in.kmax);
  int depth = 1;   // edges on the longest path from node 0 (that of node M)
  if (!star) {
    depth = 0;
    for (uint32_t u = (uint32_t)M; u >= 1u; u = (u - 1u) / (uint32_t)in.arity) ++depth;
  }
  const int bucket = min(15, (int)(((long long)work * 16) / ((long long)in.kmax * depth + 1)));
  const int within = atomicAdd(&bucket_n[bucket], 1);
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int b = 0; b < 16; ++b) {
      bucket_at[b] = acc;
      acc += bucket_n[b];
    }
  }
  __syncthreads();
  const int rank = bucket_at[bucket] + within;
  order[rank] = tid;
  __syncthreads();
  // 2. draw the path of rank tid into row tid
  {
    const long long gd = (long long)blk0.edge0 + order[tid];
    if (gd < total) {
      const int cd = (int)(gd / M);
      const uint32_t ed = (uint32_t)(gd % M) + 1u;
      const uint32_t gcd = chain_base + (uint32_t)(in.chain0 + cd);
      uint32_t* mine = lds_bits + (size_t)tid * stride;
      if (star) {
        draw_flip_set(mine, key, gcd, step, ed, N, in.kmin, in.kmax);
      } else {
        uint32_t* tmp = lds_bits + (size_t)(T + tid) * stride;
        for (uint32_t u = ed; u >= 1u; u = (u - 1u) / (uint32_t)in.arity) {
          draw_flip_set(tmp, key, gcd, step, u, N, in.kmin, in.kmax);
          for (int w = 0; w < W; ++w) {
            mine[w] ^= tmp[w];
            tmp[w] = 0u;
          }
        }
      }
    }
  }
  __syncthreads();
  // 3. this thread's own column, from row `rank`
  if (!real) return;
  const uint32_t* path = lds_bits + (size_t)rank * stride;
  const int r = root_of(key, gc, step, M, metropolis, in.law,
                        in.root_q ? ws_at<const uint64_t>(ws, in.root_q) : nullptr);
  if (e == 1u) roots_ring[(size_t)slot * total_chains + in.chain0 + c] = (int32_t)r;
  uint32_t* flipsT = flips_at(ws, in, slot);
  for (int w = 0; w < W; ++w) flipsT[(size_t)w * Bp + g] = path[w];
  if (write_base && blockIdx.y == 0 && (int)e == (r == 0 ? 1 : r)) {
    uint32_t* base = ws_at<uint32_t>(ws, in.base[step & 1u]);
    const uint32_t* spins = ws_at<const uint32_t>(ws, in.spins);
    for (int w = 0; w < W; ++w) base[(size_t)c * W + w] = spins[(size_t)c * W + w] ^ (r ? path[w] : 0u);
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
