// kernels.hpp -- device kernels of the SK MCMCMC hot path (gfx950).
//
// Data layout in HBM (all sizes padded: Np = N rounded up to 128, W = Np/32 words
// per spin bitset, B = chains*M candidate columns, Bp = B rounded up to 512):
//   J64     [Np][Np] double, row-major, zero outside the N x N block.
//   Jsplit  bf16 hi/mid/lo of the strict upper triangle of J, in matrix-core
//           fragment order: fragment (R, S, t) = rows 32R..32R+31, k = 16S..16S+15,
//           term t, stored as 64 lanes x 8 bf16 (lane l holds row 32R + l%32,
//           k = 16S + 8(l/32) + e for e = 0..7); 1 KiB per fragment.
//   spins   [chains][W] uint32 bitsets (set bit = spin -1).
//   flipsT  ring of slots, one step each, slot = step % slots; a slot is [W][Bp]
//           uint32: word w of the flip set F_{m+1} of edge m+1 of chain c at column
//           c*M + m (columns contiguous, so a matrix-core B fragment's 32 columns are
//           one 128-byte line); padding columns stay zero.
//   base    two [chains+1][W] uint32 buffers by step parity: s ^ F_r (s if r = 0)
//           per chain; row `chains` is zero (used by padding columns).
//   partial [P][Bp] double: energy contributions of row-block pair p.
//
// Candidate columns are never materialised on the hot path.  Column m of chain c is
// node m+1 of the star, except that when the root r >= 1 column r-1 holds the hub
// (node 0) instead of leaf r (the current state).  Its bitset is therefore
// base_c ^ F_{m+1}, or base_c alone for column r-1:
//   r = 0:  base = s, column m = s ^ F_{m+1} = leaf m+1;
//   r >= 1: base = s ^ F_r = hub, column m = hub ^ F_{m+1} = leaf m+1, column r-1 = hub.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_rng.hpp"

namespace mc3 {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRowBlock = 128;  // rows of J per scoring work unit (4 fragments of 32)

// One SK instance of a batch, as the kernels see it.  Byte offsets are into the
// workspace; the per-chain arrays (energies, roots, counters, records) are global over
// the batch and indexed by chain0 + c.
struct Inst {
  int32_t N, Np, W, M;
  int32_t chains, kmin, kmax, B;
  int32_t Bp, NB, P, chain0;
  double scale;
  uint64_t J64, Jpack, flips, flip_slot, base[2], partial, spins;
};

// Flip sets of the step held in ring slot `slot` (slots of flip_slot bytes each).
__device__ __forceinline__ uint32_t* flips_at(char* ws, const Inst& in, uint32_t slot) {
  return reinterpret_cast<uint32_t*>(ws + in.flips + (uint64_t)slot * in.flip_slot);
}

// A scoring work unit (row-block pair p, column tile ct of instance inst); inst < 0 is
// an idle slot of the launch grid.
struct Unit {
  int32_t inst, p, ct, pad;
};

// A proposal block: edges edge0 .. edge0 + blockDim.x - 1 (flattened chain*M + e-1) of
// instance inst.
struct PBlock {
  int32_t inst, edge0;
};

template <class T>
__device__ __forceinline__ T* ws_at(char* ws, uint64_t off) {
  return reinterpret_cast<T*>(ws + off);
}

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

// ------------------------------------------------------------------- split J

// Round a double to 8 significant bits (bfloat16 precision), ties to even, and
// return the bfloat16 bit pattern.  Inputs are finite and far from the bfloat16
// overflow/underflow limits (|J| < 2^100 and residuals > 2^-100 or exactly 0).
__device__ __forceinline__ uint16_t bf16_rne_of_double(double x, double* rounded) {
  unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned long long lsb = (b >> 45) & 1ull;
  b += 0x00000FFFFFFFFFFFull + lsb;
  b &= ~0x00001FFFFFFFFFFFull;
  double y = __longlong_as_double((long long)b);
  *rounded = y;
  float f = (float)y;  // exact: y has 8 significant bits
  return (uint16_t)(__float_as_uint(f) >> 16);
}

// Pack hi/mid/lo of the strict upper triangle of J64 into fragment order.
// One thread per (fragment R, S, term t, lane): 8 bf16 = 16 bytes.
__global__ void k_pack_split(uint4* __restrict__ Apack, const double* __restrict__ J64, int Np) {
  const long long KS = Np / 16;
  const long long nfrag_lanes = (long long)(Np / 32) * KS * 64;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nfrag_lanes) return;
  const int lane = (int)(gid % 64);
  const long long rs = gid / 64;
  const int S = (int)(rs % KS);
  const int R = (int)(rs / KS);
  const int i = 32 * R + lane % 32;
  const int k0 = 16 * S + 8 * (lane / 32);
  uint16_t h[8], m[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = k0 + e;
    const double x = (k > i) ? J64[(size_t)i * Np + k] : 0.0;
    double xh, xm, xl;
    h[e] = bf16_rne_of_double(x, &xh);
    const double r1 = x - xh;
    m[e] = bf16_rne_of_double(r1, &xm);
    const double r2 = r1 - xm;
    l[e] = bf16_rne_of_double(r2, &xl);
  }
  uint4 vh, vm, vl;
  vh.x = h[0] | ((uint32_t)h[1] << 16); vh.y = h[2] | ((uint32_t)h[3] << 16);
  vh.z = h[4] | ((uint32_t)h[5] << 16); vh.w = h[6] | ((uint32_t)h[7] << 16);
  vm.x = m[0] | ((uint32_t)m[1] << 16); vm.y = m[2] | ((uint32_t)m[3] << 16);
  vm.z = m[4] | ((uint32_t)m[5] << 16); vm.w = m[6] | ((uint32_t)m[7] << 16);
  vl.x = l[0] | ((uint32_t)l[1] << 16); vl.y = l[2] | ((uint32_t)l[3] << 16);
  vl.z = l[4] | ((uint32_t)l[5] << 16); vl.w = l[6] | ((uint32_t)l[7] << 16);
  const size_t base = ((size_t)R * KS + S) * 3;
  Apack[(base + 0) * 64 + lane] = vh;
  Apack[(base + 1) * 64 + lane] = vm;
  Apack[(base + 2) * 64 + lane] = vl;
}

// ------------------------------------------------------------------- split scoring

// Expand 8 spin bits (set = -1) into 8 bfloat16 values +-1 (0x3F80 | bit << 15):
// register p holds elements 2p (low half) and 2p+1 (high half).
__device__ __forceinline__ bf16x8 spins_to_bf16(uint32_t byte) {
  union { uint32_t u[4]; bf16x8 v; } r;
#pragma unroll
  for (int p = 0; p < 4; ++p)
    r.u[p] = ((byte << (30 - 2 * p)) & 0x80000000u) | ((byte << (15 - 2 * p)) & 0x00008000u) | 0x3F803F80u;
  return r.v;
}

// Asynchronous copy of 16 bytes per lane from global memory straight into LDS:
// lane l's bytes land at lds_base + 16 l (lds_base must be wave-uniform).
__device__ __forceinline__ void lds_dma16(const uint4* gsrc, uint4* lds_base) {
  __builtin_amdgcn_global_load_lds((const void*)gsrc,
                                   (__attribute__((address_space(3))) void*)lds_base, 16, 0, 0);
}

// Asynchronous copy of 4 bytes per lane from global memory straight into LDS:
// lane l's word lands at lds_base + 4 l.
__device__ __forceinline__ void lds_dma4(const uint32_t* gsrc, uint32_t* lds_base) {
  __builtin_amdgcn_global_load_lds((const void*)gsrc,
                                   (__attribute__((address_space(3))) void*)lds_base, 4, 0, 0);
}

// LDS stage of the split scoring loop: six A fragments per wave (its row fragment)
// and, per column of the tile, the flip-set word and the chain's base word.
template <int CF>
struct SplitStage {
  uint4 a[4][6][64];
  uint32_t flip[4 * 32 * CF];
  uint32_t base[4 * 32 * CF];
};

// One 32-k chunk of the split scoring loop: DMA of the next chunk (A fragments, flip
// words, base words) into `nxt`, then 2 k-steps x 12 A fragments x CF columns of
// MFMAs from `cur`.  Two distinct LDS stages alternate, so the compiler can see that
// reading one never waits for the copy into the other; nothing loaded from global
// memory is carried in registers across chunks.  RF_LAST: row fragments rf > RF_LAST
// of this chunk lie entirely below the diagonal (every k <= i), so their fragments
// are zero and are neither read nor multiplied.  rootmask bit cf: this lane's column
// of fragment cf is its chain's root column (bits = base only).
template <int CF, int RF_LAST = 3>
__device__ __forceinline__ void split_chunk(f32x16 (&acc)[4][CF], const SplitStage<CF>& cur, SplitStage<CF>& nxt,
                                            const uint4* next_a, const uint32_t* next_flip,
                                            const uint32_t* const (&next_base)[CF / 2], uint32_t rootmask, int lane,
                                            int wave) {
#pragma unroll
  for (int f = 0; f < 6; ++f) lds_dma16(next_a + f * 64, &nxt.a[wave][f][0]);
#pragma unroll
  for (int q = 0; q < CF / 2; ++q) {
    lds_dma4(next_flip + 64 * q, &nxt.flip[wave * 32 * CF + 64 * q]);
    lds_dma4(next_base[q], &nxt.base[wave * 32 * CF + 64 * q]);
  }
  __builtin_amdgcn_sched_barrier(0);
  uint32_t w[CF];
#pragma unroll
  for (int cf = 0; cf < CF; ++cf) {
    const int j = wave * 32 * CF + cf * 32 + (lane & 31);
    w[cf] = cur.base[j] ^ (((rootmask >> cf) & 1u) ? 0u : cur.flip[j]);
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    bf16x8 b[CF];
#pragma unroll
    for (int cf = 0; cf < CF; ++cf) b[cf] = spins_to_bf16((w[cf] >> (16 * s + 8 * (lane >> 5))) & 0xFFu);
    bf16x8 a[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      if (i % 4 > RF_LAST) continue;
      union { uint4 q; bf16x8 v; } x;
      x.q = cur.a[i % 4][s * 3 + i / 4][lane];
      a[i] = x.v;
    }
    // consecutive instructions update different accumulators
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      if (i % 4 > RF_LAST) continue;
#pragma unroll
      for (int cf = 0; cf < CF; ++cf)
        acc[i % 4][cf] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[cf], acc[i % 4][cf], 0, 0, 0);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// Energies of candidate columns on the BF16 matrix cores.
//
// E(c) = -scale * sum_i c_i h_i with h_i = sum_{j>i} J_ij c_j (strict upper triangle),
// J = hi + mid + lo.  A work unit is (row-block pair p, column tile): row blocks p and
// NB-1-p (128 rows each; their K ranges start at the block's first row, so the pair
// costs NB+1 blocks of K whatever p is).  Four waves share the A tiles through LDS,
// filled by direct global->LDS copies one 32-k chunk ahead (double-buffered); each
// wave owns 32*CF columns whose flip-set and base words come through LDS the same way
// and are combined and expanded to +-1 in registers.  The epilogue multiplies h by
// the column's spins and sums over rows in FP64; the unit writes one FP64 value per
// column.  Each block takes its unit from a table built by the host (the order of
// the table decides which XCD runs which unit).
template <int CF>
__global__ __launch_bounds__(256, (CF == 2 ? 2 : 1)) void k_score_split(
    char* __restrict__ ws, const Inst* __restrict__ insts, const Unit* __restrict__ units,
    const int32_t* __restrict__ roots_all, uint32_t slot, uint32_t parity) {
  static_assert(CF % 2 == 0, "CF must be even (64-column copies)");
  constexpr int TN = 4 * 32 * CF;
  __shared__ SplitStage<CF> st0;
  __shared__ SplitStage<CF> st1;
  const Unit un = units[blockIdx.x];
  if (un.inst < 0) return;
  const Inst& in = insts[un.inst];
  const uint4* __restrict__ Apack = ws_at<const uint4>(ws, in.Jpack);
  const uint32_t* __restrict__ flipsT = flips_at(ws, in, slot);
  const uint32_t* __restrict__ base = ws_at<const uint32_t>(ws, in.base[parity]);
  const int32_t* __restrict__ roots = roots_all + in.chain0;
  double* __restrict__ partial = ws_at<double>(ws, in.partial);
  const int chains = in.chains, M = in.M, Np = in.Np, Bp = in.Bp, NB = in.NB;
  const int p = un.p, ct = un.ct;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col_w = ct * TN + wave * 32 * CF;   // first column of this wave
  const int KS = Np / 16;
  const int W = Np / 32;
  const int B = chains * M;

  // per-lane column data: base rows of the copied columns, root-column mask
  const uint32_t* brow[CF / 2];
#pragma unroll
  for (int q = 0; q < CF / 2; ++q) {
    const int col = col_w + 64 * q + lane;
    brow[q] = base + (size_t)(col < B ? col / M : chains) * W;
  }
  uint32_t rootmask = 0u;
#pragma unroll
  for (int cf = 0; cf < CF; ++cf) {
    const int col = col_w + cf * 32 + (lane & 31);
    if (col < B) {
      const int c = col / M, r = roots[c];
      if (r >= 1 && col - c * M == r - 1) rootmask |= 1u << cf;
    }
  }

  double part[CF];
#pragma unroll
  for (int cf = 0; cf < CF; ++cf) part[cf] = 0.0;

  const int nblk = (p == NB - 1 - p) ? 1 : 2;
  for (int bi = 0; bi < nblk; ++bi) {
    const int I = bi == 0 ? p : NB - 1 - p;
    const int k0 = I * kRowBlock;
    const int kw0 = k0 >> 5;
    const int nchunk = (Np - k0) / 32;   // a multiple of 4
    f32x16 acc[4][CF];
#pragma unroll
    for (int rf = 0; rf < 4; ++rf)
#pragma unroll
      for (int cf = 0; cf < CF; ++cf)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[rf][cf][e] = 0.0f;

    // this wave copies fragment row R = 4I + wave (six fragments per chunk) and the
    // flip/base words of its own columns
    const uint4* src = Apack + (((size_t)(4 * I + wave) * KS + (k0 / 16)) * 3) * 64 + lane;
    const uint32_t* fsrc = flipsT + (size_t)kw0 * Bp + col_w + lane;
    const uint32_t* bsrc[CF / 2];
#pragma unroll
    for (int q = 0; q < CF / 2; ++q) bsrc[q] = brow[q] + kw0;
#pragma unroll
    for (int f = 0; f < 6; ++f) lds_dma16(src + f * 64, &st0.a[wave][f][0]);
#pragma unroll
    for (int q = 0; q < CF / 2; ++q) {
      lds_dma4(fsrc + 64 * q, &st0.flip[wave * 32 * CF + 64 * q]);
      lds_dma4(bsrc[q], &st0.base[wave * 32 * CF + 64 * q]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // chunk c of this row block: A at src + 6*64 c, flip words at fsrc + Bp c, base
    // words at bsrc + c.  The first four chunks cover the diagonal block: chunk c needs
    // row fragments 0..c (nchunk is a multiple of 4; past the end a copy re-reads the
    // last chunk, which is in bounds and not read again before the next row block
    // refills the stage after a barrier).
#define MC3_NEXT(cn)                                                                 \
  const uint32_t* nb##cn[CF / 2];                                                    \
  _Pragma("unroll") for (int q = 0; q < CF / 2; ++q) nb##cn[q] = bsrc[q] + (cn);
    {
      const int c1 = 1, c2 = 2;
      const int c3 = 3 < nchunk - 1 ? 3 : nchunk - 1;
      const int c4 = 4 < nchunk - 1 ? 4 : nchunk - 1;
      MC3_NEXT(c1)
      split_chunk<CF, 0>(acc, st0, st1, src + (size_t)c1 * 6 * 64, fsrc + (size_t)c1 * Bp, nbc1, rootmask, lane, wave);
      MC3_NEXT(c2)
      split_chunk<CF, 1>(acc, st1, st0, src + (size_t)c2 * 6 * 64, fsrc + (size_t)c2 * Bp, nbc2, rootmask, lane, wave);
      MC3_NEXT(c3)
      split_chunk<CF, 2>(acc, st0, st1, src + (size_t)c3 * 6 * 64, fsrc + (size_t)c3 * Bp, nbc3, rootmask, lane, wave);
      MC3_NEXT(c4)
      split_chunk<CF, 3>(acc, st1, st0, src + (size_t)c4 * 6 * 64, fsrc + (size_t)c4 * Bp, nbc4, rootmask, lane, wave);
    }
    for (int c = 4; c < nchunk; c += 2) {
      const int ca = c + 1;
      const int cb = (c + 2 < nchunk) ? c + 2 : nchunk - 1;
      MC3_NEXT(ca)
      split_chunk<CF>(acc, st0, st1, src + (size_t)ca * 6 * 64, fsrc + (size_t)ca * Bp, nbca, rootmask, lane, wave);
      MC3_NEXT(cb)
      split_chunk<CF>(acc, st1, st0, src + (size_t)cb * 6 * 64, fsrc + (size_t)cb * Bp, nbcb, rootmask, lane, wave);
    }
#undef MC3_NEXT
    // epilogue: rows I*128 + 32 rf + 8(e/4) + 4(lane/32) + e%4 of column col_w + 32 cf + lane%32
#pragma unroll
    for (int rf = 0; rf < 4; ++rf) {
#pragma unroll
      for (int cf = 0; cf < CF; ++cf) {
        const int col = col_w + cf * 32 + (lane & 31);
        const int rw = 4 * I + rf;
        const uint32_t bw = col < B ? base[(size_t)(col / M) * W + rw] : 0u;
        const uint32_t rb = ((rootmask >> cf) & 1u) ? bw : (bw ^ flipsT[(size_t)rw * Bp + col]);
        double sum = 0.0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int bit = 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
          const float h = __uint_as_float(__float_as_uint(acc[rf][cf][e]) ^ (((rb >> bit) & 1u) << 31));
          sum += (double)h;
        }
        part[cf] += sum;
      }
    }
  }
#pragma unroll
  for (int cf = 0; cf < CF; ++cf) {
    const double other = __shfl_xor(part[cf], 32);
    const double tot = part[cf] + other;
    if (lane < 32) partial[(size_t)p * Bp + col_w + cf * 32 + lane] = tot;
  }
}

// ------------------------------------------------------------------- FP64 scoring

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Pack the strict upper triangle of J64 for the FP64 matrix cores: fragment
// (R, S) = rows 16R..16R+15, k = 4S..4S+3, lane l holds J[16R + l%16][4S + l/16].
__global__ void k_pack_f64(double* __restrict__ Apack, const double* __restrict__ J64, int Np) {
  const long long KS = Np / 4;
  const long long n = (long long)(Np / 16) * KS * 64;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n) return;
  const int lane = (int)(gid % 64);
  const long long rs = gid / 64;
  const int S = (int)(rs % KS);
  const int R = (int)(rs / KS);
  const int i = 16 * R + lane % 16;
  const int k = 4 * S + lane / 16;
  Apack[gid] = (k > i) ? J64[(size_t)i * Np + k] : 0.0;
}

// LDS stage of the FP64 scoring loop (one 32-k chunk): 8 row fragments x 8 k-steps
// of A (64 doubles each) and the flip/base words of the 128 columns of the tile.
struct F64Stage {
  double a[8][8][64];
  uint32_t flip[128];
  uint32_t base[128];
};

// Copies of chunk `cn` into `st` by wave `wave`: row fragments 2*wave, 2*wave+1 (each
// 8 k-step fragments = 4 KiB contiguous, four 1-KiB copies), and one 64-word slice of
// the flip (waves 0, 1) or base (waves 2, 3) words.  Nine vector-memory operations.
__device__ __forceinline__ void f64_copy(F64Stage& st, const double* a_blk, int KS, const uint32_t* fsrc,
                                         const uint32_t* bsrc, int cn, int Bp, int lane, int wave) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int rf = 2 * wave + h;
    const double* src = a_blk + ((size_t)rf * KS + (size_t)cn * 8) * 64 + 2 * lane;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      lds_dma16(reinterpret_cast<const uint4*>(src + q * 128), reinterpret_cast<uint4*>(&st.a[rf][2 * q][0]));
  }
  if (wave < 2) lds_dma4(fsrc + (size_t)cn * Bp + 64 * wave, &st.flip[64 * wave]);
  else lds_dma4(bsrc + cn, &st.base[64 * (wave - 2)]);
}

// MFMAs of one chunk: 8 k-steps x 4 row fragments x 4 column fragments of 16x16x4.
__device__ __forceinline__ void f64_mfma(f64x4 (&acc)[4][4], const F64Stage& st, uint32_t rootmask, int lane,
                                         int wr, int wc) {
  uint32_t w[4];
#pragma unroll
  for (int cf = 0; cf < 4; ++cf) {
    const int j = wc * 64 + cf * 16 + (lane & 15);
    w[cf] = st.base[j] ^ (((rootmask >> cf) & 1u) ? 0u : st.flip[j]);
  }
  const double one = 1.0;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    double b[4];
#pragma unroll
    for (int cf = 0; cf < 4; ++cf) {
      const uint32_t bit = (w[cf] >> (4 * s + (lane >> 4))) & 1u;
      b[cf] = __longlong_as_double(__double_as_longlong(one) | ((long long)bit << 63));
    }
#pragma unroll
    for (int rf = 0; rf < 4; ++rf) {
      const double a = st.a[wr * 4 + rf][s][lane];
#pragma unroll
      for (int cf = 0; cf < 4; ++cf)
        acc[rf][cf] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[cf], acc[rf][cf], 0, 0, 0);
    }
  }
}

// Energies of candidate columns on the FP64 matrix cores (16x16x4).  Same work units
// as the split kernel (row-block pair of 128 rows x 128-column tile); the four waves
// form a 2 x 2 grid of 64 x 64 tiles; A (J) and the columns' flip/base words are
// staged through LDS by direct global->LDS copies one 32-k chunk ahead (two stages).
// Output layout of the 16x16x4 f64 instruction: C[i][j] is element i/4 of lane
// j + 16 (i % 4).
__global__ __launch_bounds__(256, 2) void k_score_f64(char* __restrict__ ws, const Inst* __restrict__ insts,
                                                      const Unit* __restrict__ units,
                                                      const int32_t* __restrict__ roots_all, uint32_t slot,
                                                      uint32_t parity) {
  constexpr int TN = 128;
  __shared__ F64Stage fs0, fs1;
  const Unit un = units[blockIdx.x];
  if (un.inst < 0) return;
  const Inst& in = insts[un.inst];
  const double* __restrict__ Apack = ws_at<const double>(ws, in.Jpack);
  const uint32_t* __restrict__ flipsT = flips_at(ws, in, slot);
  const uint32_t* __restrict__ base = ws_at<const uint32_t>(ws, in.base[parity]);
  const int32_t* __restrict__ roots = roots_all + in.chain0;
  double* __restrict__ partial = ws_at<double>(ws, in.partial);
  const int chains = in.chains, M = in.M, Np = in.Np, Bp = in.Bp, NB = in.NB;
  const int p = un.p, ct = un.ct;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int col_t = ct * TN;
  const int KS = Np / 4;
  const int W = Np / 32;
  const int B = chains * M;
  // per-lane column data: root-column mask of this lane's 4 columns, base row of the
  // column this lane copies (waves 2, 3)
  uint32_t rootmask = 0u;
#pragma unroll
  for (int cf = 0; cf < 4; ++cf) {
    const int col = col_t + wc * 64 + cf * 16 + (lane & 15);
    if (col < B) {
      const int c = col / M, r = roots[c];
      if (r >= 1 && col - c * M == r - 1) rootmask |= 1u << cf;
    }
  }
  const int ccol = col_t + 64 * (wave & 1) + lane;
  const uint32_t* brow = base + (size_t)(ccol < B ? ccol / M : chains) * W;

  double part[4] = {0.0, 0.0, 0.0, 0.0};
  const int nblk = (p == NB - 1 - p) ? 1 : 2;
  for (int bi = 0; bi < nblk; ++bi) {
    const int I = bi == 0 ? p : NB - 1 - p;
    const int k0 = I * kRowBlock;
    const int kw0 = k0 >> 5;
    const int nchunk = (Np - k0) / 32;   // a multiple of 4
    f64x4 acc[4][4];
#pragma unroll
    for (int rf = 0; rf < 4; ++rf)
#pragma unroll
      for (int cf = 0; cf < 4; ++cf) acc[rf][cf] = (f64x4){0.0, 0.0, 0.0, 0.0};
    // fragment (R = 8I + rf, S = k0/4 + 8 cn + s): a_blk + ((rf*KS + 8 cn + s) * 64)
    const double* a_blk = Apack + ((size_t)(8 * I) * KS + (size_t)(k0 / 4)) * 64;
    const uint32_t* fsrc = flipsT + (size_t)kw0 * Bp + col_t + lane;
    const uint32_t* bsrc = brow + kw0;
    f64_copy(fs0, a_blk, KS, fsrc, bsrc, 0, Bp, lane, wave);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int c = 0; c < nchunk; c += 2) {
      f64_copy(fs1, a_blk, KS, fsrc, bsrc, c + 1, Bp, lane, wave);
      __builtin_amdgcn_sched_barrier(0);
      f64_mfma(acc, fs0, rootmask, lane, wr, wc);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      // past the end the copy re-reads the last chunk (in bounds; fs0 is not read again
      // before the next row block refills it after a barrier)
      f64_copy(fs0, a_blk, KS, fsrc, bsrc, (c + 2 < nchunk) ? c + 2 : nchunk - 1, Bp, lane, wave);
      __builtin_amdgcn_sched_barrier(0);
      f64_mfma(acc, fs1, rootmask, lane, wr, wc);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    // epilogue: lane holds rows 4e + lane/16 (e = 0..3) of column lane%16
#pragma unroll
    for (int rf = 0; rf < 4; ++rf) {
      const int row0 = k0 + wr * 64 + rf * 16;
      const int rw = row0 >> 5;
#pragma unroll
      for (int cf = 0; cf < 4; ++cf) {
        const int col = col_t + wc * 64 + cf * 16 + (lane & 15);
        const uint32_t bw = col < B ? base[(size_t)(col / M) * W + rw] : 0u;
        const uint32_t rb = ((rootmask >> cf) & 1u) ? bw : (bw ^ flipsT[(size_t)rw * Bp + col]);
        double sum = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int bit = (row0 & 31) + 4 * e + (lane >> 4);
          const double h = acc[rf][cf][e];
          sum += ((rb >> bit) & 1u) ? -h : h;
        }
        part[cf] += sum;
      }
    }
  }
  // lanes l, l^16, l^32, l^48 hold the same column: fixed-order combine
#pragma unroll
  for (int cf = 0; cf < 4; ++cf) {
    double x = part[cf];
    x = x + __shfl_xor(x, 16);
    x = x + __shfl_xor(x, 32);
    part[cf] = x;
  }
  // the two row-halves (wr = 0, 1) of the tile are combined through LDS
  __syncthreads();
  double* red = &fs0.a[0][0][0];
  if (wr == 1 && lane < 16) {
#pragma unroll
    for (int cf = 0; cf < 4; ++cf) red[wc * 64 + cf * 16 + lane] = part[cf];
  }
  __syncthreads();
  if (wr == 0 && lane < 16) {
#pragma unroll
    for (int cf = 0; cf < 4; ++cf)
      partial[(size_t)p * Bp + col_t + wc * 64 + cf * 16 + lane] = part[cf] + red[wc * 64 + cf * 16 + lane];
  }
}

// ------------------------------------------------------------------- select

// Wave-wide reductions (64 lanes, fixed butterfly order: every lane ends with the
// same value).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = x + __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) { double y = __shfl_xor(x, o); x = y < x ? y : x; }
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) { double y = __shfl_xor(x, o); x = y > x ? y : x; }
  return x;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ unsigned long long wave_scan_u64(unsigned long long x, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    unsigned long long y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  return x;
}

struct Record {
  int32_t r, vstar;
  double e_cur, e_bar, margin;
  uint32_t flags, step;
};

// Node energies of chain c: the carried energy at the root, the scored columns
// elsewhere.  Column energies: -(scale * sum_p partial[p][col]), p in order.
__global__ void k_column_energies(double* __restrict__ Ecol, const double* __restrict__ partial, int P,
                                  int Bp, int B, double scale) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= B) return;
  double s = 0.0;
  for (int p = 0; p < P; ++p) s += partial[(size_t)p * Bp + col];
  Ecol[col] = -(scale * s);
}

// One wave per chain: node rule (MCMCMC) or Metropolis rate, move, record.
// One block of 256 threads per chain: node rule (MCMCMC) or Metropolis rate, move,
// record, and (next_base) the base words of step t+1.
//   1. all threads: column energies -(scale * sum_p partial[p][col]) (fixed order over
//      p) into the node-energy array En (LDS) at their node (column m is node m+1,
//      or the hub for column r-1), the root's entry = carried energy;
//   2. wave 0: minimum, fixed-point weights Qn (LDS), totals, threshold, prefix scan,
//      pick, margin, weighted energy;
//   3. all threads: the new state's bitset, base ^ F_{v*} (base alone for the hub),
//      or unchanged;
//   4. next_base: base of step t+1 = new state ^ F_{r'} of that step's root r'.
// Without a log-prior the largest exponent is -0, so exp(l - lmax) = exp(l) bit for
// bit and that shift is not formed.  Dynamic LDS: 16 (M+1) + 4 W bytes.
__global__ __launch_bounds__(256) void k_select(
    char* __restrict__ ws, const Inst* __restrict__ insts, const int32_t* __restrict__ chain_inst, int chain_off,
    int total_chains, double* __restrict__ e_cur, const int32_t* __restrict__ roots_all,
    const int32_t* __restrict__ roots_next_all, Record* __restrict__ ring, unsigned long long* __restrict__ moves,
    unsigned long long* __restrict__ near_ties, double* __restrict__ min_margin, double* __restrict__ e_bar_out,
    int metropolis, double beta, double tol, Key key, uint32_t chain_base, uint32_t step, uint32_t slot,
    uint32_t slot_next, int trace_steps, int next_base) {
  extern __shared__ double sel_lds[];
  __shared__ int sh_vstar;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = chain_off + blockIdx.x;   // global chain
  if (g >= total_chains) return;
  const Inst& in = insts[chain_inst[g]];
  const int c = g - in.chain0;            // chain within the instance
  const int M = in.M, W = in.W, Bp = in.Bp, P = in.P;
  const double scale = in.scale;
  uint32_t* __restrict__ spins = ws_at<uint32_t>(ws, in.spins);
  const uint32_t* __restrict__ flipsT = flips_at(ws, in, slot);
  const uint32_t* __restrict__ base = ws_at<const uint32_t>(ws, in.base[step & 1u]);
  const uint32_t* __restrict__ flipsT_next = flips_at(ws, in, slot_next);
  uint32_t* __restrict__ base_next = ws_at<uint32_t>(ws, in.base[(step + 1u) & 1u]);
  const double* __restrict__ partial = ws_at<const double>(ws, in.partial);
  const int32_t* __restrict__ roots = roots_all + in.chain0;
  const int32_t* __restrict__ roots_next = roots_next_all + in.chain0;
  const int nodes = M + 1;
  double* En = sel_lds;                                                              // [nodes]
  unsigned long long* Qn = reinterpret_cast<unsigned long long*>(sel_lds + nodes);   // [nodes]
  uint32_t* snew = reinterpret_cast<uint32_t*>(sel_lds + 2 * (size_t)nodes);        // [W]
  const int r = metropolis ? 0 : roots[c];
  const double ecur = e_cur[g];

  // 1. node energies
  for (int m = tid; m < M; m += 256) {
    const size_t col = (size_t)c * M + m;
    double acc = 0.0;
    for (int q = 0; q < P; ++q) acc += partial[(size_t)q * Bp + col];
    En[(r >= 1 && m == r - 1) ? 0 : m + 1] = -(scale * acc);
  }
  if (tid == 0) En[r] = ecur;
  __syncthreads();

  // 2. the rule (wave 0)
  if (wave == 0) {
    const uint32_t gc = chain_base + (uint32_t)g;
    uint4 ub = stream_block(key, kTagSelect, gc, step, 0u, 0u);
    const uint64_t u53 = u53_of(ub.x, ub.y);
    int vstar;
    double e_new, ebar, margin;
    if (metropolis) {
      const double e1 = En[1];
      const double dE = e1 - ecur;
      bool acc;
      if (dE <= 0.0) {
        acc = true;
        margin = __longlong_as_double(0x7FF0000000000000ll);
      } else {
        const double w = exp_weight(-(beta * dE));
        const double u = (double)u53 * 0x1.0p-53;
        acc = u < w;
        margin = fabs(u - w);
      }
      vstar = acc ? 1 : 0;
      e_new = acc ? e1 : ecur;
      ebar = e_new;
    } else {
      double emin = __longlong_as_double(0x7FF0000000000000ll);
      for (int v = lane; v < nodes; v += 64) emin = En[v] < emin ? En[v] : emin;
      emin = wave_min(emin);
      // fixed-point weights, their total, and the weighted energy
      unsigned long long wq = 0ull;
      double num = 0.0, den = 0.0;
      for (int v = lane; v < nodes; v += 64) {
        const double E = En[v];
        const double w = exp_weight(-(beta * (E - emin)));
        const unsigned long long q = (unsigned long long)(w * 0x1.0p52);
        Qn[v] = q;
        wq += q;
        num += w * E;
        den += w;
      }
      const unsigned long long Wq = wave_sum_u64(wq);
      num = wave_sum(num);
      den = wave_sum(den);
      ebar = num / den;
      // threshold t = floor(u53 * W / 2^53)
      const unsigned long long lo = (unsigned long long)u53 * Wq;
      const unsigned long long hi = __umul64hi((unsigned long long)u53, Wq);
      const unsigned long long t = (hi << 11) | (lo >> 53);
      // inclusive prefix sums in node order; first node with Q_v > t
      unsigned long long carry = 0ull;
      vstar = -1;
      unsigned long long qv = 0ull, Qv = 0ull;
      for (int base = 0; base < nodes; base += 64) {
        const int v = base + lane;
        const unsigned long long q = (v < nodes) ? Qn[v] : 0ull;
        const unsigned long long Q = carry + wave_scan_u64(q, lane);
        const unsigned long long hit = __ballot(v < nodes && Q > t);
        if (hit) {
          const int first = __ffsll((long long)hit) - 1;
          vstar = base + first;
          qv = __shfl(q, first);
          Qv = __shfl(Q, first);
          break;
        }
        carry = __shfl(Q, 63);
      }
      if (vstar < 0) {
        // unreachable for finite energies (the minimum-energy node has q = 2^52 > 0);
        // stay put and report a zero margin rather than index outside the graph
        vstar = r;
        margin = 0.0;
      } else {
        const unsigned long long d1 = t - (Qv - qv), d2 = Qv - t;
        margin = (double)(d1 < d2 ? d1 : d2) / (double)Wq;
      }
      e_new = En[vstar];
    }
    if (lane == 0) {
      const bool moved = vstar != r;
      const bool near = margin < tol;
      sh_vstar = vstar;
      e_cur[g] = e_new;
      e_bar_out[g] = ebar;
      moves[g] += moved ? 1ull : 0ull;
      near_ties[g] += near ? 1ull : 0ull;
      min_margin[g] = margin < min_margin[g] ? margin : min_margin[g];
      if (trace_steps > 0) {
        Record rec;
        rec.r = r;
        rec.vstar = vstar;
        rec.e_cur = e_new;
        rec.e_bar = ebar;
        rec.margin = margin;
        rec.flags = (near ? 1u : 0u) | (moved ? 2u : 0u);
        rec.step = step;
        ring[(size_t)(step % (uint32_t)trace_steps) * total_chains + g] = rec;
      }
    }
  }
  __syncthreads();

  // 3. the new state
  const int vstar = sh_vstar;
  const bool moved = vstar != r;
  for (int w = tid; w < W; w += 256) {
    uint32_t x;
    if (moved) {
      x = base[(size_t)c * W + w];
      if (vstar >= 1) x ^= flipsT[(size_t)w * Bp + (size_t)c * M + (vstar - 1)];
      spins[(size_t)c * W + w] = x;
    } else {
      x = spins[(size_t)c * W + w];
    }
    snew[w] = x;
  }
  if (!next_base) return;
  __syncthreads();

  // 4. base of the next step
  const int r1 = roots_next[c];
  for (int w = tid; w < W; w += 256) {
    uint32_t x = snew[w];
    if (r1 >= 1) x ^= flipsT_next[(size_t)w * Bp + (size_t)c * M + (r1 - 1)];
    base_next[(size_t)c * W + w] = x;
  }
}

// ------------------------------------------------------------------- means trace

// Chain means of the current and node-weighted energies of this step, one block of
// 256 threads, fixed-order tree: trace[slot] = {step, mean e_cur, mean e_bar}.
__global__ __launch_bounds__(256) void k_chain_means(double* __restrict__ trace, const double* __restrict__ e_cur,
                                                     const double* __restrict__ e_bar, int chains, uint32_t slot,
                                                     uint32_t step) {
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  for (int c = threadIdx.x; c < chains; c += 256) {
    a += e_cur[c];
    b += e_bar[c];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] = red[0][threadIdx.x] + red[0][threadIdx.x + o];
      red[1][threadIdx.x] = red[1][threadIdx.x] + red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    trace[3 * (size_t)slot] = (double)step;
    trace[3 * (size_t)slot + 1] = red[0][0] / (double)chains;
    trace[3 * (size_t)slot + 2] = red[1][0] / (double)chains;
  }
}

// ------------------------------------------------------------------- FP64 energy

// E(s) = -scale * sum_{i<j} J_ij s_i s_j in FP64, one block (256 threads) per global
// chain.  Thread t owns columns j = t, t+256, ...; row i is read coalesced; a
// fixed-order tree combines the threads.
__global__ __launch_bounds__(256) void k_energy_f64(double* __restrict__ out, char* __restrict__ ws,
                                                    const Inst* __restrict__ insts,
                                                    const int32_t* __restrict__ chain_inst) {
  __shared__ double red[256];
  const int g = blockIdx.x;
  const Inst& in = insts[chain_inst[g]];
  const int c = g - in.chain0;
  const int N = in.N, Np = in.Np, W = in.W;
  const double scale = in.scale;
  const double* __restrict__ J64 = ws_at<const double>(ws, in.J64);
  const uint32_t* s = ws_at<const uint32_t>(ws, in.spins) + (size_t)c * W;
  double acc = 0.0;
  for (int i = 0; i < N; ++i) {
    const double si = ((s[i >> 5] >> (i & 31)) & 1u) ? -1.0 : 1.0;
    const double* row = J64 + (size_t)i * Np;
    double rs = 0.0;
    for (int j = (int)threadIdx.x; j < N; j += 256) {
      if (j > i) {
        const double sj = ((s[j >> 5] >> (j & 31)) & 1u) ? -1.0 : 1.0;
        rs += row[j] * sj;
      }
    }
    acc += si * rs;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[g] = -(scale * red[0]);
}

}  // namespace mc3
