// common.hpp -- types and helpers shared by the device kernels of the SK MCMCMC hot
// path (gfx950).
//
// Data layout in HBM (all sizes padded: Np = N rounded up to 128, W = Np/32 words
// per spin bitset, B = chains*M candidate columns, Bp = B rounded up to 512):
//   J64     [Np][Np] double, row-major, zero outside the N x N block.
//   Jsplit  bf16 hi/mid/lo of the strict upper triangle of J, in matrix-core
//           fragment order: fragment (R, S, t) = rows 32R..32R+31, k = 16S..16S+15,
//           term t, stored as 64 lanes x 8 bf16 (lane l holds row 32R + l%32,
//           k = 16S + 8(l/32) + e for e = 0..7); 1 KiB per fragment.
//   spins   [chains][W] uint32 bitsets (set bit = spin -1); within a word, site k of
//           its 32 sites sits at bit site_bit(k): even sites in the low half, odd
//           sites in the high half, so that two sites 16 bits apart become the two
//           bfloat16 signs of one register with a single shift (every bitset below
//           uses this order).
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

constexpr int kRowBlock = 128;  // rows of J per scoring work unit (4 fragments of 32)

// Bit position of site k (0..31) within its word: site 2q at bit q, site 2q+1 at bit
// 16+q.
__host__ __device__ constexpr uint32_t site_bit(uint32_t k) { return ((k & 1u) << 4) | (k >> 1); }

// A word in site order (bit k = site k) rearranged into the stored order, and back.
__host__ __device__ inline uint32_t stored_word(uint32_t natural) {
  uint32_t r = 0u;
  for (uint32_t k = 0; k < 32u; ++k) r |= ((natural >> k) & 1u) << site_bit(k);
  return r;
}
__host__ __device__ inline uint32_t natural_word(uint32_t stored) {
  uint32_t r = 0u;
  for (uint32_t k = 0; k < 32u; ++k) r |= ((stored >> site_bit(k)) & 1u) << k;
  return r;
}

// One SK instance of a batch, as the kernels see it.  Byte offsets are into the
// workspace; the per-chain arrays (energies, roots, counters, records) are global over
// the batch and indexed by chain0 + c.
struct Inst {
  int32_t N, Np, W, M;
  int32_t chains, kmin, kmax, B;
  int32_t Bp, NB, P, chain0;
  int32_t arity;    // tree arity: the parent of node v >= 1 is (v-1)/arity (arity M: the star)
  int32_t law;      // root law: 0 uniform over the M+1 nodes, 1 line-graph addition process
  double scale;
  uint64_t J64, Jpack, flips, flip_slot, base[2], partial, spins;
  uint64_t field;   // [chains][Np] FP64 local fields (field-update path only)
  uint64_t prior;   // [M+1] FP64 log-prior of the nodes (line law), 0 = none
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

template <class T>
__device__ __forceinline__ T* ws_at(char* ws, uint64_t off) {
  return reinterpret_cast<T*>(ws + off);
}

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

}  // namespace mc3
