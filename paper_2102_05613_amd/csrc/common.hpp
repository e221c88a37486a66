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
  double tie_coef;  // near-tie threshold per unit of beta (4 eps_E of the precision), 0 with a fixed one
  uint64_t J64, Jpack, flips, flip_slot, base[2], partial, spins;
  uint64_t upart;   // [Np/16][chains] FP64 partial sums of the FP64 recompute
  uint64_t field;   // [chains][Np] FP64 local fields (field-update path only)
  uint64_t prior;   // [M+1] FP64 log-prior of the nodes (line and table laws), 0 = none
  uint64_t root_q;  // [M+1] uint64 cumulative fixed-point root weights (table law), 0 = none
};

// Flip sets of the step held in ring slot `slot` (slots of flip_slot bytes each).
__device__ __forceinline__ uint32_t* flips_at(char* ws, const Inst& in, uint32_t slot) {
  return reinterpret_cast<uint32_t*>(ws + in.flips + (uint64_t)slot * in.flip_slot);
}

// A scoring work unit (row-block pair p, column tile ct of instance inst); inst < 0 is
// an idle slot of the launch grid.
struct Unit {
  int32_t inst, p, ct, swap;   // swap: the split kernel takes row block NB-1-p first
};

// A proposal block: edges edge0 .. edge0 + count - 1 (flattened chain*M + e-1) of
// instance inst, count <= blockDim.x (whole chains when the tree's path sets are formed
// inside the block).
struct PBlock {
  int32_t inst, edge0, count, pad;
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

// Wave-wide operations (64 lanes, all active) on DPP lane permutations and lane reads,
// with no LDS round trips.  A reduction swaps neighbours, then pairs, then half-rows,
// then the halves of each row of 16 lanes (every lane of a row then holds the row's
// result: the operations are commutative) and combines the four rows read from lanes
// 0, 16, 32 and 48 as (r0 . r1) . (r2 . r3); sums are taken in this fixed order.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const uint32_t lo = dpp_u32<CTRL>((uint32_t)b), hi = dpp_u32<CTRL>((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}
template <class Op>
__device__ __forceinline__ double wave_reduce_f64(double x, Op op) {
  x = op(x, dpp_f64<0xB1>(x));    // quad_perm [1,0,3,2]
  x = op(x, dpp_f64<0x4E>(x));    // quad_perm [2,3,0,1]
  x = op(x, dpp_f64<0x141>(x));   // row_half_mirror
  x = op(x, dpp_f64<0x140>(x));   // row_mirror
  const double r0 = readlane_f64(x, 0), r1 = readlane_f64(x, 16), r2 = readlane_f64(x, 32), r3 = readlane_f64(x, 48);
  return op(op(r0, r1), op(r2, r3));
}
__device__ __forceinline__ double wave_sum(double x) {
  return wave_reduce_f64(x, [](double a, double b) { return a + b; });
}
__device__ __forceinline__ double wave_min(double x) {
  return wave_reduce_f64(x, [](double a, double b) { return b < a ? b : a; });
}
__device__ __forceinline__ double wave_max(double x) {
  return wave_reduce_f64(x, [](double a, double b) { return b > a ? b : a; });
}
// row_shr by N: a lane whose source lies before the start of its row reads 0
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_shr_u64(unsigned long long x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)hi << 32) | lo;
}
// Inclusive prefix sum over the lanes (exact integer arithmetic): Hillis-Steele within
// each row (shifts 1, 2, 4, 8), then the totals of the rows before.
__device__ __forceinline__ unsigned long long wave_scan_u64(unsigned long long x, int lane) {
  x += dpp_shr_u64<0x111>(x);
  x += dpp_shr_u64<0x112>(x);
  x += dpp_shr_u64<0x114>(x);
  x += dpp_shr_u64<0x118>(x);
  const unsigned long long r0 = readlane_u64(x, 15), r1 = readlane_u64(x, 31), r2 = readlane_u64(x, 47);
  const int row = lane >> 4;
  return x + (row >= 1 ? r0 : 0ull) + (row >= 2 ? r1 : 0ull) + (row >= 3 ? r2 : 0ull);
}

struct Record {
  int32_t r, vstar;
  double e_cur, e_bar, margin;
  uint32_t flags, step;
};

}  // namespace mc3
