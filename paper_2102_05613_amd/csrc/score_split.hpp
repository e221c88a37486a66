// score_split.hpp -- candidate energies on the BF16 matrix cores (J = hi + mid + lo).
#pragma once
#include "common.hpp"

namespace mc3 {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

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

}  // namespace mc3
