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

// The 8 bfloat16 values +-1 (0x3F80 | bit << 15) of sites k0 .. k0+7 (k0 even) of a
// stored word, q0 = k0 / 2: register p holds sites k0+2p (low half, stored at bit
// q0+p) and k0+2p+1 (high half, bit 16+q0+p), so one shift brings both signs into
// place.
__device__ __forceinline__ bf16x8 spins_to_bf16(uint32_t word, int q0) {
  union { uint32_t u[4]; bf16x8 v; } r;
  // the two constants are held in registers (the empty asm statements hide their
  // values from the compiler), so that each register takes a shift and one and-or
  // (that form takes no literal operands) instead of a shift, an and and an or
  uint32_t m = 0x80008000u, one = 0x3F803F80u;
  asm("" : "+s"(m));
  asm("" : "+v"(one));
#pragma unroll
  for (int p = 0; p < 4; ++p) r.u[p] = ((word << (15 - q0 - p)) & m) | one;
  return r.v;
}

// LDS stage of the split scoring loop: the four A fragment rows of the block (six
// fragments each: two 16-k steps x three terms).
template <int WAVES>
struct SplitStage {
  uint4 a[4][6][64];
};

// This wave's share of the 24 A fragments of a chunk (4 fragment rows x 6): PER =
// 24 / WAVES consecutive slots starting at slot wave * PER, i.e. one fragment row or
// part of one (PER = 6 or 3), or two whole rows (PER = 12).  src points at the wave's
// first fragment; the next fragment row is row_stride uint4 further on.
template <int WAVES>
__device__ __forceinline__ void copy_a(SplitStage<WAVES>& st, const uint4* src, size_t row_stride, int wave) {
  constexpr int PER = 24 / WAVES;
  static_assert(PER == 3 || PER == 6 || PER == 12, "2, 4 or 8 waves");
  const int slot0 = wave * PER;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int rf = (slot0 + j) / 6, f = (slot0 + j) % 6;
    const int dr = (PER == 12) ? j / 6 : 0;
    lds_dma16(src + (size_t)dr * row_stride + (size_t)(PER == 12 ? j % 6 : j) * 64, &st.a[rf][f][0]);
  }
}

// One 32-k chunk: DMA of the next chunk's A fragments into `nxt`; this chunk's flip
// and base words (loaded into registers two chunks ago) combined into the columns'
// spin words `w`; the loads of the words two chunks ahead issued into the same
// registers; then 2 k-steps x 12 A fragments x 2 column fragments of MFMAs from
// `cur`.  The closing wait lets the four word loads stay in flight (they were issued
// after the copies; loads complete in order), so global latency of the words is hidden
// behind two chunks.
template <int WAVES, int RF_LAST = 3>
__device__ __forceinline__ void split_chunk(f32x16 (&acc)[4][2], const SplitStage<WAVES>& cur,
                                            SplitStage<WAVES>& nxt, const uint4* next_a, size_t row_stride,
                                            uint32_t (&rawf)[2], uint32_t (&rawb)[2], const uint32_t* pf0,
                                            const uint32_t* pf1, const uint32_t* pb0, const uint32_t* pb1,
                                            uint32_t rootmask, int lane, int wave, uint32_t (&w)[2]) {
  copy_a<WAVES>(nxt, next_a, row_stride, wave);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int cf = 0; cf < 2; ++cf) w[cf] = rawb[cf] ^ (((rootmask >> cf) & 1u) ? 0u : rawf[cf]);
  rawf[0] = *pf0;
  rawf[1] = *pf1;
  rawb[0] = *pb0;
  rawb[1] = *pb1;
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    bf16x8 b[2];
#pragma unroll
    for (int cf = 0; cf < 2; ++cf) b[cf] = spins_to_bf16(w[cf], 8 * s + 4 * (lane >> 5));
    bf16x8 a[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      if (i % 4 > RF_LAST) continue;
      union { uint4 q; bf16x8 v; } x;
      x.q = cur.a[i % 4][s * 3 + i / 4][lane];
      a[i] = x.v;
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      if (i % 4 > RF_LAST) continue;
#pragma unroll
      for (int cf = 0; cf < 2; ++cf)
        acc[i % 4][cf] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[cf], acc[i % 4][cf], 0, 0, 0);
    }
  }
  // vmcnt(4), no wait on the other counters
  __builtin_amdgcn_s_waitcnt(4 | (7 << 4) | (15 << 8));
  __builtin_amdgcn_s_barrier();
}

// Energies of candidate columns on the BF16 matrix cores.
//
// E(c) = -scale * sum_i c_i h_i with h_i = sum_{j>i} J_ij c_j (strict upper triangle),
// J = hi + mid + lo.  A work unit is (row-block pair p, column tile of 64 WAVES
// columns; 2, 4 or 8 waves, chosen per instance so that small instances waste few
// padding columns): row blocks p and NB-1-p (128 rows each; their K ranges start at the
// block's first row, so the pair costs NB+1 blocks of K whatever p is), taken in an
// order that alternates between units.  The waves share the A fragments through LDS,
// filled by direct global->LDS copies one 32-k chunk ahead (two stages, the copy
// running on from one row block into the next); each wave owns 64 columns, whose
// flip-set and base words each lane loads into registers two chunks ahead, combines
// and expands to +-1 BF16.  The epilogue multiplies h by the column's spins (the words
// of the block's first four chunks, kept in registers) and sums over rows in FP64; the
// unit writes one FP64 value per column.  Each block takes its
// unit from a table built by the host (the order of the table decides which XCD runs
// which unit).
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES, 2) void k_score_split(
    char* __restrict__ ws, const Inst* __restrict__ insts, const Unit* __restrict__ units,
    const int32_t* __restrict__ roots_all, uint32_t slot, uint32_t parity) {
  constexpr int TN = 64 * WAVES;
  constexpr int PER = 24 / WAVES;
  static_assert(WAVES == 2 || WAVES == 4 || WAVES == 8, "2, 4 or 8 waves");
  __shared__ SplitStage<WAVES> st0;
  __shared__ SplitStage<WAVES> st1;
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
  const int col_w = ct * TN + wave * 64;   // first column of this wave
  const int KS = Np / 16;
  const int W = Np / 32;
  const int B = chains * M;
  const int rf_w = (wave * PER) / 6, f_w = (wave * PER) % 6;
  const size_t row_stride = (size_t)KS * 3 * 64;

  // this lane's two columns: flip-word columns, base rows, root-column mask
  const int col0 = col_w + (lane & 31), col1 = col0 + 32;
  const uint32_t* brow0 = base + (size_t)(col0 < B ? col0 / M : chains) * W;
  const uint32_t* brow1 = base + (size_t)(col1 < B ? col1 / M : chains) * W;
  uint32_t rootmask = 0u;
#pragma unroll
  for (int cf = 0; cf < 2; ++cf) {
    const int col = col_w + cf * 32 + (lane & 31);
    if (col < B) {
      const int c = col / M, r = roots[c];
      if (r >= 1 && col - c * M == r - 1) rootmask |= 1u << cf;
    }
  }
  double part[2] = {0.0, 0.0};

  const int nblk = (p == NB - 1 - p) ? 1 : 2;
  const int first = un.swap ? NB - 1 - p : p;
  const int second = NB - 1 - first;
  const int nA = (Np - first * kRowBlock) / 32;
  const int nTot = nA + (nblk == 2 ? (Np - second * kRowBlock) / 32 : 0);
  // word row (k / 32) of the unit's chunk g (0 .. nTot-1), clamped to the last chunk
  auto kw_of = [&](int g) {
    g = g < nTot ? g : nTot - 1;
    return g < nA ? 4 * first + g : 4 * second + (g - nA);
  };
  auto a_src = [&](int I) {
    return Apack + (((size_t)(4 * I + rf_w) * KS + 8 * I) * 3 + f_w) * 64 + lane;
  };
  uint32_t rfE[2], rbE[2], rfO[2], rbO[2];   // raw words of even and odd chunks
  {
    const int k0w = kw_of(0), k1w = kw_of(1);
    rfE[0] = flipsT[(size_t)k0w * Bp + col0];
    rfE[1] = flipsT[(size_t)k0w * Bp + col1];
    rbE[0] = brow0[k0w];
    rbE[1] = brow1[k0w];
    rfO[0] = flipsT[(size_t)k1w * Bp + col0];
    rfO[1] = flipsT[(size_t)k1w * Bp + col1];
    rbO[0] = brow0[k1w];
    rbO[1] = brow1[k1w];
    copy_a<WAVES>(st0, a_src(first), row_stride, wave);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  int g = 0;   // the unit's chunk index
  for (int bi = 0; bi < nblk; ++bi) {
    const int I = bi == 0 ? first : second;
    const int nchunk = (Np - I * kRowBlock) / 32;   // a multiple of 4
    f32x16 acc[4][2];
#pragma unroll
    for (int rf = 0; rf < 4; ++rf)
#pragma unroll
      for (int cf = 0; cf < 2; ++cf)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[rf][cf][e] = 0.0f;
    const uint4* src = a_src(I);
    const bool more = bi + 1 < nblk;
    const uint4* src_n = more ? a_src(second) : src + (size_t)(nchunk - 1) * 6 * 64;
    // A of the chunk after local chunk c (the next block's first after the last)
#define MC3_A(cn) (((cn) >= nchunk) ? src_n : src + (size_t)(cn) * 6 * 64)
#define MC3_W(gg) flipsT + (size_t)kw_of(gg) * Bp + col0, flipsT + (size_t)kw_of(gg) * Bp + col1, \
                  brow0 + kw_of(gg), brow1 + kw_of(gg)
    // the spin words of the block's own rows are those of its first four chunks (its
    // K range starts at its first row): kept for the epilogue
    uint32_t wblk[4][2], wsv[2];
    split_chunk<WAVES, 0>(acc, st0, st1, MC3_A(1), row_stride, rfE, rbE, MC3_W(g + 2), rootmask, lane, wave,
                          wblk[0]);
    split_chunk<WAVES, 1>(acc, st1, st0, MC3_A(2), row_stride, rfO, rbO, MC3_W(g + 3), rootmask, lane, wave,
                          wblk[1]);
    split_chunk<WAVES, 2>(acc, st0, st1, MC3_A(3), row_stride, rfE, rbE, MC3_W(g + 4), rootmask, lane, wave,
                          wblk[2]);
    split_chunk<WAVES, 3>(acc, st1, st0, MC3_A(4), row_stride, rfO, rbO, MC3_W(g + 5), rootmask, lane, wave,
                          wblk[3]);
    for (int c = 4; c < nchunk; c += 2) {
      split_chunk<WAVES>(acc, st0, st1, MC3_A(c + 1), row_stride, rfE, rbE, MC3_W(g + c + 2), rootmask, lane, wave,
                         wsv);
      split_chunk<WAVES>(acc, st1, st0, MC3_A(c + 2), row_stride, rfO, rbO, MC3_W(g + c + 3), rootmask, lane, wave,
                         wsv);
    }
#undef MC3_A
#undef MC3_W
    g += nchunk;
    // epilogue: rows I*128 + 32 rf + 8(e/4) + 4(lane/32) + e%4 of column col_w + 32 cf +
    // lane%32, whose spins are bits site_bit(8(e/4) + 4(lane/32) + e%4) = 2(lane/32) +
    // [16(e%2) + 4(e/4) + (e%4)/2] of word wblk[rf][cf]; the sign bit is added (an XOR)
#pragma unroll
    for (int rf = 0; rf < 4; ++rf) {
#pragma unroll
      for (int cf = 0; cf < 2; ++cf) {
        const uint32_t sb = wblk[rf][cf] >> (2 * (lane >> 5));
        double sum = 0.0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const uint32_t neg = __builtin_amdgcn_ubfe(sb, 16 * (e & 1) + 4 * (e >> 2) + ((e & 3) >> 1), 1);
          const float h = __uint_as_float(__float_as_uint(acc[rf][cf][e]) + (neg << 31));
          sum += (double)h;
        }
        part[cf] += sum;
      }
    }
  }
#pragma unroll
  for (int cf = 0; cf < 2; ++cf) {
    const double other = __shfl_xor(part[cf], 32);
    const double tot = part[cf] + other;
    if (lane < 32) partial[(size_t)p * Bp + col_w + cf * 32 + lane] = tot;
  }
}

}  // namespace mc3
