// score_f64.hpp -- candidate energies on the FP64 matrix cores, and column energies from partials.
#pragma once
#include "common.hpp"

namespace mc3 {

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
      const uint32_t bit = (w[cf] >> site_bit(4 * s + (lane >> 4))) & 1u;
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
          const uint32_t bit = site_bit((row0 & 31) + 4 * e + (lane >> 4));
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

}  // namespace mc3
