// kernels.hpp -- device kernels of the SK MCMCMC hot path (gfx950).
//
// Data layout in HBM (all sizes padded: Np = N rounded up to 128, W = Np/32 words
// per spin bitset, Bp = candidate columns rounded up to the scoring tile):
//   J64     [Np][Np] double, row-major, zero outside the N x N block.
//   Jsplit  bf16 hi/mid/lo of the strict upper triangle of J, in matrix-core
//           fragment order: fragment (R, S, t) = rows 32R..32R+31, k = 16S..16S+15,
//           term t, stored as 64 lanes x 8 bf16 (lane l holds row 32R + l%32,
//           k = 16S + 8(l/32) + e for e = 0..7); 1 KiB per fragment.
//   spins   [chains][W] uint32 bitsets (set bit = spin -1).
//   flips   [chains][M][W] uint32 flip sets of edges 1..M.
//   candT   [W][Bp] uint32: word w of every candidate column, columns contiguous so
//           a matrix-core B fragment's 32 columns are one 128-byte line.
//   partial [P][Bp] double: energy contributions of row-block pair p.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_rng.hpp"

namespace mc3 {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRowBlock = 128;  // rows of J per scoring work unit (4 fragments of 32)

// ------------------------------------------------------------------- init spins

// Spins of every chain from the init stream: word w of the chain's bitset is word w
// of stream (init, chain, step 0, edge 0); bits at and beyond N are cleared.
__global__ void k_init_spins(uint32_t* __restrict__ spins, int chains, int N, int W, Key key,
                             uint32_t chain_base) {
  int c = blockIdx.y;
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= chains || w >= W) return;
  uint32_t v = 0;
  if (w * 32 < N) {
    uint4 b = stream_block(key, kTagInit, chain_base + (uint32_t)c, 0u, 0u, (uint32_t)w / 4u);
    v = pick(b, (uint32_t)w % 4u);
    int rem = N - w * 32;
    if (rem < 32) v &= (1u << rem) - 1u;
  }
  spins[(size_t)c * W + w] = v;
}

// ------------------------------------------------------------------- propose

// One thread per (chain, edge): k_e and Floyd's k-of-N draw into the thread's own
// LDS bitset, then a coalesced copy of the block's bitsets to `flips`.  Thread
// (chain, edge 1) also draws the chain's root.  Dynamic LDS: blockDim.x * W words.
__global__ void k_propose(uint32_t* __restrict__ flips, int32_t* __restrict__ roots, int chains,
                          int M, int N, int W, int kmin, int kmax, int metropolis, Key key,
                          uint32_t chain_base, uint32_t step) {
  extern __shared__ uint32_t lds_bits[];
  const int T = blockDim.x;
  const long long g0 = (long long)blockIdx.x * T;
  const long long total = (long long)chains * M;
  // clear this block's bitsets
  for (int i = threadIdx.x; i < T * W; i += T) lds_bits[i] = 0u;
  __syncthreads();
  const long long g = g0 + threadIdx.x;
  if (g < total) {
    const int c = (int)(g / M);
    const uint32_t e = (uint32_t)(g % M) + 1u;
    const uint32_t gc = chain_base + (uint32_t)c;
    uint32_t* mine = lds_bits + (size_t)threadIdx.x * W;
    uint4 blk = stream_block(key, kTagEdge, gc, step, e, 0u);
    const int k = kmin + (int)randint(blk.x, (uint32_t)(kmax - kmin + 1));
    for (int idx = 0; idx < k; ++idx) {
      const uint32_t n = 1u + (uint32_t)idx;
      if ((n & 3u) == 0u) blk = stream_block(key, kTagEdge, gc, step, e, n >> 2);
      const uint32_t j = (uint32_t)(N - k + idx);
      const uint32_t t = randint(pick(blk, n & 3u), j + 1u);
      const uint32_t bt = mine[t >> 5] >> (t & 31u) & 1u;
      const uint32_t pos = bt ? j : t;
      mine[pos >> 5] |= 1u << (pos & 31u);
    }
    if (e == 1u) {
      uint32_t r = 0u;
      if (!metropolis) {
        uint4 rb = stream_block(key, kTagRoot, gc, step, 0u, 0u);
        r = randint(rb.x, (uint32_t)(M + 1));
      }
      roots[c] = (int32_t)r;
    }
  }
  __syncthreads();
  const long long nthreads = (total - g0) < T ? (total - g0) : T;
  const long long words = nthreads * W;
  uint32_t* dst = flips + g0 * W;
  for (long long i = threadIdx.x; i < words; i += T) dst[i] = lds_bits[i];
}

// Candidate column m of chain c is node v = m (m < r) or m + 1 (m >= r).  Its bitset
// is s ^ D_v with D_v = F_v (r = 0), F_r (v = 0, r >= 1) or F_r ^ F_v (r >= 1).
// Grid: x over columns (coalesced stores), y over words.
__global__ void k_build_candidates(uint32_t* __restrict__ candT, const uint32_t* __restrict__ spins,
                                   const uint32_t* __restrict__ flips, const int32_t* __restrict__ roots,
                                   int chains, int M, int W, int Bp) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = blockIdx.y;
  if (col >= Bp || w >= W) return;
  uint32_t out = 0u;
  if (col < chains * M) {
    const int c = col / M, m = col % M;
    const int r = roots[c];
    const int v = m < r ? m : m + 1;
    const uint32_t s = spins[(size_t)c * W + w];
    const uint32_t* fc = flips + (size_t)c * M * W;
    uint32_t d;
    if (r == 0) d = fc[(size_t)(v - 1) * W + w];
    else if (v == 0) d = fc[(size_t)(r - 1) * W + w];
    else d = fc[(size_t)(r - 1) * W + w] ^ fc[(size_t)(v - 1) * W + w];
    out = s ^ d;
  }
  candT[(size_t)w * Bp + col] = out;
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

// Expand 8 spin bits (set = -1) into 8 bfloat16 values +-1 (0x3F80 | bit << 15).
__device__ __forceinline__ bf16x8 spins_to_bf16(uint32_t byte) {
  union { uint32_t u[4]; bf16x8 v; } r;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const uint32_t x = (byte >> (2 * p)) & 3u;
    r.u[p] = ((x * 0x40008000u) & 0x80008000u) | 0x3F803F80u;
  }
  return r.v;
}

// Energies of candidate columns on the BF16 matrix cores.
//
// E(c) = -scale * sum_i c_i h_i with h_i = sum_{j>i} J_ij c_j (strict upper triangle),
// J = hi + mid + lo.  A work unit is (row-block pair p, column tile): row blocks p and
// NB-1-p (128 rows each; their K ranges start at the block's first row, so the pair
// costs NB+1 blocks of K whatever p is).  Four waves share the A tiles through LDS
// (double-buffered, 32 k per stage); each wave owns 32*CF columns whose spins are
// expanded from bitsets in registers.  The epilogue multiplies h by the column's
// spins and sums over rows in FP64; the unit writes one FP64 value per column.
// Units are laid out XCD-major so the blocks of one XCD share few row pairs of J.
template <int CF>
__global__ __launch_bounds__(256, 1) void k_score_split(const uint4* __restrict__ Apack,
                                                        const uint32_t* __restrict__ candT,
                                                        double* __restrict__ partial, int Np, int Bp,
                                                        int NB, int P, int CT) {
  constexpr int TN = 4 * 32 * CF;
  __shared__ uint4 lds[2][4][6][64];
  const int U = P * CT;
  const int per = (U + 7) / 8;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int u = xcd * per + slot;
  if (slot >= per || u >= U) return;
  const int p = u / CT, ct = u % CT;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int col_w = ct * TN + wave * 32 * CF;   // first column of this wave
  const int KS = Np / 16;

  double part[CF];
#pragma unroll
  for (int cf = 0; cf < CF; ++cf) part[cf] = 0.0;

  const int nblk = (p == NB - 1 - p) ? 1 : 2;
  for (int bi = 0; bi < nblk; ++bi) {
    const int I = bi == 0 ? p : NB - 1 - p;
    const int k0 = I * kRowBlock;
    const int nchunk = (Np - k0) / 32;
    f32x16 acc[4][CF];
#pragma unroll
    for (int rf = 0; rf < 4; ++rf)
#pragma unroll
      for (int cf = 0; cf < CF; ++cf)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[rf][cf][e] = 0.0f;

    // this thread stages fragment row R = 4I + wave, lane `lane`, six fragments per chunk
    const uint4* src = Apack + (((size_t)(4 * I + wave) * KS + (k0 / 16)) * 3) * 64 + lane;
    uint4 stage[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) stage[f] = src[f * 64];
#pragma unroll
    for (int f = 0; f < 6; ++f) lds[0][wave][f][lane] = stage[f];
    __syncthreads();

    for (int c = 0; c < nchunk; ++c) {
      const int buf = c & 1;
      if (c + 1 < nchunk) {
        const uint4* s2 = src + (size_t)(c + 1) * 6 * 64;
#pragma unroll
        for (int f = 0; f < 6; ++f) stage[f] = s2[f * 64];
      }
      const int kw = (k0 >> 5) + c;
      uint32_t bits[CF];
#pragma unroll
      for (int cf = 0; cf < CF; ++cf) bits[cf] = candT[(size_t)kw * Bp + col_w + cf * 32 + (lane & 31)];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        bf16x8 b[CF];
#pragma unroll
        for (int cf = 0; cf < CF; ++cf) b[cf] = spins_to_bf16((bits[cf] >> (16 * s + 8 * (lane >> 5))) & 0xFFu);
#pragma unroll
        for (int rf = 0; rf < 4; ++rf) {
#pragma unroll
          for (int t = 0; t < 3; ++t) {
            union { uint4 q; bf16x8 v; } a;
            a.q = lds[buf][rf][s * 3 + t][lane];
#pragma unroll
            for (int cf = 0; cf < CF; ++cf)
              acc[rf][cf] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, b[cf], acc[rf][cf], 0, 0, 0);
          }
        }
      }
      if (c + 1 < nchunk) {
#pragma unroll
        for (int f = 0; f < 6; ++f) lds[buf ^ 1][wave][f][lane] = stage[f];
      }
      __syncthreads();
    }
    // epilogue: rows I*128 + 32 rf + 8(e/4) + 4(lane/32) + e%4 of column col_w + 32 cf + lane%32
#pragma unroll
    for (int rf = 0; rf < 4; ++rf) {
#pragma unroll
      for (int cf = 0; cf < CF; ++cf) {
        const uint32_t rb = candT[(size_t)(4 * I + rf) * Bp + col_w + cf * 32 + (lane & 31)];
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
    const double tot = (lane < 32) ? part[cf] + other : other + part[cf];
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

// Energies of candidate columns on the FP64 matrix cores (16x16x4).  Same work
// units as the split kernel (row-block pair of 128 rows x column tile); the four
// waves form a 2 x 2 grid of 64 x 64 tiles; A (J) is staged through LDS, 16 k per
// stage, double-buffered; B (+-1) is built from the candidate bitsets.
// Output layout of the 16x16x4 f64 instruction: C[i][j] is element i/4 of lane
// j + 16 (i % 4).
__global__ __launch_bounds__(256, 2) void k_score_f64(const double* __restrict__ Apack,
                                                      const uint32_t* __restrict__ candT,
                                                      double* __restrict__ partial, int Np, int Bp,
                                                      int NB, int P, int CT) {
  constexpr int TN = 128;
  __shared__ double lds[2][8][4][64];
  const int U = P * CT;
  const int per = (U + 7) / 8;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int u = xcd * per + slot;
  if (slot >= per || u >= U) return;
  const int p = u / CT, ct = u % CT;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int col_w = ct * TN + wc * 64;
  const int KS = Np / 4;
  const double one = 1.0;

  double part[4] = {0.0, 0.0, 0.0, 0.0};
  const int nblk = (p == NB - 1 - p) ? 1 : 2;
  for (int bi = 0; bi < nblk; ++bi) {
    const int I = bi == 0 ? p : NB - 1 - p;
    const int k0 = I * kRowBlock;
    const int nchunk = (Np - k0) / 16;
    f64x4 acc[4][4];
#pragma unroll
    for (int rf = 0; rf < 4; ++rf)
#pragma unroll
      for (int cf = 0; cf < 4; ++cf) acc[rf][cf] = (f64x4){0.0, 0.0, 0.0, 0.0};
    // staging: thread stages local row fragment tid/32 (of 8), 4 fragments x 64 lanes
    // = 256 doubles per piece; this thread copies doubles (tid%32)*8 .. +7 of it.
    const int piece = tid >> 5, off = (tid & 31) * 8;
    const double* src = Apack + ((size_t)(8 * I + piece) * KS + (k0 / 4)) * 64 + off;
    double2 stage[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) stage[q] = *(const double2*)(src + 2 * q);
    double* ldsflat0 = &lds[0][piece][0][0] + off;
#pragma unroll
    for (int q = 0; q < 4; ++q) *(double2*)(ldsflat0 + 2 * q) = stage[q];
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
      const int buf = c & 1;
      if (c + 1 < nchunk) {
        const double* s2 = src + (size_t)(c + 1) * 4 * 64;
#pragma unroll
        for (int q = 0; q < 4; ++q) stage[q] = *(const double2*)(s2 + 2 * q);
      }
      // spins of the chunk's 16 rows of k for this wave's 64 columns
      const int kbase = k0 + 16 * c;
      uint32_t bw[4];
#pragma unroll
      for (int cf = 0; cf < 4; ++cf) bw[cf] = candT[(size_t)(kbase >> 5) * Bp + col_w + cf * 16 + (lane & 15)];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double b[4];
#pragma unroll
        for (int cf = 0; cf < 4; ++cf) {
          const uint32_t bit = (bw[cf] >> ((kbase & 31) + 4 * s + (lane >> 4))) & 1u;
          b[cf] = __longlong_as_double(__double_as_longlong(one) | ((long long)bit << 63));
        }
#pragma unroll
        for (int rf = 0; rf < 4; ++rf) {
          const double a = lds[buf][wr * 4 + rf][s][lane];
#pragma unroll
          for (int cf = 0; cf < 4; ++cf)
            acc[rf][cf] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[cf], acc[rf][cf], 0, 0, 0);
        }
      }
      if (c + 1 < nchunk) {
        double* d = &lds[buf ^ 1][piece][0][0] + off;
#pragma unroll
        for (int q = 0; q < 4; ++q) *(double2*)(d + 2 * q) = stage[q];
      }
      __syncthreads();
    }
    // epilogue: lane holds rows 4e + lane/16 (e = 0..3) of column lane%16
#pragma unroll
    for (int rf = 0; rf < 4; ++rf) {
      const int row0 = k0 + wr * 64 + rf * 16;
#pragma unroll
      for (int cf = 0; cf < 4; ++cf) {
        const uint32_t rb = candT[(size_t)(row0 >> 5) * Bp + col_w + cf * 16 + (lane & 15)];
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
  double* red = &lds[0][0][0][0];
  if (wr == 1 && lane < 16) {
#pragma unroll
    for (int cf = 0; cf < 4; ++cf) red[wc * 64 + cf * 16 + lane] = part[cf];
  }
  __syncthreads();
  if (wr == 0 && lane < 16) {
#pragma unroll
    for (int cf = 0; cf < 4; ++cf)
      partial[(size_t)p * Bp + col_w + cf * 16 + lane] = part[cf] + red[wc * 64 + cf * 16 + lane];
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
// Column energies are reduced from the scoring partials here (fixed order over p) and
// kept in Ecol for the later passes of the same lane.
__global__ __launch_bounds__(256) void k_select(
    uint32_t* __restrict__ spins, double* __restrict__ e_cur, const uint32_t* __restrict__ candT,
    const double* __restrict__ partial, int P, double scale, double* __restrict__ Ecol,
    const int32_t* __restrict__ roots, Record* __restrict__ ring,
    unsigned long long* __restrict__ moves, unsigned long long* __restrict__ near_ties,
    double* __restrict__ min_margin, int chains, int M, int W, int Bp, int metropolis, double beta,
    double tol, Key key, uint32_t chain_base, uint32_t step, int trace_steps) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= chains) return;
  const uint32_t gc = chain_base + (uint32_t)c;
  const int r = roots[c];
  const double ecur = e_cur[c];
  double* Ec = Ecol + (size_t)c * M;
  for (int m = lane; m < M; m += 64) {
    const size_t col = (size_t)c * M + m;
    double acc = 0.0;
    for (int q = 0; q < P; ++q) acc += partial[(size_t)q * Bp + col];
    Ec[m] = -(scale * acc);
  }
  uint4 ub = stream_block(key, kTagSelect, gc, step, 0u, 0u);
  const uint64_t u53 = u53_of(ub.x, ub.y);

  int vstar;
  double e_new, ebar, margin;
  if (metropolis) {
    const double e1 = Ec[0];
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
    const int nodes = M + 1;
    // pass 1: minimum energy over the nodes
    double emin = __longlong_as_double(0x7FF0000000000000ll);
    for (int v = lane; v < nodes; v += 64) {
      const double E = (v == r) ? ecur : Ec[v < r ? v : v - 1];
      emin = E < emin ? E : emin;
    }
    emin = wave_min(emin);
    // pass 2: log-weight maximum (a no-op shift without a log-prior, kept so the
    // exponent is formed exactly as the rule states it)
    double lmax = -__longlong_as_double(0x7FF0000000000000ll);
    for (int v = lane; v < nodes; v += 64) {
      const double E = (v == r) ? ecur : Ec[v < r ? v : v - 1];
      const double l = -(beta * (E - emin));
      lmax = l > lmax ? l : lmax;
    }
    lmax = wave_max(lmax);
    // pass 3: fixed-point weights, their total, and the weighted energy
    unsigned long long wq = 0ull;
    double num = 0.0, den = 0.0;
    for (int v = lane; v < nodes; v += 64) {
      const double E = (v == r) ? ecur : Ec[v < r ? v : v - 1];
      const double w = exp_weight(-(beta * (E - emin)) - lmax);
      wq += (unsigned long long)(w * 0x1.0p52);
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
    // pass 4: inclusive prefix sums in node order; first node with Q_v > t
    unsigned long long carry = 0ull;
    vstar = -1;
    unsigned long long qv = 0ull, Qv = 0ull;
    for (int base = 0; base < nodes; base += 64) {
      const int v = base + lane;
      unsigned long long q = 0ull;
      if (v < nodes) {
        const double E = (v == r) ? ecur : Ec[v < r ? v : v - 1];
        const double w = exp_weight(-(beta * (E - emin)) - lmax);
        q = (unsigned long long)(w * 0x1.0p52);
      }
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
    e_new = (vstar == r) ? ecur : Ec[vstar < r ? vstar : vstar - 1];
  }
  const int cur_node = metropolis ? 0 : r;
  const bool moved = vstar != cur_node;
  if (moved) {
    const int m = metropolis ? 0 : (vstar < r ? vstar : vstar - 1);
    const int col = c * M + m;
    for (int w = lane; w < W; w += 64) spins[(size_t)c * W + w] = candT[(size_t)w * Bp + col];
  }
  if (lane == 0) {
    const bool near = margin < tol;
    e_cur[c] = e_new;
    moves[c] += moved ? 1ull : 0ull;
    near_ties[c] += near ? 1ull : 0ull;
    min_margin[c] = margin < min_margin[c] ? margin : min_margin[c];
    if (trace_steps > 0) {
      Record rec;
      rec.r = metropolis ? 0 : r;
      rec.vstar = vstar;
      rec.e_cur = e_new;
      rec.e_bar = ebar;
      rec.margin = margin;
      rec.flags = (near ? 1u : 0u) | (moved ? 2u : 0u);
      rec.step = step;
      ring[(size_t)(step % (uint32_t)trace_steps) * chains + c] = rec;
    }
  }
}

// ------------------------------------------------------------------- FP64 energy

// E(s) = -scale * sum_{i<j} J_ij s_i s_j in FP64, one block (256 threads) per chain.
// Thread t owns columns j = t, t+256, ...; row i is read coalesced; a fixed-order
// tree combines the threads.
__global__ __launch_bounds__(256) void k_energy_f64(double* __restrict__ out, const uint32_t* __restrict__ spins,
                                                    const double* __restrict__ J64, int N, int Np, int W,
                                                    double scale) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const uint32_t* s = spins + (size_t)c * W;
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
  if (threadIdx.x == 0) out[c] = -(scale * red[0]);
}

}  // namespace mc3
