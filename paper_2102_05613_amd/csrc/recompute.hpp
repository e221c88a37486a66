// recompute.hpp -- every chain's pair sum recomputed in FP64 on the matrix cores.
#pragma once
#include "common.hpp"

namespace mc3 {

typedef double f64x4r __attribute__((ext_vector_type(4)));

// A recompute work unit: rows 16 rt .. 16 rt + 15 of instance inst against chains
// 64 ct .. 64 ct + 63 of it; inst < 0 is an idle slot.
struct RecUnit {
  int32_t inst, rt, ct, pad;
};

// The pair sum of each chain's current state, U = sum_{i<j} J_ij s_i s_j
// (Sec. "The Sherrington-Kirkpatrick model"), through the field: with J64 symmetric
// and zero on the diagonal, 2 U = sum_i s_i h_i, h = J64 s.  H = J64 S for the
// chains' spin columns runs on the FP64 matrix cores (16x16x4); a unit writes
// upart[rt][c] = sum over its 16 rows of s_i h_i for each of its chains, and
// k_recompute_finish adds the row tiles.
//
// Four waves split the K range (the columns of J64) into quarters; each wave holds a
// 16 x 64 tile of H (four 16x16 fragments, one per 16 chains).  The k index of the
// instruction is relabelled so that a lane loads contiguous couplings: in step s of a
// 32-column chunk starting at k0, lane l supplies row l%16 at column
// k0 + 8 (l/16) + s and the spin of chain l%16 at the same column, so the eight steps
// cover the chunk's 32 columns once.  The waves' tiles are added through LDS in wave
// order, then each lane multiplies its rows by the chain's spins (rows 4e + l/16 of
// column l%16 in element e), and lanes l, l^16, l^32, l^48 are combined.  +-1 couplings
// give exact integers.
__global__ __launch_bounds__(256) void k_recompute_f64(char* __restrict__ ws, const Inst* __restrict__ insts,
                                                       const RecUnit* __restrict__ units) {
  __shared__ double red[3][4][4][64];
  const RecUnit un = units[blockIdx.x];
  if (un.inst < 0) return;
  const Inst& in = insts[un.inst];
  const int Np = in.Np, W = in.W, chains = in.chains;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i0 = 16 * un.rt, c0 = 64 * un.ct;
  const int ncf = min(4, (chains - c0 + 15) / 16);
  const double* __restrict__ J64 = ws_at<const double>(ws, in.J64);
  const uint32_t* __restrict__ spins = ws_at<const uint32_t>(ws, in.spins);
  const int Kq = Np / 4;   // a multiple of 32
  const int kb = wave * Kq;
  const int q = lane >> 4;
  const double* __restrict__ arow = J64 + (size_t)(i0 + (lane & 15)) * Np + kb + 8 * q;
  const uint32_t* srow[4];
  bool valid[4];
#pragma unroll
  for (int cf = 0; cf < 4; ++cf) {
    const int c = c0 + 16 * cf + (lane & 15);
    valid[cf] = c < chains;
    srow[cf] = spins + (size_t)(valid[cf] ? c : 0) * W;
  }
  f64x4r acc[4];
#pragma unroll
  for (int cf = 0; cf < 4; ++cf) acc[cf] = (f64x4r){0.0, 0.0, 0.0, 0.0};
  for (int kk = 0; kk < Kq; kk += 32) {
    double a[8];
    const double2* ap = reinterpret_cast<const double2*>(arow + kk);
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const double2 v = ap[h];
      a[2 * h] = v.x;
      a[2 * h + 1] = v.y;
    }
    const int w = (kb + kk) >> 5;
    uint32_t sw[4];
#pragma unroll
    for (int cf = 0; cf < 4; ++cf) sw[cf] = cf < ncf ? srow[cf][w] : 0u;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
#pragma unroll
      for (int cf = 0; cf < 4; ++cf) {
        if (cf >= ncf) continue;
        const uint32_t bit = (sw[cf] >> site_bit(8 * q + s)) & 1u;
        const double b = valid[cf] ? (bit ? -1.0 : 1.0) : 0.0;
        acc[cf] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b, acc[cf], 0, 0, 0);
      }
    }
  }
  if (wave >= 1) {
#pragma unroll
    for (int cf = 0; cf < 4; ++cf)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[wave - 1][cf][e][lane] = acc[cf][e];
  }
  __syncthreads();
  if (wave != 0) return;
  double* __restrict__ upart = ws_at<double>(ws, in.upart);
  const uint32_t rword = (uint32_t)i0 >> 5;   // the 16 rows lie in one spin word
#pragma unroll
  for (int cf = 0; cf < 4; ++cf) {
    if (cf >= ncf) continue;
    const uint32_t sw = valid[cf] ? srow[cf][rword] : 0u;
    double sum = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double h = ((acc[cf][e] + red[0][cf][e][lane]) + red[1][cf][e][lane]) + red[2][cf][e][lane];
      const uint32_t bit = (sw >> site_bit((uint32_t)((i0 & 31) + 4 * e + q))) & 1u;
      sum += bit ? -h : h;
    }
    sum = sum + __shfl_xor(sum, 16);
    sum = sum + __shfl_xor(sum, 32);
    const int c = c0 + 16 * cf + lane;
    if (lane < 16 && c < chains) upart[(size_t)un.rt * chains + c] = sum;
  }
}

// Per global chain: U = (sum of the row tiles' upart in order) / 2 and E = -(scale U).
// mode 0: carry them (u_cur, e_cur).  mode 1 (the periodic check): the carried
// energy's distance to E is the drift, its largest value per chain is kept and a
// drift above drift_tol (|E| + 1) is counted; the recomputed values replace the
// carried ones (the repair).
__global__ void k_recompute_finish(char* __restrict__ ws, const Inst* __restrict__ insts,
                                   const int32_t* __restrict__ chain_inst, int total_chains,
                                   double* __restrict__ u_cur, double* __restrict__ e_cur,
                                   double* __restrict__ drift, unsigned long long* __restrict__ drift_events,
                                   double drift_tol, int mode) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_chains) return;
  const Inst& in = insts[chain_inst[g]];
  const int c = g - in.chain0;
  const double* __restrict__ upart = ws_at<const double>(ws, in.upart);
  const int nrt = in.Np / 16;
  double S = 0.0;
  for (int rt = 0; rt < nrt; ++rt) S += upart[(size_t)rt * in.chains + c];
  const double U = 0.5 * S;
  const double E = -(in.scale * U);
  if (mode == 1) {
    const double d = fabs(-(in.scale * u_cur[g]) - E);
    if (!(d <= drift[g])) drift[g] = d;                          // a NaN drift is kept
    if (!(d <= drift_tol * (fabs(E) + 1.0))) drift_events[g] += 1ull;
  }
  u_cur[g] = U;
  e_cur[g] = E;
}

}  // namespace mc3
