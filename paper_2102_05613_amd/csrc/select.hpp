// select.hpp -- the node rule, the move, the means trace and FP64 energies.
#pragma once
#include "common.hpp"

namespace mc3 {

// ------------------------------------------------------------------- select

// The selection of one chain-step, computed by one whole wave (every lane gets the
// result).  En[0..M] are the node energies (the current node r holds the carried
// energy), Qn is LDS scratch for the fixed-point weights.  MCMCMC: Emin, weights
// w_v = exp(-(beta (E_v - Emin))), q_v = floor(w_v 2^52), inclusive prefix sums in
// node order, threshold t = floor(u53 W / 2^53), v* = min{v : Q_v > t}; the margin is
// the draw's distance to the edges of its interval as a fraction of W, and the
// node-weighted energy sum w E / sum w.  Metropolis (M = 1): accept iff dE <= 0 or
// u53 / 2^53 < exp(-(beta dE)).  With a log-prior lambda (the line process) the
// exponents are l_v = -(beta (E_v - Emin)) + lambda_v and the weights
// exp(l_v - max l); without one the largest exponent is -0, so exp(l - lmax) =
// exp(l) bit for bit and that shift is not formed.
struct RuleOut {
  int vstar;
  double e_new, ebar, margin;
};

__device__ __forceinline__ RuleOut apply_rule(const double* En, unsigned long long* Qn, int M, int r, double ecur,
                                              int metropolis, double beta, uint64_t u53, int lane,
                                              const double* __restrict__ prior) {
  RuleOut o;
  const int nodes = M + 1;
  if (metropolis) {
    const double e1 = En[1];
    const double dE = e1 - ecur;
    bool acc;
    if (dE <= 0.0) {
      acc = true;
      o.margin = __longlong_as_double(0x7FF0000000000000ll);
    } else {
      const double w = exp_weight(-(beta * dE));
      const double u = (double)u53 * 0x1.0p-53;
      acc = u < w;
      o.margin = fabs(u - w);
    }
    o.vstar = acc ? 1 : 0;
    o.e_new = acc ? e1 : ecur;
    o.ebar = o.e_new;
    return o;
  }
  // lane l holds nodes [l K, l K + K): node order is lane order
  const int K = (nodes + 63) >> 6;
  const int v0 = lane * K, v1 = min(v0 + K, nodes);
  double emin = __longlong_as_double(0x7FF0000000000000ll);
  for (int v = v0; v < v1; ++v) emin = En[v] < emin ? En[v] : emin;
  emin = wave_min(emin);
  double lmax = 0.0;
  if (prior) {
    lmax = __longlong_as_double(0xFFF0000000000000ll);
    for (int v = v0; v < v1; ++v) {
      const double l = -(beta * (En[v] - emin)) + prior[v];
      lmax = l > lmax ? l : lmax;
    }
    lmax = wave_max(lmax);
  }
  // fixed-point weights, their total, and the weighted energy
  unsigned long long wq = 0ull;
  double num = 0.0, den = 0.0;
  for (int v = v0; v < v1; ++v) {
    const double E = En[v];
    const double w = prior ? exp_weight((-(beta * (E - emin)) + prior[v]) - lmax) : exp_weight(-(beta * (E - emin)));
    const unsigned long long q = (unsigned long long)(w * 0x1.0p52);
    Qn[v] = q;
    wq += q;
    num += w * E;
    den += w;
  }
  const unsigned long long S = wave_scan_u64(wq, lane);   // Q at the lane's last node
  const unsigned long long Wq = readlane_u64(S, 63);
  num = wave_sum(num);
  den = wave_sum(den);
  o.ebar = num / den;
  // threshold t = floor(u53 * W / 2^53)
  const unsigned long long lo = (unsigned long long)u53 * Wq;
  const unsigned long long hi = __umul64hi((unsigned long long)u53, Wq);
  const unsigned long long t = (hi << 11) | (lo >> 53);
  // inclusive prefix sums Q_v in node order; the first node with Q_v > t lies in the
  // first lane that finds one among its own nodes
  unsigned long long Q = S - wq;
  int vhit = -1;
  unsigned long long qh = 0ull, Qh = 0ull;
  for (int v = v0; v < v1; ++v) {
    const unsigned long long q = Qn[v];
    Q += q;
    if (vhit < 0 && Q > t) {
      vhit = v;
      qh = q;
      Qh = Q;
    }
  }
  const unsigned long long hit = __ballot(vhit >= 0);
  int vstar;
  if (hit == 0ull) {
    // unreachable for finite energies (the minimum-energy node has q = 2^52 > 0);
    // stay put and report a zero margin rather than index outside the graph
    vstar = r;
    o.margin = 0.0;
  } else {
    const int first = __ffsll((long long)hit) - 1;
    vstar = __builtin_amdgcn_readlane(vhit, first);
    const unsigned long long qv = readlane_u64(qh, first), Qv = readlane_u64(Qh, first);
    const unsigned long long d1 = t - (Qv - qv), d2 = Qv - t;
    o.margin = (double)(d1 < d2 ? d1 : d2) / (double)Wq;
  }
  o.vstar = vstar;
  o.e_new = En[vstar];
  return o;
}

// The node rule with generation-probability ratios rho_v = P_gen(T|c_v) / P_gen(T|c_0)
// (App. "Markov chain of graphs of configurations", Eq. eq_det_balance_graph_solution),
// computed by one whole wave: y_v = exp(-(beta (E_v - Emin))) rho_v, w_v = y_v / max y,
// then the fixed-point draw of apply_rule; the node-weighted energy with the weights w.
__device__ __forceinline__ RuleOut apply_rule_ratio(const double* En, const double* rho, unsigned long long* Qn, int M,
                                                    int r, double beta, uint64_t u53, int lane) {
  RuleOut o;
  const int nodes = M + 1;
  const int K = (nodes + 63) >> 6;
  const int v0 = lane * K, v1 = min(v0 + K, nodes);
  double emin = __longlong_as_double(0x7FF0000000000000ll);
  for (int v = v0; v < v1; ++v) emin = En[v] < emin ? En[v] : emin;
  emin = wave_min(emin);
  double ymax = 0.0;
  for (int v = v0; v < v1; ++v) {
    const double y = exp_weight(-(beta * (En[v] - emin))) * rho[v];
    ymax = y > ymax ? y : ymax;
  }
  ymax = wave_max(ymax);
  unsigned long long wq = 0ull;
  double num = 0.0, den = 0.0;
  for (int v = v0; v < v1; ++v) {
    const double E = En[v];
    const double w = (exp_weight(-(beta * (E - emin))) * rho[v]) / ymax;
    const unsigned long long q = (unsigned long long)(w * 0x1.0p52);
    Qn[v] = q;
    wq += q;
    num += w * E;
    den += w;
  }
  const unsigned long long S = wave_scan_u64(wq, lane);
  const unsigned long long Wq = readlane_u64(S, 63);
  num = wave_sum(num);
  den = wave_sum(den);
  o.ebar = num / den;
  const unsigned long long lo = (unsigned long long)u53 * Wq;
  const unsigned long long hi = __umul64hi((unsigned long long)u53, Wq);
  const unsigned long long t = (hi << 11) | (lo >> 53);
  unsigned long long Q = S - wq;
  int vhit = -1;
  unsigned long long qh = 0ull, Qh = 0ull;
  for (int v = v0; v < v1; ++v) {
    const unsigned long long q = Qn[v];
    Q += q;
    if (vhit < 0 && Q > t) {
      vhit = v;
      qh = q;
      Qh = Q;
    }
  }
  const unsigned long long hit = __ballot(vhit >= 0);
  if (hit == 0ull) {
    o.vstar = r;
    o.margin = 0.0;
  } else {
    const int first = __ffsll((long long)hit) - 1;
    o.vstar = __builtin_amdgcn_readlane(vhit, first);
    const unsigned long long qv = readlane_u64(qh, first), Qv = readlane_u64(Qh, first);
    const unsigned long long d1 = t - (Qv - qv), d2 = Qv - t;
    o.margin = (double)(d1 < d2 ? d1 : d2) / (double)Wq;
  }
  o.e_new = En[o.vstar];
  return o;
}

// Per-chain bookkeeping of a selected step (one lane): carried energy e_new,
// node-weighted energy, counters and, with a ring, the step's record.  tau is the
// near-tie threshold of this step.
__device__ __forceinline__ void record_outcome(const RuleOut& o, double e_new, int g, int r, double tau,
                                               uint32_t step, int trace_steps, int total_chains, double* e_cur,
                                               double* e_bar_out, unsigned long long* moves,
                                               unsigned long long* near_ties, double* min_margin, Record* ring) {
  const bool moved = o.vstar != r;
  const bool near = o.margin < tau;
  e_cur[g] = e_new;
  e_bar_out[g] = o.ebar;
  moves[g] += moved ? 1ull : 0ull;
  near_ties[g] += near ? 1ull : 0ull;
  min_margin[g] = o.margin < min_margin[g] ? o.margin : min_margin[g];
  if (trace_steps > 0) {
    Record rec;
    rec.r = r;
    rec.vstar = o.vstar;
    rec.e_cur = e_new;
    rec.e_bar = o.ebar;
    rec.margin = o.margin;
    rec.flags = (near ? 1u : 0u) | (moved ? 2u : 0u);
    rec.step = step;
    ring[(size_t)(step % (uint32_t)trace_steps) * total_chains + g] = rec;
  }
}

// beta of step t under the linear schedule beta0 -> beta1 over `total` steps, in the
// host's operation order: beta0 + (beta1 - beta0) (t / (total - 1)), beta0 if total <= 1.
__device__ __forceinline__ double beta_of(double beta0, double beta1, long long total, uint32_t t) {
  return total <= 1 ? beta0 : beta0 + (beta1 - beta0) * ((double)t / (double)(total - 1));
}

// Node energies of chain c into En (LDS), by the threads t = 0 .. nt-1 of a group: the
// column energies -(scale * sum_p partial[p][col]) (fixed order over p) at their node
// (column m is node m+1, or the hub for column r-1), and the root's entry the carried
// energy.
__device__ __forceinline__ void node_energies(double* En, const double* __restrict__ partial, int P, size_t Bp,
                                              size_t col0, int M, int r, double scale, double ecur, int t, int nt) {
  for (int m = t; m < M; m += nt) {
    const size_t col = col0 + m;
    double acc = 0.0;
    for (int q = 0; q < P; ++q) acc += partial[(size_t)q * Bp + col];
    En[(r >= 1 && m == r - 1) ? 0 : m + 1] = -(scale * acc);
  }
  if (t == 0) En[r] = ecur;
}

// The words of one chain's state that a group of NT threads handles (thread t owns
// words t, t + NT, ...; W <= 256): current spins, this step's base and the next step's
// root column, loaded before the rule so that only the chosen node's column waits for
// it.
template <int NT>
struct ChainWords {
  static constexpr int K = 256 / NT;
  uint32_t s_old[K], b_cur[K], f_next[K];

  // col_next: the next step's root column c*M + r'-1, or < 0 when r' = 0 or there is
  // no next step
  __device__ __forceinline__ void load(const uint32_t* __restrict__ spins_c, const uint32_t* __restrict__ base_c,
                                       const uint32_t* __restrict__ flipsT_next, size_t Bp, long long col_next,
                                       int W, int t) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int w = t + k * NT;
      s_old[k] = b_cur[k] = f_next[k] = 0u;
      if (w < W) {
        s_old[k] = spins_c[w];
        b_cur[k] = base_c[w];
        if (col_next >= 0) f_next[k] = flipsT_next[(size_t)w * Bp + (size_t)col_next];
      }
    }
  }

  // Word k of the state after the move to node vstar: base ^ P(v*) (the base alone
  // for node 0), the old word when v* = r.
  __device__ __forceinline__ uint32_t new_word(const uint32_t* __restrict__ flipsT, size_t Bp, size_t col0,
                                               int vstar, int r, int W, int t, int k) const {
    const int w = t + k * NT;
    if (w >= W || vstar == r) return s_old[k];
    uint32_t x = b_cur[k];
    if (vstar >= 1) x ^= flipsT[(size_t)w * Bp + col0 + (size_t)(vstar - 1)];
    return x;
  }

  // The move (x[k] = new_word(.., k)) and, with next_base, the next step's base = new
  // state ^ P(r').
  __device__ __forceinline__ void store(uint32_t* __restrict__ spins_c, uint32_t* __restrict__ base_next_c,
                                        const uint32_t (&x)[K], bool moved, bool next_base, int W, int t) const {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int w = t + k * NT;
      if (w < W) {
        if (moved) spins_c[w] = x[k];
        if (next_base) base_next_c[w] = x[k] ^ f_next[k];
      }
    }
  }
};

// Sum over 256 threads in a fixed order: each wave's DPP tree, then waves 0..3 in order.
// red4: 4 doubles of LDS.  Every thread gets the result.
__device__ __forceinline__ double block_sum256(double x, double* red4, int tid) {
  x = wave_sum(x);
  if ((tid & 63) == 0) red4[tid >> 6] = x;
  __syncthreads();
  const double t = ((red4[0] + red4[1]) + red4[2]) + red4[3];
  __syncthreads();
  return t;
}

// The exact change of the pair sum U = sum_{i<j} J_ij s_i s_j when the sites of D flip
// (s the old state): the pairs with one site in D change sign, so
//   dU = -2 sum_{i in D} s_i sum_{j not in D} J_ij s_j = -2 cross,
// |D| rows of the symmetric J64 in FP64 (exact integers for +-1 couplings).  This
// returns part (sl, rs) of the cross sum: the columns j outside D in column slice sl of
// kMoveCols, [sl wc, (sl + 1) wc) with wc = ceil(N / kMoveCols), over the listed rows a
// with a % RS == rs.  Called by all 256 threads; dW, sW: the words of D and of the old
// state in LDS; Dl: LDS for |D| site entries (site | sign << 15).  Wave 0 lists the
// sites in word order (lane l takes words 4l .. 4l+3, W <= 256); then the threads form
// R groups of CW (CW a power of two >= wc up to 256, R = 256 / CW): thread t takes
// columns j0 + t % CW, + CW, .. of the slice and the rows rs + RS (t / CW), + RS R, ..,
// eight rows of loads at a time.
constexpr int kMoveCols = 8;

__device__ __forceinline__ double flip_cross(const double* __restrict__ J64, int N, int Np, int W,
                                             const uint32_t* dW, const uint32_t* sW, uint16_t* Dl, int* sh_nd,
                                             double* red4, int tid, int sl, int rs, int RS) {
  const int lane = tid & 63;
  if (tid < 64) {
    uint32_t wd[4];
    unsigned long long cnt = 0ull;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int w = 4 * lane + q;
      wd[q] = w < W ? dW[w] : 0u;
      cnt += (unsigned long long)__popc(wd[q]);
    }
    const unsigned long long incl = wave_scan_u64(cnt, lane);
    int pos = (int)(incl - cnt);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int w = 4 * lane + q;
      uint32_t bits = wd[q];
      while (bits) {
        const int b = __ffs((int)bits) - 1;
        bits &= bits - 1u;
        const int k = b < 16 ? 2 * b : 2 * (b - 16) + 1;   // inverse of site_bit
        const uint32_t neg = (sW[w] >> b) & 1u;
        Dl[pos++] = (uint16_t)((32 * w + k) | (int)(neg << 15));
      }
    }
    if (lane == 63) *sh_nd = (int)incl;
  }
  __syncthreads();
  const int nd = *sh_nd;
  const int wc = (N + kMoveCols - 1) / kMoveCols;
  int CW = 32;
  while (CW < wc && CW < 256) CW <<= 1;
  const int R = (256 / CW) * RS;
  const int j0 = sl * wc, j1 = min(N, j0 + wc), rg = rs + RS * (tid / CW);
  double cross = 0.0;
  for (int j = j0 + tid % CW; j < j1; j += CW) {
    const uint32_t wj = (uint32_t)j >> 5, bj = site_bit((uint32_t)j & 31u);
    if ((dW[wj] >> bj) & 1u) continue;
    const double* __restrict__ col = J64 + j;
    double gsum = 0.0;
    int a = rg;
    for (; a + 7 * R < nd; a += 8 * R) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = col[(size_t)(Dl[a + q * R] & 0x7FFF) * Np];
#pragma unroll
      for (int q = 0; q < 8; ++q) gsum = gsum + ((Dl[a + q * R] >> 15) ? -v[q] : v[q]);
    }
    for (; a < nd; a += R) {
      const double v = col[(size_t)(Dl[a] & 0x7FFF) * Np];
      gsum = gsum + ((Dl[a] >> 15) ? -v : v);
    }
    cross = cross + (((sW[wj] >> bj) & 1u) ? -gsum : gsum);
  }
  return block_sum256(cross, red4, tid);
}

// Part (sl, rs) of the cross sum of every global chain that moved (mflag), from the
// chain's words of D and of its old state (moveD [chains][2 Wmax]: D, then old spins)
// written by the selection.  Block b takes slice sl = b % kMoveCols, q = b / kMoveCols,
// chain chain_off + q / RS and row part rs = q % RS: workgroups go to the 8 XCDs in
// turn, so each XCD reads one column slice of J64 (an eighth of it) and keeps it in
// its own L2.  The part goes to xpart[g][rs kMoveCols + sl].  Dynamic LDS: 8 Wmax +
// 2 Nmax bytes.
__global__ __launch_bounds__(256) void k_move_delta(char* __restrict__ ws, const Inst* __restrict__ insts,
                                                    const int32_t* __restrict__ chain_inst, int chain_off,
                                                    const uint32_t* __restrict__ moveD, int Wmax,
                                                    const int32_t* __restrict__ mflag, double* __restrict__ xpart,
                                                    int RS) {
  extern __shared__ uint32_t mv_lds[];
  __shared__ int sh_nd;
  __shared__ double sh_red[4];
  const int q = (int)(blockIdx.x / kMoveCols), sl = (int)(blockIdx.x % kMoveCols), tid = threadIdx.x;
  const int g = chain_off + q / RS, rs = q % RS;
  if (!mflag[g]) return;
  const Inst& in = insts[chain_inst[g]];
  const int W = in.W;
  uint32_t* dW = mv_lds;
  uint32_t* sW = dW + Wmax;
  const uint32_t* src = moveD + (size_t)g * 2 * Wmax;
  for (int w = tid; w < W; w += 256) {
    dW[w] = src[w];
    sW[w] = src[Wmax + w];
  }
  __syncthreads();
  const double x = flip_cross(ws_at<const double>(ws, in.J64), in.N, in.Np, W, dW, sW,
                              reinterpret_cast<uint16_t*>(sW + Wmax), &sh_nd, sh_red, tid, sl, rs, RS);
  if (tid == 0) xpart[(size_t)g * kMoveCols * RS + (size_t)rs * kMoveCols + sl] = x;
}

// The carried pair sum of every chain that moved at `step` and whose difference is not
// yet added (mflag): U += -2 (sum of its kMoveCols RS parts, in order); E = -(scale U)
// into e_cur and into the step's record; the flag cleared.  With a step clock the step
// is *clk + step.
__global__ void k_move_finish(const Inst* __restrict__ insts, const int32_t* __restrict__ chain_inst, int chain_off,
                              int n, int total_chains, int32_t* __restrict__ mflag,
                              const double* __restrict__ xpart, int RS, double* __restrict__ u_cur,
                              double* __restrict__ e_cur, Record* __restrict__ ring, int trace_steps, uint32_t step,
                              const uint32_t* __restrict__ clk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int g = chain_off + i;
  if (!mflag[g]) return;
  if (clk) step += *clk;
  double cross = 0.0;
  const int P = kMoveCols * RS;
  for (int p = 0; p < P; ++p) cross += xpart[(size_t)g * P + p];
  const double U = u_cur[g] + (-2.0 * cross);
  const double E = -(insts[chain_inst[g]].scale * U);
  u_cur[g] = U;
  e_cur[g] = E;
  mflag[g] = 0;
  if (trace_steps > 0) ring[(size_t)(step % (uint32_t)trace_steps) * total_chains + g].e_cur = E;
}

// One block of 256 threads per chain: node rule (MCMCMC) or Metropolis rate, move,
// record, and (next_base) the base words of step t+1.  beta: the kernel argument;
// per instance from sched ([instances][3]: beta0, beta1, total) when sched is
// non-null; with a step clock (clk non-null, replayed graphs) the step is
// *clk + step and beta that step's value of the schedule (beta0, beta1, total).  The
// chain carries its unscaled pair sum U (u_cur; E = -(scale U)).  Near ties: margin <
// tol + beta tie_coef.
//   1. all threads: the node energies (node_energies; the current node's is
//      -(scale U));
//   2. wave 0: the rule (apply_rule);
//   3. thread w: the new state's word and the next step's base word (ChainWords),
//      loaded before step 1;
//   4. the new U: exact = 0: the chosen column's pair sum as scored; exact = 1: the
//      words of the set D* of flipped sites and of the old state go to moveD and the
//      chain's mflag is set; k_move_delta sums the exact FP64 difference dU(D*) from
//      the rows of D* (spread over many blocks) after this launch, and the next
//      selection (or k_move_finish) adds it, rewriting the carried energy and the
//      record's.  A chain whose flag is still set on entry first adds the previous
//      step's difference;
//   5. thread 0: the bookkeeping and the record.
// Dynamic LDS: 16 (M+1) bytes.
__global__ __launch_bounds__(256) void k_select(
    char* __restrict__ ws, const Inst* __restrict__ insts, const int32_t* __restrict__ chain_inst, int chain_off,
    int total_chains, double* __restrict__ e_cur, double* __restrict__ u_cur, const int32_t* __restrict__ roots_all,
    const int32_t* __restrict__ roots_next_all, Record* __restrict__ ring, unsigned long long* __restrict__ moves,
    unsigned long long* __restrict__ near_ties, double* __restrict__ min_margin, double* __restrict__ e_bar_out,
    int metropolis, double beta, double tol, Key key, uint32_t chain_base, uint32_t step, uint32_t slot,
    uint32_t slot_next, int trace_steps, int next_base, const uint32_t* __restrict__ clk, double beta0,
    double beta1, long long total, const double* __restrict__ sched, int exact, uint32_t* __restrict__ moveD,
    int Wmax, int32_t* __restrict__ mflag, const double* __restrict__ xpart, int move_rs) {
  extern __shared__ double sel_lds[];
  __shared__ int sh_vstar;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = chain_off + blockIdx.x;   // global chain
  if (g >= total_chains) return;
  const int ii = chain_inst[g];
  if (clk) {
    step += *clk;
    beta = beta_of(beta0, beta1, total, step);
  } else if (sched) {
    beta = beta_of(sched[3 * ii], sched[3 * ii + 1], (long long)sched[3 * ii + 2], step);
  }
  const Inst& in = insts[ii];
  const int c = g - in.chain0;            // chain within the instance
  const int M = in.M, W = in.W;
  const size_t Bp = (size_t)in.Bp, col0 = (size_t)c * M;
  uint32_t* __restrict__ spins = ws_at<uint32_t>(ws, in.spins) + (size_t)c * W;
  const uint32_t* __restrict__ flipsT = flips_at(ws, in, slot);
  const uint32_t* __restrict__ base = ws_at<const uint32_t>(ws, in.base[step & 1u]) + (size_t)c * W;
  const uint32_t* __restrict__ flipsT_next = flips_at(ws, in, slot_next);
  uint32_t* __restrict__ base_next = ws_at<uint32_t>(ws, in.base[(step + 1u) & 1u]) + (size_t)c * W;
  const double* __restrict__ partial = ws_at<const double>(ws, in.partial);
  const int nodes = M + 1;
  double* En = sel_lds;                                                              // [nodes]
  unsigned long long* Qn = reinterpret_cast<unsigned long long*>(sel_lds + nodes);   // [nodes]
  const int r = metropolis ? 0 : roots_all[in.chain0 + c];
  double U = u_cur[g];
  if (exact && mflag[g]) {
    // the move of step-1, whose difference k_move_delta has summed and no kernel has
    // added yet: the same sum as k_move_finish's, in the same order
    const int P = kMoveCols * move_rs;
    double cross = 0.0;
    for (int q = 0; q < P; ++q) cross += xpart[(size_t)g * P + q];
    U = U + (-2.0 * cross);
    if (tid == 0) {
      const double E = -(in.scale * U);
      u_cur[g] = U;
      e_cur[g] = E;
      if (trace_steps > 0) ring[(size_t)((step - 1u) % (uint32_t)trace_steps) * total_chains + g].e_cur = E;
    }
  }
  const double ecur = -(in.scale * U);
  long long col_next = -1;
  if (next_base) {
    const int r1 = roots_next_all[in.chain0 + c];
    if (r1 >= 1) col_next = (long long)col0 + (r1 - 1);
  }
  ChainWords<256> cw;
  cw.load(spins, base, flipsT_next, Bp, col_next, W, tid);

  node_energies(En, partial, in.P, Bp, col0, M, r, in.scale, ecur, tid, 256);
  __syncthreads();
  RuleOut o;
  if (wave == 0) {
    const uint4 ub = stream_block(key, kTagSelect, chain_base + (uint32_t)g, step, 0u, 0u);
    o = apply_rule(En, Qn, M, r, ecur, metropolis, beta, u53_of(ub.x, ub.y), lane,
                   in.prior ? ws_at<const double>(ws, in.prior) : nullptr);
    if (lane == 0) sh_vstar = o.vstar;
  }
  __syncthreads();
  const int vstar = sh_vstar;
  const bool moved = vstar != r;
  uint32_t x[ChainWords<256>::K];
  x[0] = cw.new_word(flipsT, Bp, col0, vstar, r, W, tid, 0);
  cw.store(spins, base_next, x, moved, next_base != 0, W, tid);
  double u_new = U;
  if (exact) {
    if (tid == 0) mflag[g] = moved ? 1 : 0;
    if (moved && tid < W) {
      moveD[(size_t)g * 2 * Wmax + tid] = cw.s_old[0] ^ x[0];
      moveD[(size_t)g * 2 * Wmax + Wmax + tid] = cw.s_old[0];
    }
  } else if (moved) {
    if (tid == 0) {
      // the chosen node's column: node v >= 1 is column v-1, the hub (r >= 1) column r-1
      const size_t col = col0 + (size_t)(vstar >= 1 ? vstar - 1 : r - 1);
      double acc = 0.0;
      for (int q = 0; q < in.P; ++q) acc += partial[(size_t)q * Bp + col];
      u_new = acc;
    }
  }
  if (tid == 0) {
    // exact, moved: k_move_finish replaces the energy recorded here
    if (!(exact && moved)) u_cur[g] = u_new;
    record_outcome(o, -(in.scale * u_new), g, r, tol + beta * in.tie_coef, step, trace_steps, total_chains, e_cur,
                   e_bar_out, moves, near_ties, min_margin, ring);
  }
}

// ------------------------------------------------------------------- means trace

// Chain means of the current and node-weighted energies of this step, one block of
// 256 threads, fixed-order tree: trace[slot] = {step, mean e_cur, mean e_bar}.  With a
// step clock the step is *clk + step and the slot step % mean_steps.
__global__ __launch_bounds__(256) void k_chain_means(double* __restrict__ trace, const double* __restrict__ e_cur,
                                                     const double* __restrict__ e_bar, int chains, uint32_t slot,
                                                     uint32_t step, const uint32_t* __restrict__ clk,
                                                     uint32_t mean_steps) {
  if (clk) {
    step += *clk;
    slot = step % mean_steps;
  }
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

// ------------------------------------------------------------------- step clock

// The step clock of replayed graphs: clk = value (add = 0) or clk += value (one thread).
__global__ void k_clock(uint32_t* __restrict__ clk, uint32_t value, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) clk[0] = add ? clk[0] + value : value;
}

}  // namespace mc3
