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

__device__ RuleOut apply_rule(const double* En, unsigned long long* Qn, int M, int r, double ecur, int metropolis,
                              double beta, uint64_t u53, int lane, const double* __restrict__ prior) {
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
  double emin = __longlong_as_double(0x7FF0000000000000ll);
  for (int v = lane; v < nodes; v += 64) emin = En[v] < emin ? En[v] : emin;
  emin = wave_min(emin);
  double lmax = 0.0;
  if (prior) {
    lmax = __longlong_as_double(0xFFF0000000000000ll);
    for (int v = lane; v < nodes; v += 64) {
      const double l = -(beta * (En[v] - emin)) + prior[v];
      lmax = l > lmax ? l : lmax;
    }
    lmax = wave_max(lmax);
  }
  // fixed-point weights, their total, and the weighted energy
  unsigned long long wq = 0ull;
  double num = 0.0, den = 0.0;
  for (int v = lane; v < nodes; v += 64) {
    const double E = En[v];
    const double w = prior ? exp_weight((-(beta * (E - emin)) + prior[v]) - lmax) : exp_weight(-(beta * (E - emin)));
    const unsigned long long q = (unsigned long long)(w * 0x1.0p52);
    Qn[v] = q;
    wq += q;
    num += w * E;
    den += w;
  }
  const unsigned long long Wq = wave_sum_u64(wq);
  num = wave_sum(num);
  den = wave_sum(den);
  o.ebar = num / den;
  // threshold t = floor(u53 * W / 2^53)
  const unsigned long long lo = (unsigned long long)u53 * Wq;
  const unsigned long long hi = __umul64hi((unsigned long long)u53, Wq);
  const unsigned long long t = (hi << 11) | (lo >> 53);
  // inclusive prefix sums in node order; first node with Q_v > t
  unsigned long long carry = 0ull;
  int vstar = -1;
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
    o.margin = 0.0;
  } else {
    const unsigned long long d1 = t - (Qv - qv), d2 = Qv - t;
    o.margin = (double)(d1 < d2 ? d1 : d2) / (double)Wq;
  }
  o.vstar = vstar;
  o.e_new = En[vstar];
  return o;
}

// Per-chain bookkeeping of a selected step (one lane): carried energy, node-weighted
// energy, counters and, with a ring, the step's record.
__device__ void record_outcome(const RuleOut& o, int g, int r, double tol, uint32_t step, int trace_steps,
                               int total_chains, double* e_cur, double* e_bar_out, unsigned long long* moves,
                               unsigned long long* near_ties, double* min_margin, Record* ring) {
  const bool moved = o.vstar != r;
  const bool near = o.margin < tol;
  e_cur[g] = o.e_new;
  e_bar_out[g] = o.ebar;
  moves[g] += moved ? 1ull : 0ull;
  near_ties[g] += near ? 1ull : 0ull;
  min_margin[g] = o.margin < min_margin[g] ? o.margin : min_margin[g];
  if (trace_steps > 0) {
    Record rec;
    rec.r = r;
    rec.vstar = o.vstar;
    rec.e_cur = o.e_new;
    rec.e_bar = o.ebar;
    rec.margin = o.margin;
    rec.flags = (near ? 1u : 0u) | (moved ? 2u : 0u);
    rec.step = step;
    ring[(size_t)(step % (uint32_t)trace_steps) * total_chains + g] = rec;
  }
}

// One block of 256 threads per chain: node rule (MCMCMC) or Metropolis rate, move,
// record, and (next_base) the base words of step t+1.
//   1. all threads: column energies -(scale * sum_p partial[p][col]) (fixed order over
//      p) into the node-energy array En (LDS) at their node (column m is node m+1,
//      or the hub for column r-1), the root's entry = carried energy;
//   2. wave 0: the rule (apply_rule) and the bookkeeping;
//   3. thread w (one word each, W <= 256): the new state's word, base ^ P(v*) (base
//      alone for node 0), or unchanged; its spins, base and next-root words are loaded
//      before step 1, so only the chosen node's column waits for the rule;
//   4. next_base: base of step t+1 = new state ^ P(r') of that step's root r'.
// Dynamic LDS: 16 (M+1) + 4 W bytes.
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
  const int r = metropolis ? 0 : roots[c];
  const double ecur = e_cur[g];

  // words of this thread (W <= 256): current spins, base, and the next step's root
  // column, loaded now so that only the chosen node's column waits for the rule
  const int w = tid;
  uint32_t s_old = 0u, b_cur = 0u, f_next = 0u;
  if (w < W) {
    s_old = spins[(size_t)c * W + w];
    b_cur = base[(size_t)c * W + w];
    if (next_base) {
      const int r1 = roots_next[c];
      if (r1 >= 1) f_next = flipsT_next[(size_t)w * Bp + (size_t)c * M + (r1 - 1)];
    }
  }

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
    const uint4 ub = stream_block(key, kTagSelect, chain_base + (uint32_t)g, step, 0u, 0u);
    const RuleOut o = apply_rule(En, Qn, M, r, ecur, metropolis, beta, u53_of(ub.x, ub.y), lane,
                                 in.prior ? ws_at<const double>(ws, in.prior) : nullptr);
    if (lane == 0) {
      sh_vstar = o.vstar;
      record_outcome(o, g, r, tol, step, trace_steps, total_chains, e_cur, e_bar_out, moves, near_ties, min_margin,
                     ring);
    }
  }
  __syncthreads();

  // 3. the new state, and 4. the base of the next step
  const int vstar = sh_vstar;
  const bool moved = vstar != r;
  if (w < W) {
    uint32_t x = s_old;
    if (moved) {
      x = b_cur;
      if (vstar >= 1) x ^= flipsT[(size_t)w * Bp + (size_t)c * M + (vstar - 1)];
      spins[(size_t)c * W + w] = x;
    }
    if (next_base) base_next[(size_t)c * W + w] = x ^ f_next;
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
// chain; optionally also the unscaled pair sum U = sum_{i<j} J_ij s_i s_j.  Thread t owns columns j = t, t+256, ...; row i is read coalesced; a
// fixed-order tree combines the threads.
__global__ __launch_bounds__(256) void k_energy_f64(double* __restrict__ out, double* __restrict__ pair_sum,
                                                    char* __restrict__ ws, const Inst* __restrict__ insts,
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
    const double si = ((s[i >> 5] >> site_bit(i & 31)) & 1u) ? -1.0 : 1.0;
    const double* row = J64 + (size_t)i * Np;
    double rs = 0.0;
    for (int j = (int)threadIdx.x; j < N; j += 256) {
      if (j > i) {
        const double sj = ((s[j >> 5] >> site_bit(j & 31)) & 1u) ? -1.0 : 1.0;
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
  if (threadIdx.x == 0) {
    out[g] = -(scale * red[0]);
    if (pair_sum) pair_sum[g] = red[0];
  }
}

}  // namespace mc3
