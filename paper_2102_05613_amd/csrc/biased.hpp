// biased.hpp -- the state-dependent single-site proposal on the star (field-update path).
#pragma once
#include "common.hpp"
#include "delta.hpp"
#include "select.hpp"

namespace mc3 {

// The two-body proposal may depend on the state (Sec. "Problem statement"): here a
// single site i is proposed from state c with probability p_i(c) proportional to
// exp(-alpha dE_i(c)), dE_i(c) = 2 scale s_i h_i(c) the energy change of flipping it.
// In fixed point: a_i = -(alpha ((2 scale) (s_i h_i))), q_i = floor(exp(a_i - max a) 2^52),
// W = sum q; a draw from the 53-bit uniform u53 is min { i : q_0 + .. + q_i > t },
// t = floor(u53 W / 2^53).
//
// The graph is the M-ary star with a uniform root r (App. "General graph populating
// process"): r = 0: the hub is the current state; r >= 1: the current state is leaf r
// and the hub is it with site i_r ~ p(.|current) flipped; every other leaf e is the
// hub with site i_e ~ p(.|hub) flipped (u53 from words 0, 1 of edge e's stream).
// Relative to the hub, the graph's generation probability from leaf v is
// rho_v = p_{i_v}(c_v) / p_{i_v}(hub), taken as (q_{i_v}(c_v) W(hub)) / (q_{i_v}(hub) W(c_v));
// the node rule is apply_rule_ratio.  When the hub cannot generate leaf r
// (q_{i_r}(hub) = 0) no other node can generate the graph and the chain stays.
// These proposals depend on the state, so they are drawn inside the step, never ahead.

constexpr int kBiasedMaxN = 1024;   // spins (two fields and two weight scans in LDS)
constexpr int kBiasedMaxM = 512;    // leaves

__host__ __device__ constexpr size_t biased_lds_bytes(int Nmax, int Mmax, int Wmax) {
  return 32 * (size_t)Nmax + 28 * ((size_t)Mmax + 1) + 8 * (size_t)Wmax;
}

// Fixed-point site weights of the state (field h, spins sb) as inclusive running sums
// Q[0..N) in site order; every thread of the block calls it and gets W = Q[N-1].
// Thread t takes the contiguous sites [t P, t P + P), P = ceil(N / 256); the block's
// maximum and scan go through red (8 doubles) and redq (4 words).
__device__ __forceinline__ unsigned long long site_scan(const double* h, const uint32_t* sb, int N, double alpha,
                                                        double scale2, unsigned long long* Q, double* red,
                                                        unsigned long long* redq, int tid) {
  const int lane = tid & 63, wave = tid >> 6;
  const int P = (N + 255) >> 8;
  const int i0 = tid * P, i1 = min(i0 + P, N);
  double amax = __longlong_as_double(0xFFF0000000000000ll);
  for (int i = i0; i < i1; ++i) {
    const double a = -(alpha * (scale2 * (spin_of(sb, i) * h[i])));
    amax = a > amax ? a : amax;
  }
  amax = wave_max(amax);
  if (lane == 0) red[wave] = amax;
  __syncthreads();
  amax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  unsigned long long part = 0ull;
  for (int i = i0; i < i1; ++i) {
    const double a = -(alpha * (scale2 * (spin_of(sb, i) * h[i])));
    const unsigned long long q = (unsigned long long)(exp_weight(a - amax) * 0x1.0p52);
    part += q;
    Q[i] = q;
  }
  const unsigned long long incl = wave_scan_u64(part, lane);
  if (lane == 63) redq[wave] = incl;
  __syncthreads();
  unsigned long long base = incl - part;
  for (int w = 0; w < wave; ++w) base += redq[w];
  for (int i = i0; i < i1; ++i) {
    base += Q[i];
    Q[i] = base;
  }
  const unsigned long long W = ((redq[0] + redq[1]) + redq[2]) + redq[3];
  __syncthreads();
  return W;
}

// The first site whose running sum exceeds floor(u53 W / 2^53).
__device__ __forceinline__ int draw_site(const unsigned long long* Q, int N, unsigned long long W, uint64_t u53) {
  const unsigned long long lo = (unsigned long long)u53 * W, hi = __umul64hi((unsigned long long)u53, W);
  const unsigned long long t = (hi << 11) | (lo >> 53);
  int a = 0, b = N - 1;
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (Q[mid] > t)
      b = mid;
    else
      a = mid + 1;
  }
  return a;
}

__device__ __forceinline__ unsigned long long weight_at(const unsigned long long* Q, int i) {
  return Q[i] - (i ? Q[i - 1] : 0ull);
}

// n steps of every chain with the biased single-site proposal, one block (256
// threads) per global chain, the state, field and pair sum held in LDS:
//   1. thread 0 draws the root;
//   2. r >= 1: the current state's weights (site_scan), i_r, the hub's field
//      h' = h - 2 J[i_r, :] s_{i_r} and pair sum U' = U - 2 s_{i_r} h_{i_r};
//   3. the hub's weights, the other leaves' sites (thread per leaf);
//   4. energies: hub -(scale U'), leaf v -(scale (U' - 2 s'_{i_v} h'_{i_v})), the current
//      state's the carried -(scale U);
//   5. rho per leaf: one wave per leaf v forms the weights of c_v (field
//      h' - 2 J[i_v, :] s'_{i_v}) for W(c_v) and q_{i_v}(c_v) (leaf r reuses step 2's);
//   6. wave 0: apply_rule_ratio; thread 0: bookkeeping;
//   7. the move (field, spins, pair sum).
// Dynamic LDS: biased_lds_bytes(Nmax, Mmax, Wmax).
__global__ __launch_bounds__(256) void k_step_biased(
    char* __restrict__ ws, const Inst* __restrict__ insts, const int32_t* __restrict__ chain_inst,
    int total_chains, int Nmax, int Mmax, int Wmax, double* __restrict__ e_cur, double* __restrict__ u_cur,
    Record* __restrict__ ring, unsigned long long* __restrict__ moves, unsigned long long* __restrict__ near_ties,
    double* __restrict__ min_margin, double* __restrict__ e_bar_out, double* __restrict__ vals, int mean_steps,
    double alpha, double beta0, double beta1, long long total, double tol, Key key, uint32_t chain_base,
    uint32_t step0, int nsteps, int trace_steps, const double* __restrict__ sched) {
  extern __shared__ double bl[];
  __shared__ int sh_r, sh_vstar;
  __shared__ unsigned long long sh_W[2];
  __shared__ double red[8];
  __shared__ unsigned long long redq[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x;
  const int ii = chain_inst[g];
  const Inst& in = insts[ii];
  if (sched) {
    beta0 = sched[3 * ii];
    beta1 = sched[3 * ii + 1];
    total = (long long)sched[3 * ii + 2];
  }
  const int c = g - in.chain0;
  const int N = in.N, Np = in.Np, W = in.W, M = in.M;
  const double scale = in.scale, scale2 = 2.0 * in.scale;
  const double* __restrict__ J64 = ws_at<const double>(ws, in.J64);
  uint32_t* __restrict__ spins_g = ws_at<uint32_t>(ws, in.spins) + (size_t)c * W;
  double* __restrict__ field_g = ws_at<double>(ws, in.field) + (size_t)c * Np;
  // LDS carve-up
  double* h = bl;                                                                  // [Nmax]
  double* h2 = h + Nmax;                                                           // [Nmax] hub field
  unsigned long long* Qc = reinterpret_cast<unsigned long long*>(h2 + Nmax);       // [Nmax]
  unsigned long long* Qh = Qc + Nmax;                                              // [Nmax]
  double* En = reinterpret_cast<double*>(Qh + Nmax);                               // [Mmax+1]
  double* rho = En + (Mmax + 1);                                                   // [Mmax+1]
  unsigned long long* Qn = reinterpret_cast<unsigned long long*>(rho + (Mmax + 1));  // [Mmax+1]
  int32_t* site = reinterpret_cast<int32_t*>(Qn + (Mmax + 1));                     // [Mmax+1]
  uint32_t* sb = reinterpret_cast<uint32_t*>(site + (Mmax + 1));                  // [Wmax]
  uint32_t* sb2 = sb + Wmax;                                                       // [Wmax] hub spins

  for (int i = tid; i < N; i += 256) h[i] = field_g[i];
  for (int w = tid; w < W; w += 256) sb[w] = spins_g[w];
  double U = u_cur[g];
  const uint32_t gc = chain_base + (uint32_t)g;
  __syncthreads();

  for (int it = 0; it < nsteps; ++it) {
    const uint32_t step = step0 + (uint32_t)it;
    const double beta = beta_of(beta0, beta1, total, step);
    if (tid == 0) sh_r = root_of(key, gc, step, M, 0, 0, nullptr);
    __syncthreads();
    const int r = sh_r;
    // 2. the hub
    double Uh = U;
    if (r >= 1) {
      const unsigned long long Wc = site_scan(h, sb, N, alpha, scale2, Qc, red, redq, tid);
      if (tid == 0) {
        const uint4 eb = stream_block(key, kTagEdge, gc, step, (uint32_t)r, 0u);
        site[r] = draw_site(Qc, N, Wc, u53_of(eb.x, eb.y));
        sh_W[0] = Wc;
      }
      __syncthreads();
      const int ir = site[r];
      const double sr = spin_of(sb, ir);
      for (int j = tid; j < N; j += 256) h2[j] = h[j] - 2.0 * (J64[(size_t)ir * Np + j] * sr);
      for (int w = tid; w < W; w += 256) sb2[w] = sb[w] ^ (w == (ir >> 5) ? 1u << site_bit(ir & 31) : 0u);
      Uh = U + (-2.0 * (sr * h[ir]));
    } else {
      for (int j = tid; j < N; j += 256) h2[j] = h[j];
      for (int w = tid; w < W; w += 256) sb2[w] = sb[w];
    }
    __syncthreads();
    // 3. the hub's weights and the leaves' sites
    const unsigned long long Wh = site_scan(h2, sb2, N, alpha, scale2, Qh, red, redq, tid);
    for (int e = tid + 1; e <= M; e += 256) {
      if (e == r) continue;
      const uint4 eb = stream_block(key, kTagEdge, gc, step, (uint32_t)e, 0u);
      site[e] = draw_site(Qh, N, Wh, u53_of(eb.x, eb.y));
    }
    __syncthreads();
    // 4. energies
    for (int v = tid; v <= M; v += 256) {
      if (v == 0)
        En[0] = -(scale * Uh);
      else if (v == r)
        En[v] = -(scale * U);
      else {
        const int i = site[v];
        En[v] = -(scale * (Uh + (-2.0 * (spin_of(sb2, i) * h2[i]))));
      }
    }
    // 5. generation-probability ratios
    if (tid == 0) rho[0] = 1.0;
    for (int v = 1 + wave; v <= M; v += 4) {
      const int iv = site[v];
      unsigned long long qv, Wv;
      if (v == r) {
        qv = weight_at(Qc, iv);
        Wv = sh_W[0];
      } else {
        // weights of c_v = hub with site iv flipped: field h' - 2 J[iv, :] s'_iv
        const double siv = spin_of(sb2, iv);
        const double* __restrict__ Jr = J64 + (size_t)iv * Np;
        double amax = __longlong_as_double(0xFFF0000000000000ll);
        for (int j = lane; j < N; j += 64) {
          const double hj = h2[j] - 2.0 * (Jr[j] * siv);
          const double sj = j == iv ? -spin_of(sb2, j) : spin_of(sb2, j);
          const double a = -(alpha * (scale2 * (sj * hj)));
          amax = a > amax ? a : amax;
        }
        amax = wave_max(amax);
        unsigned long long part = 0ull, qi = 0ull;
        for (int j = lane; j < N; j += 64) {
          const double hj = h2[j] - 2.0 * (Jr[j] * siv);
          const double sj = j == iv ? -spin_of(sb2, j) : spin_of(sb2, j);
          const double a = -(alpha * (scale2 * (sj * hj)));
          const unsigned long long q = (unsigned long long)(exp_weight(a - amax) * 0x1.0p52);
          part += q;
          if (j == iv) qi = q;
        }
        Wv = readlane_u64(wave_scan_u64(part, lane), 63);
        qv = readlane_u64(qi, iv & 63);
      }
      if (lane == 0) rho[v] = ((double)qv * (double)Wh) / ((double)weight_at(Qh, iv) * (double)Wv);
    }
    __syncthreads();
    // 6. the rule
    if (wave == 0) {
      RuleOut o;
      if (r >= 1 && weight_at(Qh, site[r]) == 0ull) {
        o.vstar = r;
        o.e_new = En[r];
        o.ebar = En[r];
        o.margin = __longlong_as_double(0x7FF0000000000000ll);
      } else {
        const uint4 ub = stream_block(key, kTagSelect, gc, step, 0u, 0u);
        o = apply_rule_ratio(En, rho, Qn, M, r, beta, u53_of(ub.x, ub.y), lane);
      }
      if (lane == 0) {
        sh_vstar = o.vstar;
        record_outcome(o, o.e_new, g, r, tol + beta * in.tie_coef, step, trace_steps, total_chains, e_cur,
                       e_bar_out, moves, near_ties, min_margin, ring);
        if (mean_steps > 0) {
          double* vv = vals + ((size_t)(step % (uint32_t)mean_steps) * total_chains + g) * 2;
          vv[0] = o.e_new;
          vv[1] = o.ebar;
        }
      }
    }
    __syncthreads();
    // 7. the move
    const int vstar = sh_vstar;
    if (vstar != r) {
      if (vstar == 0) {
        for (int j = tid; j < N; j += 256) h[j] = h2[j];
        for (int w = tid; w < W; w += 256) sb[w] = sb2[w];
        U = Uh;
      } else {
        const int i = site[vstar];
        const double si = spin_of(sb2, i);
        const double* __restrict__ Jr = J64 + (size_t)i * Np;
        U = Uh + (-2.0 * (si * h2[i]));
        for (int j = tid; j < N; j += 256) h[j] = h2[j] - 2.0 * (Jr[j] * si);
        for (int w = tid; w < W; w += 256) sb[w] = sb2[w] ^ (w == (i >> 5) ? 1u << site_bit(i & 31) : 0u);
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < N; i += 256) field_g[i] = h[i];
  for (int w = tid; w < W; w += 256) spins_g[w] = sb[w];
  if (tid == 0) u_cur[g] = U;
}

}  // namespace mc3
