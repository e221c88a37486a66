// delta.hpp -- the field-update path: energies as differences from the current state.
#pragma once
#include "common.hpp"
#include "select.hpp"

namespace mc3 {

// ------------------------------------------------------------------- field-update path
//
// Energies as differences from the current state (a scorer for small flip sets).
// Per chain the device keeps the unscaled pair sum U = sum_{i<j} J_ij s_i s_j
// (E = -(scale U)) and the local field h_i = sum_j J_ij s_j.  Flipping the sites of a
// set D changes U by
//   dU(D) = -2 sum_{i in D} s_i h_i + 4 sum_{i<j in D} J_ij s_i s_j,
// and h by h_i -= 2 sum_{j in D} J_ij s_j (old spins).  The node v of the star differs
// from the current state (node r) by the path flip set D_v = F_r xor F_v (F_0 = {}):
// F_v for r = 0, F_r for the hub, F_r xor F_v for the other leaves.  With +-1
// couplings U and h stay exact integers, so energies equal the pair sum's.

constexpr int kDeltaMaxK = 16;    // flip-set size limit of the field-update path
constexpr int kDeltaMaxM = 512;   // graph size limit (leaves)
constexpr int kDeltaMaxN = 4096;  // spins (the field lives in LDS)

__host__ __device__ constexpr size_t delta_lds_bytes(int Nmax, int Mmax, int Wmax) {
  return 8 * (size_t)Nmax + 24 * ((size_t)Mmax + 1) + 4 * (size_t)Wmax + 2 * (size_t)kDeltaMaxK * Mmax +
         2 * 256 * 2 * (size_t)kDeltaMaxK + (size_t)Mmax;
}

// h = J s for every chain (one block per global chain; thread i owns rows i, i+256, ..;
// j ascending).
__global__ __launch_bounds__(256) void k_field_init(char* __restrict__ ws, const Inst* __restrict__ insts,
                                                    const int32_t* __restrict__ chain_inst) {
  const int g = blockIdx.x;
  const Inst& in = insts[chain_inst[g]];
  const int c = g - in.chain0;
  const int N = in.N, Np = in.Np, W = in.W;
  const double* __restrict__ J64 = ws_at<const double>(ws, in.J64);
  const uint32_t* s = ws_at<const uint32_t>(ws, in.spins) + (size_t)c * W;
  double* h = ws_at<double>(ws, in.field) + (size_t)c * Np;
  for (int i = threadIdx.x; i < N; i += 256) {
    const double* row = J64 + (size_t)i * Np;
    double acc = 0.0;
    for (int j = 0; j < N; ++j) {
      const double sj = ((s[j >> 5] >> site_bit(j & 31)) & 1u) ? -1.0 : 1.0;
      acc += row[j] * sj;
    }
    h[i] = acc;
  }
}

__device__ __forceinline__ double spin_of(const uint32_t* bits, int i) {
  return ((bits[i >> 5] >> site_bit(i & 31)) & 1u) ? -1.0 : 1.0;
}

// Whether node u (>= 1) is node x or one of its ancestors (breadth-first labels:
// ancestors have smaller labels).
__device__ __forceinline__ bool on_path_up(int u, int x, int arity) {
  while (x > u) x = (x - 1) / arity;
  return x == u;
}

// Toggle site t in the list out[0..n): remove it if present, append it otherwise.
__device__ __forceinline__ void toggle_site(uint16_t* out, int& n, uint16_t t) {
  for (int a = 0; a < n; ++a)
    if (out[a] == t) {
      out[a] = out[n - 1];
      --n;
      return;
    }
  out[n++] = t;
}

// Path flip set D_v of node v (root r) into out[]; returns |D_v|.
// Star (arity >= M): sites of F_v not in F_r (in F_v's order), then sites of F_r not in
// F_v (in F_r's order).  Other trees: the flip sets of the edges on the path from r up
// to the common ancestor, then from v up to it, each site toggled into the list.  The
// host keeps |D_v| <= 2 kDeltaMaxK.
__device__ __forceinline__ int path_set(const uint16_t* sites, const uint8_t* ks, int r, int v, uint16_t* out,
                                        int M, int arity) {
  int n = 0;
  if (arity < M) {
    for (int u = r; u >= 1; u = (u - 1) / arity) {
      if (on_path_up(u, v, arity)) continue;
      for (int a = 0; a < ks[u - 1]; ++a) toggle_site(out, n, sites[(size_t)(u - 1) * kDeltaMaxK + a]);
    }
    for (int u = v; u >= 1; u = (u - 1) / arity) {
      if (on_path_up(u, r, arity)) continue;
      for (int a = 0; a < ks[u - 1]; ++a) toggle_site(out, n, sites[(size_t)(u - 1) * kDeltaMaxK + a]);
    }
    return n;
  }
  const uint16_t* fv = v >= 1 ? sites + (size_t)(v - 1) * kDeltaMaxK : nullptr;
  const uint16_t* fr = r >= 1 ? sites + (size_t)(r - 1) * kDeltaMaxK : nullptr;
  const int kv = v >= 1 ? ks[v - 1] : 0;
  const int kr = r >= 1 ? ks[r - 1] : 0;
  for (int a = 0; a < kv; ++a) {
    bool both = false;
    for (int b = 0; b < kr; ++b) both |= fr[b] == fv[a];
    if (!both) out[n++] = fv[a];
  }
  for (int b = 0; b < kr; ++b) {
    bool both = false;
    for (int a = 0; a < kv; ++a) both |= fv[a] == fr[b];
    if (!both) out[n++] = fr[b];
  }
  return n;
}

// n steps of the whole path for every chain, one block (256 threads) per global
// chain, the chain's state, field and pair sum held in LDS across the steps:
//   1. threads e-1 draw edge e's flip set (k_e, then Floyd's k-of-N on the same words
//      as k_propose, the membership test scanning the list drawn so far); thread 0
//      draws the root;
//   2. thread v (each node v != r) forms D_v and dU(D_v), En[v] = -(scale (U + dU));
//      En[r] = -(scale U);
//   3. wave 0: the rule (apply_rule) and the bookkeeping;
//   4. on a move: h -= 2 J[:, D*] s_D* (rows of J, coalesced), then the spins of D*
//      flip and U += dU(D*).
// beta_t = beta0 + (beta1 - beta0) (t / (total - 1)) as on the host, the schedule of the
// chain's instance from sched ([instances][3]) when it is non-null.  Near ties: margin
// < tol + beta tie_coef.  Per-step chain
// values (e_cur, e_bar) go to vals[t % mean_steps][g] for the means trace.
// Dynamic LDS: delta_lds_bytes(Nmax, Mmax, Wmax).
__global__ __launch_bounds__(256) void k_step_delta(
    char* __restrict__ ws, const Inst* __restrict__ insts, const int32_t* __restrict__ chain_inst,
    int total_chains, int Nmax, int Mmax, int Wmax,
    double* __restrict__ e_cur, double* __restrict__ u_cur, Record* __restrict__ ring,
    unsigned long long* __restrict__ moves, unsigned long long* __restrict__ near_ties,
    double* __restrict__ min_margin, double* __restrict__ e_bar_out, double* __restrict__ vals, int mean_steps,
    int metropolis, double beta0, double beta1, long long total, double tol, Key key, uint32_t chain_base,
    uint32_t step0, int nsteps, int trace_steps, const double* __restrict__ sched) {
  extern __shared__ double dl[];
  __shared__ int sh_r, sh_vstar, sh_nd;
  __shared__ uint16_t dstar[2 * kDeltaMaxK];
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
  const double scale = in.scale;
  const double* __restrict__ J64 = ws_at<const double>(ws, in.J64);
  uint32_t* __restrict__ spins_g = ws_at<uint32_t>(ws, in.spins) + (size_t)c * W;
  double* __restrict__ field_g = ws_at<double>(ws, in.field) + (size_t)c * Np;
  // LDS carve-up
  double* h = dl;                                                               // [Nmax]
  double* En = h + Nmax;                                                        // [Mmax+1]
  double* dU = En + (Mmax + 1);                                                 // [Mmax+1]
  unsigned long long* Qn = reinterpret_cast<unsigned long long*>(dU + (Mmax + 1));  // [Mmax+1]
  uint32_t* sbits = reinterpret_cast<uint32_t*>(Qn + (Mmax + 1));              // [Wmax]
  uint16_t* sites = reinterpret_cast<uint16_t*>(sbits + Wmax);                 // [Mmax][K]
  uint16_t* dbuf = sites + (size_t)Mmax * kDeltaMaxK;                          // [256][2K]
  uint8_t* ks = reinterpret_cast<uint8_t*>(dbuf + 256 * 2 * kDeltaMaxK);       // [Mmax]

  for (int i = tid; i < N; i += 256) h[i] = field_g[i];
  for (int w = tid; w < W; w += 256) sbits[w] = spins_g[w];
  double U = u_cur[g];
  const uint32_t gc = chain_base + (uint32_t)g;
  __syncthreads();

  for (int it = 0; it < nsteps; ++it) {
    const uint32_t step = step0 + (uint32_t)it;
    const double beta = beta_of(beta0, beta1, total, step);
    // 1. root and flip sets
    if (tid == 0)
      sh_r = root_of(key, gc, step, M, metropolis, in.law, in.root_q ? ws_at<const uint64_t>(ws, in.root_q) : nullptr);
    for (int e1 = tid; e1 < M; e1 += 256) {
      const uint32_t e = (uint32_t)e1 + 1u;
      uint16_t* my = sites + (size_t)e1 * kDeltaMaxK;
      uint4 blk = stream_block(key, kTagEdge, gc, step, e, 0u);
      const int k = in.kmin + (int)randint(blk.x, (uint32_t)(in.kmax - in.kmin + 1));
      for (int idx = 0; idx < k; ++idx) {
        const uint32_t n = 1u + (uint32_t)idx;
        if ((n & 3u) == 0u) blk = stream_block(key, kTagEdge, gc, step, e, n >> 2);
        const uint32_t j = (uint32_t)(N - k + idx);
        const uint32_t t = randint(pick(blk, n & 3u), j + 1u);
        bool seen = false;
        for (int q = 0; q < idx; ++q) seen |= my[q] == (uint16_t)t;
        my[idx] = (uint16_t)(seen ? j : t);
      }
      ks[e1] = (uint8_t)k;
    }
    __syncthreads();
    const int r = sh_r;
    // 2. node energies
    for (int v = tid; v <= M; v += 256) {
      if (v == r) continue;
      uint16_t* D = dbuf + (size_t)tid * 2 * kDeltaMaxK;
      const int nd = path_set(sites, ks, r, v, D, M, in.arity);
      double lin = 0.0, pair = 0.0;
      for (int a = 0; a < nd; ++a) {
        const int i = D[a];
        const double si = spin_of(sbits, i);
        lin += si * h[i];
        const double* Ji = J64 + (size_t)i * Np;
        double row = 0.0;
        for (int b = a + 1; b < nd; ++b) row += Ji[D[b]] * spin_of(sbits, D[b]);
        pair += si * row;
      }
      const double d = -2.0 * lin + 4.0 * pair;
      dU[v] = d;
      En[v] = -(scale * (U + d));
    }
    if (tid == 0) En[r] = -(scale * U);
    __syncthreads();
    // 3. the rule
    if (wave == 0) {
      const uint4 ub = stream_block(key, kTagSelect, gc, step, 0u, 0u);
      const RuleOut o = apply_rule(En, Qn, M, r, -(scale * U), metropolis, beta, u53_of(ub.x, ub.y), lane,
                                   in.prior ? ws_at<const double>(ws, in.prior) : nullptr);
      if (lane == 0) {
        sh_vstar = o.vstar;
        record_outcome(o, o.e_new, g, r, tol + beta * in.tie_coef, step, trace_steps, total_chains, e_cur,
                       e_bar_out, moves, near_ties, min_margin, ring);
        if (mean_steps > 0) {
          double* vv = vals + ((size_t)(step % (uint32_t)mean_steps) * total_chains + g) * 2;
          vv[0] = o.e_new;
          vv[1] = o.ebar;
        }
        if (o.vstar != r) sh_nd = path_set(sites, ks, r, o.vstar, dstar, M, in.arity);
      }
    }
    __syncthreads();
    // 4. the move
    const int vstar = sh_vstar;
    if (vstar != r) {
      const int nd = sh_nd;
      for (int i = tid; i < N; i += 256) {
        double x = h[i];
        for (int a = 0; a < nd; ++a) {
          const int j = dstar[a];
          x -= 2.0 * (J64[(size_t)j * Np + i] * spin_of(sbits, j));
        }
        h[i] = x;
      }
      __syncthreads();
      if (tid == 0) {
        for (int a = 0; a < nd; ++a) sbits[dstar[a] >> 5] ^= 1u << site_bit(dstar[a] & 31);
      }
      U += dU[vstar];
      __syncthreads();
    }
  }
  for (int i = tid; i < N; i += 256) field_g[i] = h[i];
  for (int w = tid; w < W; w += 256) spins_g[w] = sbits[w];
  if (tid == 0) u_cur[g] = U;
}

// Chain means of `n` consecutive steps from per-chain values vals[slot][g][2] (slot =
// step % mean_steps): one block per step, the same fixed-order tree as k_chain_means.
__global__ __launch_bounds__(256) void k_chain_means_steps(double* __restrict__ trace,
                                                           const double* __restrict__ vals, int chains,
                                                           int mean_steps, uint32_t step0) {
  __shared__ double red[2][256];
  const uint32_t step = step0 + blockIdx.x;
  const uint32_t slot = step % (uint32_t)mean_steps;
  const double* v = vals + (size_t)slot * chains * 2;
  double a = 0.0, b = 0.0;
  for (int c = threadIdx.x; c < chains; c += 256) {
    a += v[2 * (size_t)c];
    b += v[2 * (size_t)c + 1];
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

}  // namespace mc3

namespace mc3 {

// ------------------------------------------------------------------- field update, any flip-set size
//
// The star with flip sets of any size, energies as FP64 differences: the field of the
// hub h' is formed once per step (r >= 1: h' = h - 2 sum_{j in F_r} s_j J[j, :]), and
// leaf v = hub with F_v flipped has
//   dU_hub(F_v) = -2 sum_{i in F_v} s'_i h'_i + 4 sum_{i<j in F_v} J_ij s'_i s'_j
// (|F_v| field reads and |F_v|(|F_v|-1)/2 coupling gathers); the pair sum of the hub is
// U' = U - sum_{i in F_r} s_i (h_i + h'_i) (the pair term of F_r through the two
// fields).  Flip sets are drawn in the kernel exactly as k_propose draws them (Floyd's
// k-of-N on the edge stream), into one bitset per edge.

__host__ __device__ constexpr size_t delta_star_lds_bytes(int Nmax, int Mmax, int Wmax, int Kmax) {
  return 16 * (size_t)Nmax + 24 * ((size_t)Mmax + 1) + 8 * (size_t)Wmax + 4 * (size_t)Mmax * Wmax +
         2 * 4 * (size_t)Kmax;
}

// The sites of a bitset row (W <= 256 words, stored order) as a list in word order, by
// one whole wave (lane l takes words 4l .. 4l+3); returns the count (every lane).
__device__ __forceinline__ int wave_list_sites(const uint32_t* bits, int W, uint16_t* list, int lane) {
  uint32_t wd[4];
  unsigned long long cnt = 0ull;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int w = 4 * lane + q;
    wd[q] = w < W ? bits[w] : 0u;
    cnt += (unsigned long long)__popc(wd[q]);
  }
  const unsigned long long incl = wave_scan_u64(cnt, lane);
  int pos = (int)(incl - cnt);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t b = wd[q];
    while (b) {
      const int k = __ffs((int)b) - 1;
      b &= b - 1u;
      list[pos++] = (uint16_t)(32 * (4 * lane + q) + (k < 16 ? 2 * k : 2 * (k - 16) + 1));
    }
  }
  return (int)readlane_u64(incl, 63);
}

// dst = src - 2 sum_{a < n} s_{list[a]} J[list[a], :] (the field after flipping the
// listed sites of the state with spins sb), all 256 threads, eight rows of loads at a
// time per column, rows in list order.
__device__ __forceinline__ void field_flip(double* dst, const double* src, const uint16_t* list, int n,
                                           const uint32_t* sb, const double* __restrict__ J64, int N, int Np,
                                           int tid) {
  for (int i = tid; i < N; i += 256) {
    double x = src[i];
    int a = 0;
    for (; a + 8 <= n; a += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = J64[(size_t)list[a + q] * Np + i];
#pragma unroll
      for (int q = 0; q < 8; ++q) x -= 2.0 * (v[q] * spin_of(sb, list[a + q]));
    }
    for (; a < n; ++a) x -= 2.0 * (J64[(size_t)list[a] * Np + i] * spin_of(sb, list[a]));
    dst[i] = x;
  }
}

// n steps of every chain on the star with flip sets of any size, one block (256
// threads) per global chain, the state, its field and the hub's in LDS:
//   1. thread e-1 draws edge e's flip set into its bitset; thread 0 the root;
//   2. r >= 1: the hub's field, spins and pair sum; r = 0: the current ones;
//   3. wave w takes leaves v = 1 + w, 5 + w, ..: lists F_v, lane l sums s'_i h'_i over
//      sites l, l+64, .. and the pairs (a, b > a) of rows a = l, l+64, ..; DPP sums;
//   4. wave 0: the rule (apply_rule) and the bookkeeping;
//   5. the move: to the hub (its field), to leaf v (field_flip of F_v from the hub's).
// Dynamic LDS: delta_star_lds_bytes(Nmax, Mmax, Wmax, Kmax).
__global__ __launch_bounds__(256) void k_step_delta_star(
    char* __restrict__ ws, const Inst* __restrict__ insts, const int32_t* __restrict__ chain_inst,
    int total_chains, int Nmax, int Mmax, int Wmax, int Kmax, double* __restrict__ e_cur, double* __restrict__ u_cur,
    Record* __restrict__ ring, unsigned long long* __restrict__ moves, unsigned long long* __restrict__ near_ties,
    double* __restrict__ min_margin, double* __restrict__ e_bar_out, double* __restrict__ vals, int mean_steps,
    int metropolis, double beta0, double beta1, long long total, double tol, Key key, uint32_t chain_base,
    uint32_t step0, int nsteps, int trace_steps, const double* __restrict__ sched) {
  extern __shared__ double dsl[];
  __shared__ int sh_r, sh_vstar, sh_n;
  __shared__ double red4[4];
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
  const double scale = in.scale;
  const double* __restrict__ J64 = ws_at<const double>(ws, in.J64);
  uint32_t* __restrict__ spins_g = ws_at<uint32_t>(ws, in.spins) + (size_t)c * W;
  double* __restrict__ field_g = ws_at<double>(ws, in.field) + (size_t)c * Np;
  double* h = dsl;                                                                 // [Nmax]
  double* h2 = h + Nmax;                                                           // [Nmax] hub field
  double* En = h2 + Nmax;                                                          // [Mmax+1]
  double* dU = En + (Mmax + 1);                                                    // [Mmax+1]
  unsigned long long* Qn = reinterpret_cast<unsigned long long*>(dU + (Mmax + 1));  // [Mmax+1]
  uint32_t* sb = reinterpret_cast<uint32_t*>(Qn + (Mmax + 1));                    // [Wmax]
  uint32_t* sb2 = sb + Wmax;                                                       // [Wmax]
  uint32_t* fb = sb2 + Wmax;                                                       // [Mmax][Wmax]
  uint16_t* lists = reinterpret_cast<uint16_t*>(fb + (size_t)Mmax * Wmax);        // [4][Kmax]
  uint16_t* my = lists + (size_t)wave * Kmax;

  for (int i = tid; i < N; i += 256) h[i] = field_g[i];
  for (int w = tid; w < W; w += 256) sb[w] = spins_g[w];
  double U = u_cur[g];
  const uint32_t gc = chain_base + (uint32_t)g;
  __syncthreads();

  for (int it = 0; it < nsteps; ++it) {
    const uint32_t step = step0 + (uint32_t)it;
    const double beta = beta_of(beta0, beta1, total, step);
    // 1. root and flip sets
    if (tid == 0)
      sh_r = root_of(key, gc, step, M, metropolis, in.law, in.root_q ? ws_at<const uint64_t>(ws, in.root_q) : nullptr);
    for (int e1 = tid; e1 < M; e1 += 256) {
      uint32_t* set = fb + (size_t)e1 * Wmax;
      for (int w = 0; w < W; ++w) set[w] = 0u;
      const uint32_t e = (uint32_t)e1 + 1u;
      uint4 blk = stream_block(key, kTagEdge, gc, step, e, 0u);
      const int k = in.kmin + (int)randint(blk.x, (uint32_t)(in.kmax - in.kmin + 1));
      for (int idx = 0; idx < k; ++idx) {
        const uint32_t nw = 1u + (uint32_t)idx;
        if ((nw & 3u) == 0u) blk = stream_block(key, kTagEdge, gc, step, e, nw >> 2);
        const uint32_t j = (uint32_t)(N - k + idx);
        const uint32_t t = randint(pick(blk, nw & 3u), j + 1u);
        const bool taken = ((set[t >> 5] >> site_bit(t & 31u)) & 1u) != 0u;
        const uint32_t pos = taken ? j : t;
        set[pos >> 5] |= 1u << site_bit(pos & 31u);
      }
    }
    __syncthreads();
    const int r = sh_r;
    // 2. the hub
    double Uh = U;
    if (r >= 1) {
      const uint32_t* Fr = fb + (size_t)(r - 1) * Wmax;
      if (wave == 0) {
        const int n = wave_list_sites(Fr, W, lists, lane);
        if (lane == 0) sh_n = n;
      }
      __syncthreads();
      const int nr = sh_n;
      field_flip(h2, h, lists, nr, sb, J64, N, Np, tid);
      for (int w = tid; w < W; w += 256) sb2[w] = sb[w] ^ Fr[w];
      __syncthreads();
      double part = 0.0;
      for (int a = tid; a < nr; a += 256) {
        const int i = lists[a];
        part += spin_of(sb, i) * (h[i] + h2[i]);
      }
      Uh = U - block_sum256(part, red4, tid);
    } else {
      for (int i = tid; i < N; i += 256) h2[i] = h[i];
      for (int w = tid; w < W; w += 256) sb2[w] = sb[w];
    }
    __syncthreads();
    // 3. leaves
    for (int v = 1 + wave; v <= M; v += 4) {
      if (v == r) continue;
      const int n = wave_list_sites(fb + (size_t)(v - 1) * Wmax, W, my, lane);
      double lin = 0.0, pair = 0.0;
      for (int a = lane; a < n; a += 64) {
        const int i = my[a];
        const double si = spin_of(sb2, i);
        lin += si * h2[i];
        const double* __restrict__ Ji = J64 + (size_t)i * Np;
        double row = 0.0;
        for (int b = a + 1; b < n; ++b) row += Ji[my[b]] * spin_of(sb2, my[b]);
        pair += si * row;
      }
      lin = wave_sum(lin);
      pair = wave_sum(pair);
      if (lane == 0) {
        const double d = -2.0 * lin + 4.0 * pair;
        dU[v] = d;
        En[v] = -(scale * (Uh + d));
      }
    }
    if (tid == 0) {
      En[0] = -(scale * Uh);
      if (r >= 1) En[r] = -(scale * U);
    }
    __syncthreads();
    // 4. the rule
    if (wave == 0) {
      const uint4 ub = stream_block(key, kTagSelect, gc, step, 0u, 0u);
      const RuleOut o = apply_rule(En, Qn, M, r, -(scale * U), metropolis, beta, u53_of(ub.x, ub.y), lane,
                                   in.prior ? ws_at<const double>(ws, in.prior) : nullptr);
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
    // 5. the move
    const int vstar = sh_vstar;
    if (vstar != r) {
      if (vstar == 0) {
        for (int i = tid; i < N; i += 256) h[i] = h2[i];
        for (int w = tid; w < W; w += 256) sb[w] = sb2[w];
        U = Uh;
      } else {
        const uint32_t* Fv = fb + (size_t)(vstar - 1) * Wmax;
        if (wave == 0) {
          const int n = wave_list_sites(Fv, W, lists, lane);
          if (lane == 0) sh_n = n;
        }
        __syncthreads();
        field_flip(h, h2, lists, sh_n, sb2, J64, N, Np, tid);
        for (int w = tid; w < W; w += 256) sb[w] = sb2[w] ^ Fv[w];
        U = Uh + dU[vstar];
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < N; i += 256) field_g[i] = h[i];
  for (int w = tid; w < W; w += 256) spins_g[w] = sb[w];
  if (tid == 0) u_cur[g] = U;
}

}  // namespace mc3
