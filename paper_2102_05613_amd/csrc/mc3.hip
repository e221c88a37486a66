// mc3.hip -- C ABI of the MI355X MCMCMC hot path for the SK spin glass.
// The declarations and their contracts are in include/mc3.h.
//
// A context holds a batch of SK instances (a single-instance context is a batch of
// one).  Every kernel reads its instance from a device table, so one launch covers
// the whole batch: propose over a table of (instance, first edge) blocks, score over
// a table of (instance, row-block pair, column tile) work units, select over the
// global chain range.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mc3.h"
#include "kernels.hpp"

namespace {

constexpr size_t kAlign = 256;
constexpr int kColPad = 512;     // candidate columns of an instance are padded to this
constexpr int kTileF64 = 128;    // columns per FP64-scoring unit
constexpr int kClasses = 3;      // split-scoring tile widths: 128, 256, 512 columns (2, 4, 8 waves)
constexpr int kMoveRowsMax = 8;  // row parts per chain of the exact energy update, at most
constexpr int kMaxAhead = 16;    // steps of flip sets drawn per proposal launch, at most
constexpr size_t kFlipBudget = size_t(512) << 20;  // bytes of flip-set ring, about

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

// The workspace of contexts made by mc3_create_noalloc: a fixed device array, one copy
// per GPU the library runs on, held until the process ends.  Host code never passes
// this name to a kernel (on the host it is only a stand-in for the symbol): it uses the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[MC3_NOALLOC_BYTES];

namespace {

// Row parts of the exact energy update: enough blocks (about 2048) for a few chains.
int move_row_parts(int total_chains) {
  return std::max(1, std::min(kMoveRowsMax, 256 / std::max(1, total_chains)));
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};     // the array's device address, per device
bool g_scratch_busy[kMaxDevices] = {};     // a live context holds that device's array

// Reserve the current device's array: its address (looked up once per device, with the
// device current) in *ptr.  MC3_E_STATE if a context already holds it.
mc3_status reserve_scratch(int dev, void** ptr) {
  if (dev < 0 || dev >= kMaxDevices) return MC3_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_busy[dev]) return MC3_E_STATE;
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return MC3_E_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  g_scratch_busy[dev] = true;
  *ptr = g_scratch_ptr[dev];
  return MC3_OK;
}

void release_scratch(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev >= 0 && dev < kMaxDevices) g_scratch_busy[dev] = false;
}

struct InstH {
  mc3_instance_desc desc;
  int arity = 1;                                       // resolved: parent of v is (v-1)/arity
  size_t prior = 0;                                    // log-prior table (line and table laws), 0 = none
  size_t root_q = 0;                                   // cumulative fixed-point root weights (table law)
  int Np, W, Wn, B, Bp, NB, P, chain0, col0;
  size_t J64, Jpack, flips, base[2], partial, spins;  // byte offsets into the workspace
  size_t flip_slot;                                    // bytes of one step's flip sets
  size_t field = 0;                                    // [chains][Np] FP64 fields (field-update path)
  size_t upart = 0;                                    // [Np/16][chains] FP64 recompute partial sums
  double scale = 1.0;
  double tie_coef = 0.0;                               // near-tie threshold per unit of beta
  bool have_J = false;
  int cls = 0;                         // scoring tile class (split: 64 << cls ... columns)
  int unit_off = 0, unit_grid = 0;     // this instance's own unit table (per-instance launches)
  int pblock_off = 0, pblock_cnt = 0;  // its proposal blocks
};

struct Plan {
  std::vector<InstH> inst;
  bool delta = false;   // field-update scorer (else the matrix-core pair sum)
  bool delta_star = false;   // ... the kernel for stars with flip sets of any size
  int Kmax = 0;
  size_t delta_lds = 0;
  int total_chains = 0, total_cols = 0, Wmax = 0, Wn_max = 0, Mmax = 0;
  int prop_T = 256, prop_stride = 1, prop_rows = 1;
  int ahead = 1;    // steps proposed per launch in mc3_step_n
  int nslots = 2;   // flip-set and root ring slots (ahead + 1)
  std::vector<mc3::Unit> units_global[kClasses], units_local;
  std::vector<mc3::PBlock> pblocks;
  std::vector<mc3::RecUnit> rec_units;   // the FP64 recompute's units, every instance
  std::vector<int32_t> chain_inst;
  size_t insts = 0, chain_inst_off = 0, units_global_off[kClasses] = {0, 0, 0}, units_local_off = 0, pblocks_off = 0,
         rec_units_off = 0;
  size_t sched = 0;   // [instances][3] per-instance beta schedules (beta0, beta1, total)
  size_t drift_ev = 0;   // [chains] drift events of the periodic recompute
  size_t moveD = 0, mflag = 0, xpart = 0;   // the exact energy update's per-chain move buffers
  size_t clock = 0;   // the step clock of replayed graphs (one uint32)
  size_t e_cur = 0, e_bar = 0, roots = 0, candT = 0, ring = 0, means = 0, moves = 0, near = 0, minm = 0, drift = 0,
         u_cur = 0, vals = 0, total = 0;
};

const char* validate_instance(const mc3_instance_desc& d, int rule) {
  if (d.N < 2 || d.N > 8192) return "N must be in [2, 8192]";
  if (d.M < 1 || d.M > 4000) return "M must be in [1, 4000]";
  if (d.chains < 1) return "chains must be >= 1";
  if ((long long)d.chains * d.M > (1ll << 24)) return "chains * M must be <= 2^24";
  if (d.kmin < 1 || d.kmax < d.kmin || d.kmax > d.N) return "need 1 <= kmin <= kmax <= N";
  if (rule == MC3_RULE_METROPOLIS && d.M != 1) return "rule METROPOLIS requires M == 1";
  return nullptr;
}

// The table law in fixed point: S = sum of g in node order, q_v = floor(g_v / S * 2^52),
// Qcum[v] = q_0 + .. + q_v.  False for a negative or non-finite weight or a zero total.
bool root_table(const double* g, int M, std::vector<uint64_t>* Qcum) {
  double S = 0.0;
  for (int v = 0; v <= M; ++v) {
    if (!(g[v] >= 0.0) || g[v] == HUGE_VAL) return false;
    S += g[v];
  }
  if (!(S > 0.0) || S == HUGE_VAL) return false;
  uint64_t acc = 0;
  if (Qcum) Qcum->resize(M + 1);
  for (int v = 0; v <= M; ++v) {
    acc += (uint64_t)std::floor(g[v] / S * 0x1.0p52);
    if (Qcum) (*Qcum)[v] = acc;
  }
  return acc > 0;
}

const char* validate_batch(const mc3_batch_config* c) {
  if (!c) return "config is NULL";
  if (c->n_instances < 1 || c->n_instances > (1 << 20)) return "n_instances must be in [1, 2^20]";
  if (!c->instances) return "instances is NULL";
  if (c->precision != MC3_FP64 && c->precision != MC3_SPLIT_BF16) return "unknown precision";
  if (c->rule != MC3_RULE_MCMCMC && c->rule != MC3_RULE_METROPOLIS) return "unknown rule";
  if (c->scorer != MC3_SCORER_GEMM && c->scorer != MC3_SCORER_DELTA && c->scorer != MC3_SCORER_AUTO)
    return "unknown scorer";
  if (c->arity < 0) return "arity must be >= 0";
  if (c->law != MC3_LAW_UNIFORM && c->law != MC3_LAW_LINE && c->law != MC3_LAW_TABLE && c->law != MC3_LAW_BIASED)
    return "unknown graph law";
  if (c->law == MC3_LAW_BIASED) {
    if (c->rule != MC3_RULE_MCMCMC) return "the biased proposal needs rule MCMCMC";
    if (c->scorer == MC3_SCORER_GEMM) return "the biased proposal runs on the field-update scorer";
    if (!std::isfinite(c->bias)) return "bias must be finite";
  }
  if (c->law == MC3_LAW_TABLE && !c->law_table) return "law TABLE needs law_table";
  if (c->trace_steps < 0) return "trace_steps must be >= 0";
  if (c->mean_steps < 0) return "mean_steps must be >= 0";
  if (c->tile_cols != 0 && c->tile_cols != 128 && c->tile_cols != 256 && c->tile_cols != 512)
    return "tile_cols must be 0, 128, 256 or 512";
  if (!(c->near_tie_tol == c->near_tie_tol)) return "near_tie_tol is NaN";
  if (c->recompute_every < 0) return "recompute_every must be >= 0";
  if (c->energy_update != MC3_ENERGY_EXACT && c->energy_update != MC3_ENERGY_SCORED) return "unknown energy_update";
  if (!(c->drift_tol == c->drift_tol)) return "drift_tol is NaN";
  long long chains = 0, cols = 0;
  size_t table_at = 0;
  for (int i = 0; i < c->n_instances; ++i) {
    if (const char* e = validate_instance(c->instances[i], c->rule)) return e;
    const int M = c->instances[i].M;
    const int a = (c->arity == 0 || c->arity > M) ? M : c->arity;
    if (c->law == MC3_LAW_LINE && a != 1) return "the line law needs arity 1";
    if (c->law == MC3_LAW_BIASED && (a != M || c->instances[i].kmin != 1 || c->instances[i].kmax != 1))
      return "the biased proposal needs the star and single-site edges (kmin = kmax = 1)";
    if (c->law == MC3_LAW_TABLE && !root_table(c->law_table + table_at, M, nullptr))
      return "law_table: weights must be finite and >= 0 with a positive fixed-point total per instance";
    table_at += M + 1;
    chains += c->instances[i].chains;
    cols += (long long)c->instances[i].chains * c->instances[i].M;
  }
  if (chains + c->chain_base > (1ll << 28)) return "chain_base + total chains must be <= 2^28";
  if (cols > (1ll << 31) - 1) return "total candidate columns must be < 2^31";
  if (chains * (long long)c->trace_steps > (1ll << 31)) return "total chains * trace_steps must be <= 2^31";
  return nullptr;
}

int resolved_arity(const mc3_batch_config& c, int M) { return (c.arity == 0 || c.arity > M) ? M : c.arity; }

// Longest path between two nodes of the tree on M+1 nodes with the given arity, in
// edges: M for a line, otherwise twice the depth of node M (the deepest label).
int longest_path(int M, int arity) {
  if (arity == 1) return M;
  int depth = 0;
  for (int v = M; v >= 1; v = (v - 1) / arity) ++depth;
  return 2 * depth;
}

// Whether the field-update scorer can run this batch (its limits), and its LDS bytes.
// path_limit bounds kmax times the longest path (the size of a path flip set).
bool delta_fits(const mc3_batch_config& c, size_t* lds, int path_limit) {
  int Nmax = 0, Mmax = 0, Wmax = 0;
  for (int i = 0; i < c.n_instances; ++i) {
    const mc3_instance_desc& d = c.instances[i];
    if (d.kmax > mc3::kDeltaMaxK || d.M > mc3::kDeltaMaxM || d.N > mc3::kDeltaMaxN) return false;
    const int path = longest_path(d.M, resolved_arity(c, d.M));
    if ((long long)d.kmax * path > path_limit) return false;
    Nmax = std::max(Nmax, d.N);
    Mmax = std::max(Mmax, d.M);
    Wmax = std::max(Wmax, (d.N + mc3::kRowBlock - 1) / mc3::kRowBlock * mc3::kRowBlock / 32);
  }
  *lds = mc3::delta_lds_bytes(Nmax, Mmax, Wmax);
  return *lds <= 65536;
}

// LDS a workgroup may hold on gfx950 (160 KiB; kernels that take more than 64 KiB of
// dynamic LDS raise their limit with hipFuncSetAttribute before the launch).
constexpr size_t kLdsPerBlock = 160u << 10;

// The field-update scorer for stars with flip sets of any size (k_step_delta_star):
// whether its LDS fits, and how much.
bool delta_star_fits(const mc3_batch_config& c, size_t* lds) {
  int Nmax = 0, Mmax = 0, Wmax = 0, Kmax = 0;
  for (int i = 0; i < c.n_instances; ++i) {
    const mc3_instance_desc& d = c.instances[i];
    if (resolved_arity(c, d.M) != d.M) return false;
    Nmax = std::max(Nmax, d.N);
    Mmax = std::max(Mmax, d.M);
    Kmax = std::max(Kmax, d.kmax);
    Wmax = std::max(Wmax, (d.N + mc3::kRowBlock - 1) / mc3::kRowBlock * mc3::kRowBlock / 32);
  }
  *lds = mc3::delta_star_lds_bytes(Nmax, Mmax, Wmax, Kmax);
  return *lds <= kLdsPerBlock;
}

// Resolve the scorer: 1 = field update, 2 = field update for stars with flip sets of any
// size, 0 = pair sum, -1 = field update requested but outside both kernels' limits.
int resolve_delta(const mc3_batch_config& c, size_t* lds) {
  if (c.law == MC3_LAW_BIASED) {   // its own persistent kernel (field update, state-dependent draws)
    int Nmax = 0, Mmax = 0, Wmax = 0;
    for (int i = 0; i < c.n_instances; ++i) {
      const mc3_instance_desc& d = c.instances[i];
      if (d.N > mc3::kBiasedMaxN || d.M > mc3::kBiasedMaxM) return -1;
      Nmax = std::max(Nmax, d.N);
      Mmax = std::max(Mmax, d.M);
      Wmax = std::max(Wmax, (d.N + mc3::kRowBlock - 1) / mc3::kRowBlock * mc3::kRowBlock / 32);
    }
    *lds = mc3::biased_lds_bytes(Nmax, Mmax, Wmax);
    return *lds <= 65536 ? 1 : -1;
  }
  if (c.scorer == MC3_SCORER_GEMM) return 0;
  if (c.scorer == MC3_SCORER_DELTA) {
    if (delta_fits(c, lds, 2 * mc3::kDeltaMaxK)) return 1;
    return delta_star_fits(c, lds) ? 2 : -1;
  }
  return delta_fits(c, lds, 16) ? 1 : 0;
}

// Tile class of an instance's split scoring: 512-column tiles (8 waves share each A
// tile, half the A copies per MFMA of 4 waves) from 2048 columns up, 128-column tiles
// (2 waves) for at most 128 columns, 256 otherwise.
int split_class(int B) { return B >= 2048 ? 2 : (B > 128 ? 1 : 0); }
int class_waves(int cls) { return 2 << cls; }
int tile_class(int tile_cols) { return tile_cols == 512 ? 2 : (tile_cols == 256 ? 1 : 0); }

// Cost of a scoring unit in 128x128 K blocks: the pair (p, NB-1-p) spans NB+1 blocks
// of the upper triangle, the self-paired middle block row NB-p.
int unit_cost(int NB, int p) { return p == NB - 1 - p ? NB - p : NB + 1; }

// The batch plan: dimensions, tables and the workspace layout.
Plan make_plan(const mc3_batch_config& cfg) {
  Plan pl;
  const int n = cfg.n_instances;
  const int scorer = resolve_delta(cfg, &pl.delta_lds);
  pl.delta = scorer >= 1;
  pl.delta_star = scorer == 2;
  for (int i = 0; i < n; ++i) pl.Kmax = std::max(pl.Kmax, cfg.instances[i].kmax);
  pl.inst.resize(n);
  for (int i = 0; i < n; ++i) {
    InstH& h = pl.inst[i];
    h.desc = cfg.instances[i];
    const mc3_instance_desc& d = h.desc;
    h.Np = (d.N + mc3::kRowBlock - 1) / mc3::kRowBlock * mc3::kRowBlock;
    h.W = h.Np / 32;
    h.Wn = (d.N + 31) / 32;
    h.B = d.chains * d.M;
    h.Bp = (h.B + kColPad - 1) / kColPad * kColPad;
    h.NB = h.Np / mc3::kRowBlock;
    h.P = (h.NB + 1) / 2;
    h.arity = resolved_arity(cfg, d.M);
    h.chain0 = pl.total_chains;
    h.col0 = pl.total_cols;
    pl.total_chains += d.chains;
    pl.total_cols += h.B;
    pl.Wmax = std::max(pl.Wmax, h.W);
    pl.Wn_max = std::max(pl.Wn_max, h.Wn);
    pl.Mmax = std::max(pl.Mmax, d.M);
  }
  // flip-set ring: `ahead` steps are proposed at once; one more slot holds the step
  // being selected while the next group is written
  size_t slot_bytes = 0;
  for (const InstH& h : pl.inst) slot_bytes += (size_t)h.W * h.Bp * 4;
  pl.ahead = (int)std::max<size_t>(1, std::min<size_t>(kMaxAhead, kFlipBudget / slot_bytes));
  pl.nslots = pl.ahead + 1;
  // proposal blocks: one LDS bitset per thread (two when paths are longer than one
  // edge) within 64 KiB, row stride W+1 where 64 threads fit; 64 to 256 threads in
  // steps of 64, or 32 when two rows of the widest bitsets (W = 256) leave no room
  // for 64
  pl.prop_rows = 1;
  for (const InstH& h : pl.inst)
    if (h.arity < h.desc.M) pl.prop_rows = 2;
  pl.prop_stride = pl.Wmax + 1;
  int T = (int)(65536 / ((size_t)pl.prop_rows * pl.prop_stride * 4));
  if (T < 64) {
    pl.prop_stride = pl.Wmax;
    T = (int)(65536 / ((size_t)pl.prop_rows * pl.prop_stride * 4));
  }
  T = std::min(T, 256);
  pl.prop_T = T >= 64 ? T / 64 * 64 : 32;
  for (int i = 0; i < n; ++i) {
    InstH& h = pl.inst[i];
    const long long edges = (long long)h.desc.chains * h.desc.M;
    h.pblock_off = (int)pl.pblocks.size();
    if (h.arity < h.desc.M && h.desc.M <= pl.prop_T) {
      // whole chains per block: the path sets are formed inside the block
      const int cpb = pl.prop_T / h.desc.M;
      for (int c0 = 0; c0 < h.desc.chains; c0 += cpb)
        pl.pblocks.push_back(mc3::PBlock{i, (int32_t)((long long)c0 * h.desc.M),
                                         std::min(cpb, h.desc.chains - c0) * h.desc.M, 0});
    } else {
      for (long long e0 = 0; e0 < edges; e0 += pl.prop_T)
        pl.pblocks.push_back(mc3::PBlock{i, (int32_t)e0, (int32_t)std::min<long long>(pl.prop_T, edges - e0), 0});
    }
    h.pblock_cnt = (int)pl.pblocks.size() - h.pblock_off;
    for (int c = 0; c < h.desc.chains; ++c) pl.chain_inst.push_back(i);
    for (int ct = 0; ct < (h.desc.chains + 63) / 64; ++ct)
      for (int rt = 0; rt < h.Np / 16; ++rt) pl.rec_units.push_back(mc3::RecUnit{i, rt, ct, 0});
  }
  // Scoring units.  One instance: XCD-major placement -- grid slot b runs on XCD b % 8
  // and the units of one XCD are consecutive in (pair, tile) order, so each XCD's L2
  // holds the J rows of few pairs; the tiles of a pair alternate which row block they
  // take first; trailing slots are idle.  A batch: the pairs of every instance (each a
  // group of its CT tiles, which read the same J rows) by decreasing cost, then
  // decreasing CT (stable, so instance order breaks ties), longest first; eight groups
  // at a time are laid out with stride 8 -- slot 8 j + x holds tile j of group x, so a
  // group's tiles run together on one XCD and take the same row block first, and all
  // but the first read of its J rows hit that XCD's L2; slots past a group's CT idle.
  struct Group {
    int inst, p, CT, cost;
  };
  std::vector<Group> groups[kClasses];
  for (int i = 0; i < n; ++i) {
    InstH& h = pl.inst[i];
    h.cls = cfg.precision != MC3_SPLIT_BF16 ? 0 : cfg.tile_cols ? tile_class(cfg.tile_cols) : split_class(h.B);
    const int TN = cfg.precision == MC3_SPLIT_BF16 ? 64 * class_waves(h.cls) : kTileF64;
    const int CT = (h.B + TN - 1) / TN;  // tiles holding at least one real column
    const int U = h.P * CT;
    const int per = (U + 7) / 8;
    h.unit_off = (int)pl.units_local.size();
    h.unit_grid = 8 * per;
    for (int b = 0; b < 8 * per; ++b) {
      const int u = (b & 7) * per + (b >> 3);
      mc3::Unit un{-1, 0, 0, 0};
      if (u < U) un = mc3::Unit{i, u / CT, u % CT, ((u / CT) + (u % CT)) & 1};
      pl.units_local.push_back(un);
    }
    for (int p = 0; p < h.P; ++p) groups[h.cls].push_back(Group{i, p, CT, unit_cost(h.NB, p)});
  }
  if (n == 1) {
    pl.units_global[pl.inst[0].cls] = pl.units_local;
  } else {
    for (int k = 0; k < kClasses; ++k) {
      std::vector<Group>& gs = groups[k];
      std::stable_sort(gs.begin(), gs.end(),
                       [](const Group& a, const Group& b) { return a.cost != b.cost ? a.cost > b.cost : a.CT > b.CT; });
      for (size_t g0 = 0; g0 < gs.size(); g0 += 8) {
        const size_t ng = std::min<size_t>(8, gs.size() - g0);
        int cmax = 0;
        for (size_t x = 0; x < ng; ++x) cmax = std::max(cmax, gs[g0 + x].CT);
        for (int j = 0; j < cmax; ++j)
          for (size_t x = 0; x < 8; ++x) {
            mc3::Unit un{-1, 0, 0, 0};
            if (x < ng && j < gs[g0 + x].CT) un = mc3::Unit{gs[g0 + x].inst, gs[g0 + x].p, j, 0};
            pl.units_global[k].push_back(un);
          }
      }
    }
  }
  // workspace layout
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, kAlign);
    return at;
  };
  const size_t C = (size_t)pl.total_chains;
  pl.insts = take((size_t)n * sizeof(mc3::Inst));
  pl.chain_inst_off = take(C * 4);
  for (int k = 0; k < kClasses; ++k) pl.units_global_off[k] = take(pl.units_global[k].size() * sizeof(mc3::Unit));
  pl.units_local_off = take(pl.units_local.size() * sizeof(mc3::Unit));
  pl.pblocks_off = take(pl.pblocks.size() * sizeof(mc3::PBlock));
  pl.rec_units_off = take(pl.rec_units.size() * sizeof(mc3::RecUnit));
  pl.sched = take((size_t)n * 3 * sizeof(double));
  pl.clock = take(4);
  pl.e_cur = take(C * 8);
  pl.e_bar = take(C * 8);
  pl.roots = take((size_t)pl.nslots * C * 4);
  pl.moves = take(C * 8);
  pl.near = take(C * 8);
  pl.minm = take(C * 8);
  pl.drift = take(C * 8);
  pl.drift_ev = take(C * 8);
  pl.u_cur = take(C * 8);
  if (!pl.delta) {
    pl.moveD = take(C * 2 * (size_t)pl.Wmax * 4);
    pl.mflag = take(C * 4);
    pl.xpart = take(C * (size_t)mc3::kMoveCols * kMoveRowsMax * 8);
  }
  pl.ring = take((size_t)cfg.trace_steps * C * sizeof(mc3::Record));
  pl.means = take((size_t)cfg.mean_steps * 3 * sizeof(double));
  if (pl.delta) pl.vals = take((size_t)cfg.mean_steps * C * 2 * sizeof(double));
  size_t candT = 0;
  for (int i = 0; i < n; ++i) {
    InstH& h = pl.inst[i];
    const size_t np2 = (size_t)h.Np * h.Np;
    h.J64 = take(np2 * sizeof(double));
    h.Jpack = take(cfg.precision == MC3_SPLIT_BF16 ? np2 * 3 * sizeof(uint16_t) : np2 * sizeof(double));
    h.flip_slot = (size_t)h.W * h.Bp * 4;
    h.flips = take((size_t)pl.nslots * h.flip_slot);
    for (int q = 0; q < 2; ++q) h.base[q] = take((size_t)(h.desc.chains + 1) * h.W * 4);
    h.partial = take((size_t)h.P * h.Bp * 8);
    h.spins = take((size_t)h.desc.chains * h.W * 4);
    if (pl.delta) h.field = take((size_t)h.desc.chains * h.Np * 8);
    h.upart = take((size_t)(h.Np / 16) * h.desc.chains * 8);
    if (cfg.law == MC3_LAW_LINE || cfg.law == MC3_LAW_TABLE) h.prior = take((size_t)(h.desc.M + 1) * 8);
    if (cfg.law == MC3_LAW_TABLE) h.root_q = take((size_t)(h.desc.M + 1) * 8);
    candT = std::max(candT, (size_t)h.W * h.Bp * 4);
  }
  pl.candT = take(candT);
  pl.total = o;
  return pl;
}

mc3_batch_config single_to_batch(const mc3_config* c, mc3_instance_desc* one) {
  mc3_batch_config b;
  std::memset(&b, 0, sizeof b);
  one->N = c->N;
  one->M = c->M;
  one->chains = c->chains;
  one->kmin = c->kmin;
  one->kmax = c->kmax;
  b.n_instances = 1;
  b.precision = c->precision;
  b.rule = c->rule;
  b.trace_steps = c->trace_steps;
  b.mean_steps = c->mean_steps;
  b.chain_base = c->chain_base;
  b.seed = c->seed;
  b.near_tie_tol = c->near_tie_tol;
  b.instances = one;
  b.scorer = c->scorer;
  b.arity = c->arity;
  b.law = c->law;
  b.law_table = c->law_table;
  b.tile_cols = c->tile_cols;
  b.recompute_every = c->recompute_every;
  b.energy_update = c->energy_update;
  b.drift_tol = c->drift_tol;
  b.bias = c->bias;
  return b;
}

}  // namespace

struct mc3_ctx {
  mc3_batch_config cfg;
  std::vector<mc3_instance_desc> descs;
  Plan pl;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  bool have_chains = false, have_proposal = false, have_scores = false, poisoned = false;
  bool noalloc = false;      // the workspace is the device's fixed array (mc3_create_noalloc)
  uint32_t proposal_step = 0;
  double tol = 0.0;          // fixed part of the near-tie threshold (plus beta * tie_coef per instance)
  double drift_tol = 1e-9;   // relative drift counted as an event by the periodic recompute
  int64_t steps_done = 0;
  int64_t recomputes = 0;    // periodic or explicit FP64 recomputes since init_chains
  std::vector<double> sched_host;   // the last per-instance schedules uploaded
  // optional HIP-event timing of the scoring launches
  bool timing = false;
  int32_t t_every = 1;      // bracket every t_every-th scoring launch
  int64_t t_seen = 0;       // scoring launches since timing was enabled
  std::vector<hipEvent_t> t_start, t_stop;
  std::vector<char> t_pending;
  size_t t_next = 0;
  double t_total_ms = 0.0;
  int64_t t_count = 0;
  bool star_lds_set = false;   // k_step_delta_star's dynamic LDS limit raised past 64 KiB
  // mc3_step_n_graph: the captured body, the stream it is captured on, and what it was
  // captured for (schedule, and the first step's residue modulo the body length)
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  double g_beta0 = 0.0, g_beta1 = 0.0;
  int64_t g_total = 0, g_len = 0, g_phase = -1;
  std::string err;

  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  mc3::Key key() const { return mc3::Key{(uint32_t)cfg.seed, (uint32_t)(cfg.seed >> 32)}; }
  uint32_t slot(uint32_t step) const { return step % (uint32_t)pl.nslots; }
  int32_t* roots(uint32_t step) const { return at<int32_t>(pl.roots) + (size_t)slot(step) * pl.total_chains; }
  const mc3::Inst* insts() const { return at<const mc3::Inst>(pl.insts); }
  const int32_t* chain_inst() const { return at<const int32_t>(pl.chain_inst_off); }
  bool metropolis() const { return cfg.rule == MC3_RULE_METROPOLIS; }
  bool all_J() const {
    for (const InstH& h : pl.inst)
      if (!h.have_J) return false;
    return true;
  }
};

namespace {

mc3_status fail(mc3_ctx* c, mc3_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
    if (s == MC3_E_DEVICE) c->poisoned = true;
  }
  return s;
}

mc3_status check_launch(mc3_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, MC3_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return MC3_OK;
}

mc3_status hip_ok(mc3_ctx* c, hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(c, MC3_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return MC3_OK;
}

#define MC3_TRY(expr)            \
  do {                           \
    mc3_status _s = (expr);      \
    if (_s != MC3_OK) return _s; \
  } while (0)

mc3_status usable(mc3_ctx* c) {
  if (!c) return MC3_E_ARG;
  if (c->poisoned) return fail(c, MC3_E_STATE, "context poisoned by an earlier device error");
  c->err.clear();
  return MC3_OK;
}

// Device copy of the instance table (sizes, byte offsets, scales); synchronous.
mc3_status upload_insts(mc3_ctx* c) {
  const Plan& pl = c->pl;
  std::vector<mc3::Inst> t(pl.inst.size());
  for (size_t i = 0; i < pl.inst.size(); ++i) {
    const InstH& h = pl.inst[i];
    mc3::Inst& d = t[i];
    std::memset(&d, 0, sizeof d);
    d.N = h.desc.N;
    d.Np = h.Np;
    d.W = h.W;
    d.M = h.desc.M;
    d.chains = h.desc.chains;
    d.kmin = h.desc.kmin;
    d.kmax = h.desc.kmax;
    d.B = h.B;
    d.Bp = h.Bp;
    d.NB = h.NB;
    d.P = h.P;
    d.chain0 = h.chain0;
    d.arity = h.arity;
    d.law = c->cfg.law;
    d.scale = h.scale;
    d.tie_coef = h.tie_coef;
    d.upart = h.upart;
    d.J64 = h.J64;
    d.Jpack = h.Jpack;
    d.flips = h.flips;
    d.flip_slot = h.flip_slot;
    d.base[0] = h.base[0];
    d.base[1] = h.base[1];
    d.partial = h.partial;
    d.spins = h.spins;
    d.field = h.field;
    d.prior = h.prior;
    d.root_q = h.root_q;
  }
  MC3_TRY(hip_ok(c, hipMemcpyAsync(c->at<char>(pl.insts), t.data(), t.size() * sizeof(mc3::Inst),
                                   hipMemcpyHostToDevice, c->stream), "upload instance table"));
  return hip_ok(c, hipStreamSynchronize(c->stream), "upload sync");
}

// Every chain's pair sum U and energy recomputed in FP64 from its spins on the matrix
// cores (k_recompute_f64, then k_recompute_finish): mode 0 sets them (init, resume);
// mode 1 is the periodic check -- records the drift of the carried energy, counts
// drift events, carries the recomputed values.  The field-update path also recomputes
// its fields h = J s.
mc3_status launch_recompute(mc3_ctx* c, int mode) {
  const Plan& pl = c->pl;
  hipLaunchKernelGGL(mc3::k_recompute_f64, dim3((unsigned)pl.rec_units.size()), dim3(256), 0, c->stream, c->ws,
                     c->insts(), c->at<const mc3::RecUnit>(pl.rec_units_off));
  MC3_TRY(check_launch(c, "recompute kernel"));
  hipLaunchKernelGGL(mc3::k_recompute_finish, dim3((pl.total_chains + 255) / 256), dim3(256), 0, c->stream, c->ws,
                     c->insts(), c->chain_inst(), pl.total_chains, c->at<double>(pl.u_cur), c->at<double>(pl.e_cur),
                     c->at<double>(pl.drift), c->at<unsigned long long>(pl.drift_ev), c->drift_tol, mode);
  MC3_TRY(check_launch(c, "recompute finish kernel"));
  if (pl.delta) {
    hipLaunchKernelGGL(mc3::k_field_init, dim3(pl.total_chains), dim3(256), 0, c->stream, c->ws, c->insts(),
                       c->chain_inst());
    MC3_TRY(check_launch(c, "field kernel"));
  }
  if (mode == 1) c->recomputes += 1;
  return MC3_OK;
}

// The periodic recompute after the selection of global step t.
bool recompute_due(const mc3_ctx* c, uint32_t t) {
  const int32_t K = c->cfg.recompute_every;
  return K > 0 && ((uint64_t)t + 1u) % (uint64_t)K == 0u;
}

mc3_status maybe_recompute(mc3_ctx* c, uint32_t t) {
  if (!recompute_due(c, t)) return MC3_OK;
  return launch_recompute(c, 1);
}

mc3_status no_delta(mc3_ctx* c, const char* what) {
  if (!c->pl.delta) return MC3_OK;
  return fail(c, MC3_E_UNSUPPORTED, "%s: not available with the field-update scorer (use mc3_step_n)", what);
}

// n steps of the field-update path: persistent per-chain launches of at most 2048
// steps each, then the chain means of the steps still in the trace ring.
mc3_status do_step_n_delta(mc3_ctx* c, uint32_t step0, int64_t n, double beta0, double beta1, int64_t total,
                           const double* sched = nullptr) {
  const Plan& pl = c->pl;
  int Nmax = 0;
  for (const InstH& h : pl.inst) Nmax = std::max(Nmax, h.desc.N);
  const int64_t K = c->cfg.recompute_every;
  for (int64_t done = 0; done < n;) {
    int chunk = (int)std::min<int64_t>(2048, n - done);
    if (K > 0) {   // end the launch at the next step t with (t + 1) % K == 0
      const int64_t t0 = (int64_t)step0 + done;
      chunk = (int)std::min<int64_t>(chunk, K - t0 % K);
    }
    if (c->cfg.law == MC3_LAW_BIASED) {
      hipLaunchKernelGGL(mc3::k_step_biased, dim3(pl.total_chains), dim3(256), pl.delta_lds, c->stream, c->ws,
                         c->insts(), c->chain_inst(), pl.total_chains, Nmax, pl.Mmax, pl.Wmax,
                         c->at<double>(pl.e_cur), c->at<double>(pl.u_cur), c->at<mc3::Record>(pl.ring),
                         c->at<unsigned long long>(pl.moves), c->at<unsigned long long>(pl.near),
                         c->at<double>(pl.minm), c->at<double>(pl.e_bar), c->at<double>(pl.vals), c->cfg.mean_steps,
                         c->cfg.bias, beta0, beta1, (long long)total, c->tol, c->key(), c->cfg.chain_base,
                         step0 + (uint32_t)done, chunk, c->cfg.trace_steps, sched);
      MC3_TRY(check_launch(c, "biased step kernel"));
      done += chunk;
      MC3_TRY(maybe_recompute(c, step0 + (uint32_t)(done - 1)));
      continue;
    }
    if (pl.delta_star) {
      if (pl.delta_lds > 65536 && !c->star_lds_set) {
        MC3_TRY(hip_ok(c, hipFuncSetAttribute(reinterpret_cast<const void*>(&mc3::k_step_delta_star),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.delta_lds),
                       "field-update star kernel LDS"));
        c->star_lds_set = true;
      }
      hipLaunchKernelGGL(mc3::k_step_delta_star, dim3(pl.total_chains), dim3(256), pl.delta_lds, c->stream, c->ws,
                         c->insts(), c->chain_inst(), pl.total_chains, Nmax, pl.Mmax, pl.Wmax, pl.Kmax,
                         c->at<double>(pl.e_cur), c->at<double>(pl.u_cur), c->at<mc3::Record>(pl.ring),
                         c->at<unsigned long long>(pl.moves), c->at<unsigned long long>(pl.near),
                         c->at<double>(pl.minm), c->at<double>(pl.e_bar), c->at<double>(pl.vals), c->cfg.mean_steps,
                         c->metropolis() ? 1 : 0, beta0, beta1, (long long)total, c->tol, c->key(),
                         c->cfg.chain_base, step0 + (uint32_t)done, chunk, c->cfg.trace_steps, sched);
      MC3_TRY(check_launch(c, "field-update star kernel"));
      done += chunk;
      MC3_TRY(maybe_recompute(c, step0 + (uint32_t)(done - 1)));
      continue;
    }
    hipLaunchKernelGGL(mc3::k_step_delta, dim3(pl.total_chains), dim3(256), pl.delta_lds, c->stream, c->ws,
                       c->insts(), c->chain_inst(), pl.total_chains, Nmax, pl.Mmax, pl.Wmax,
                       c->at<double>(pl.e_cur), c->at<double>(pl.u_cur), c->at<mc3::Record>(pl.ring),
                       c->at<unsigned long long>(pl.moves), c->at<unsigned long long>(pl.near),
                       c->at<double>(pl.minm), c->at<double>(pl.e_bar), c->at<double>(pl.vals), c->cfg.mean_steps,
                       c->metropolis() ? 1 : 0, beta0, beta1, (long long)total, c->tol, c->key(),
                       c->cfg.chain_base, step0 + (uint32_t)done, chunk, c->cfg.trace_steps, sched);
    MC3_TRY(check_launch(c, "field-update step kernel"));
    done += chunk;
    MC3_TRY(maybe_recompute(c, step0 + (uint32_t)(done - 1)));
  }
  if (c->cfg.mean_steps > 0) {
    const int64_t keep = std::min<int64_t>(n, c->cfg.mean_steps);
    hipLaunchKernelGGL(mc3::k_chain_means_steps, dim3((unsigned)keep), dim3(256), 0, c->stream,
                       c->at<double>(pl.means), c->at<const double>(pl.vals), pl.total_chains, c->cfg.mean_steps,
                       step0 + (uint32_t)(n - keep));
    MC3_TRY(check_launch(c, "means kernel"));
  }
  c->steps_done += n;
  c->have_proposal = c->have_scores = false;
  return MC3_OK;
}

// Proposal blocks [b0, b0 + nb) of the block table for steps step0 .. step0+nsteps-1
// (at most nslots - 1 of them); with write_base, also the base words of step0.
mc3_status launch_propose(mc3_ctx* c, uint32_t step0, int nsteps, bool write_base, int b0, int nb,
                          const uint32_t* clk = nullptr) {
  const Plan& pl = c->pl;
  const size_t lds = (size_t)pl.prop_rows * pl.prop_T * pl.prop_stride * 4;
  hipLaunchKernelGGL(mc3::k_propose, dim3(nb, nsteps), dim3(pl.prop_T), lds, c->stream, c->ws, c->insts(),
                     c->at<const mc3::PBlock>(pl.pblocks_off) + b0, c->at<int32_t>(pl.roots), pl.total_chains,
                     (uint32_t)pl.nslots, write_base ? 1 : 0, pl.prop_stride, pl.prop_rows, c->metropolis() ? 1 : 0,
                     c->key(), c->cfg.chain_base, step0, clk);
  return check_launch(c, "propose kernel");
}

mc3_status propose_all(mc3_ctx* c, uint32_t step0, int nsteps, bool write_base, const uint32_t* clk = nullptr) {
  return launch_propose(c, step0, nsteps, write_base, 0, (int)c->pl.pblocks.size(), clk);
}

mc3_status timing_collect(mc3_ctx* c, size_t i) {
  if (!c->t_pending[i]) return MC3_OK;
  MC3_TRY(hip_ok(c, hipEventSynchronize(c->t_stop[i]), "timing sync"));
  float ms = 0.0f;
  MC3_TRY(hip_ok(c, hipEventElapsedTime(&ms, c->t_start[i], c->t_stop[i]), "timing read"));
  c->t_total_ms += ms;
  c->t_count += 1;
  c->t_pending[i] = 0;
  return MC3_OK;
}

// One scoring launch over `grid` entries of a unit table of tile class `cls` (the
// whole batch's, or one instance's own), for the flip sets of the last proposal.
mc3_status launch_score_units(mc3_ctx* c, size_t table_off, int grid, int cls) {
  const uint32_t t = c->proposal_step;
  const mc3::Unit* units = c->at<const mc3::Unit>(table_off);
  if (c->cfg.precision == MC3_SPLIT_BF16) {
    if (cls == 2)
      hipLaunchKernelGGL(mc3::k_score_split<8>, dim3(grid), dim3(512), 0, c->stream, c->ws, c->insts(), units,
                         c->roots(t), c->slot(t), t & 1u);
    else if (cls == 1)
      hipLaunchKernelGGL(mc3::k_score_split<4>, dim3(grid), dim3(256), 0, c->stream, c->ws, c->insts(), units,
                         c->roots(t), c->slot(t), t & 1u);
    else
      hipLaunchKernelGGL(mc3::k_score_split<2>, dim3(grid), dim3(128), 0, c->stream, c->ws, c->insts(), units,
                         c->roots(t), c->slot(t), t & 1u);
  } else
    hipLaunchKernelGGL(mc3::k_score_f64, dim3(grid), dim3(256), 0, c->stream, c->ws, c->insts(), units,
                       c->roots(t), c->slot(t), t & 1u);
  return check_launch(c, "score kernel");
}

// Scoring launches (one per tile class in `tables`), bracketed by timing events
// when timing is on.
struct ScoreLaunch {
  size_t off;
  int grid, cls;
};

mc3_status score_timed(mc3_ctx* c, const ScoreLaunch* tables, int n) {
  size_t i = 0;
  const bool timed = c->timing && (c->t_seen++ % c->t_every) == 0;
  if (timed) {
    i = c->t_next;
    c->t_next = (c->t_next + 1) % c->t_start.size();
    MC3_TRY(timing_collect(c, i));
    MC3_TRY(hip_ok(c, hipEventRecord(c->t_start[i], c->stream), "timing event"));
  }
  for (int k = 0; k < n; ++k)
    if (tables[k].grid > 0) MC3_TRY(launch_score_units(c, tables[k].off, tables[k].grid, tables[k].cls));
  if (timed) {
    MC3_TRY(hip_ok(c, hipEventRecord(c->t_stop[i], c->stream), "timing event"));
    c->t_pending[i] = 1;
  }
  return MC3_OK;
}

mc3_status do_score(mc3_ctx* c, double* E_out) {
  const Plan& pl = c->pl;
  ScoreLaunch tl[kClasses];
  for (int k = 0; k < kClasses; ++k) tl[k] = ScoreLaunch{pl.units_global_off[k], (int)pl.units_global[k].size(), k};
  MC3_TRY(score_timed(c, tl, kClasses));
  if (E_out) {
    for (const InstH& h : pl.inst) {
      hipLaunchKernelGGL(mc3::k_column_energies, dim3((h.B + 255) / 256), dim3(256), 0, c->stream, E_out + h.col0,
                         c->at<const double>(h.partial), h.P, h.Bp, h.B, h.scale);
      MC3_TRY(check_launch(c, "column energy kernel"));
    }
  }
  c->have_scores = true;
  return MC3_OK;
}

// The step clock of a captured graph body: its kernels take steps relative to `base`
// and add the clock's value, and the selection forms beta from the schedule.
struct ClockArg {
  const uint32_t* clk = nullptr;
  uint32_t base = 0;
  double beta0 = 0.0, beta1 = 0.0;
  int64_t total = 0;
};

mc3_status launch_moves(mc3_ctx* c, int g0, int n);

// Selection of global chains [g0, g0 + n) at `step`; with next_base, also the base
// words of step+1 (whose flip sets and roots must already be proposed).  Ring slots are
// those of `step` itself; with a clock the kernel takes step - base.

mc3_status launch_select(mc3_ctx* c, uint32_t step, double beta, bool next_base, int g0, int n,
                         const ClockArg& ck = ClockArg{}, const double* sched = nullptr) {
  const Plan& pl = c->pl;
  const size_t lds = (size_t)(pl.Mmax + 1) * 16;
  const bool exact = c->cfg.energy_update == MC3_ENERGY_EXACT;
  hipLaunchKernelGGL(mc3::k_select, dim3(n), dim3(256), lds, c->stream, c->ws, c->insts(), c->chain_inst(), g0,
                     pl.total_chains, c->at<double>(pl.e_cur), c->at<double>(pl.u_cur), c->roots(step),
                     c->roots(step + 1u),
                     c->at<mc3::Record>(pl.ring), c->at<unsigned long long>(pl.moves),
                     c->at<unsigned long long>(pl.near), c->at<double>(pl.minm), c->at<double>(pl.e_bar),
                     c->metropolis() ? 1 : 0, beta, c->tol, c->key(), c->cfg.chain_base,
                     ck.clk ? step - ck.base : step, c->slot(step), c->slot(step + 1u), c->cfg.trace_steps,
                     next_base ? 1 : 0, ck.clk, ck.beta0, ck.beta1, (long long)ck.total, sched, exact ? 1 : 0,
                     c->at<uint32_t>(pl.moveD), pl.Wmax, c->at<int32_t>(pl.mflag), c->at<const double>(pl.xpart),
                     move_row_parts(pl.total_chains));
  MC3_TRY(check_launch(c, "select kernel"));
  if (!exact) return MC3_OK;
  return launch_moves(c, g0, n);
}

// The exact energy update of the chains [g0, g0 + n) that moved at the last
// selection: their difference from the rows of the flipped sites, kMoveCols x RS blocks per chain (a
// column slice of J64 each, the rows split RS ways; RS depends on the plan alone, so a
// chain's sum has the same order in every launch).  The next selection adds it into
// the carried energy and the step's record, or flush_moves does.
mc3_status launch_moves(mc3_ctx* c, int g0, int n) {
  const Plan& pl = c->pl;
  int Nmax = 0;
  for (const InstH& h : pl.inst) Nmax = std::max(Nmax, h.desc.N);
  const int RS = move_row_parts(pl.total_chains);
  hipLaunchKernelGGL(mc3::k_move_delta, dim3(n * mc3::kMoveCols * RS), dim3(256),
                     (size_t)8 * pl.Wmax + (size_t)2 * Nmax, c->stream, c->ws, c->insts(), c->chain_inst(), g0,
                     c->at<const uint32_t>(pl.moveD), pl.Wmax, c->at<const int32_t>(pl.mflag),
                     c->at<double>(pl.xpart), RS);
  return check_launch(c, "move kernel");
}

// With the exact energy update: the differences of the moves of `step` (the last
// selection) that no selection has added yet, added into the carried energies and the
// step's records (k_move_finish; chains whose flag is clear are left alone).  Run
// before anything that reads the carried energies other than the next selection: the
// means, the periodic recompute, and the end of every call that selects.
mc3_status flush_moves(mc3_ctx* c, uint32_t step, const ClockArg& ck = ClockArg{}) {
  const Plan& pl = c->pl;
  if (c->cfg.energy_update != MC3_ENERGY_EXACT || pl.delta) return MC3_OK;
  const int n = pl.total_chains;
  hipLaunchKernelGGL(mc3::k_move_finish, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->insts(), c->chain_inst(),
                     0, n, pl.total_chains, c->at<int32_t>(pl.mflag), c->at<const double>(pl.xpart),
                     move_row_parts(pl.total_chains), c->at<double>(pl.u_cur), c->at<double>(pl.e_cur),
                     c->at<mc3::Record>(pl.ring), c->cfg.trace_steps, ck.clk ? step - ck.base : step, ck.clk);
  return check_launch(c, "move finish kernel");
}

mc3_status launch_means(mc3_ctx* c, uint32_t step, const ClockArg& ck = ClockArg{}) {
  const Plan& pl = c->pl;
  if (c->cfg.mean_steps <= 0) return MC3_OK;
  hipLaunchKernelGGL(mc3::k_chain_means, dim3(1), dim3(256), 0, c->stream, c->at<double>(pl.means),
                     c->at<const double>(pl.e_cur), c->at<const double>(pl.e_bar), pl.total_chains,
                     step % (uint32_t)c->cfg.mean_steps, ck.clk ? step - ck.base : step, ck.clk,
                     (uint32_t)c->cfg.mean_steps);
  return check_launch(c, "means kernel");
}

mc3_status after_select(mc3_ctx* c, uint32_t step, bool next_base) {
  if (c->cfg.mean_steps > 0 || recompute_due(c, step)) MC3_TRY(flush_moves(c, step));
  MC3_TRY(launch_means(c, step));
  MC3_TRY(maybe_recompute(c, step));
  c->have_proposal = next_base;
  c->have_scores = false;
  if (next_base) c->proposal_step = step + 1u;
  c->steps_done += 1;
  return MC3_OK;
}

// One selection as a call of its own (mc3_select): the carried energies are complete
// when it returns.
mc3_status do_select(mc3_ctx* c, uint32_t step, double beta, bool next_base = false,
                     const double* sched = nullptr) {
  MC3_TRY(launch_select(c, step, beta, next_base, 0, c->pl.total_chains, ClockArg{}, sched));
  MC3_TRY(after_select(c, step, next_base));
  return flush_moves(c, step);
}

// The selection of step t inside a run of steps: with the exact energy update the
// moves' differences are summed after it (k_move_delta) and added by the next
// selection, so the run's last step is flushed by its caller.
mc3_status select_in_run(mc3_ctx* c, uint32_t t, double beta, bool next_base, const double* sched) {
  MC3_TRY(launch_select(c, t, beta, next_base, 0, c->pl.total_chains, ClockArg{}, sched));
  return after_select(c, t, next_base);
}

double beta_at(uint32_t t, double beta0, double beta1, int64_t total) {
  if (total <= 1) return beta0;
  return beta0 + (beta1 - beta0) * ((double)t / (double)(total - 1));
}

// n steps on the caller's stream.  Flip sets and roots do not depend on the states, so
// they are drawn `ahead` steps per launch into the ring (slot = step % (ahead + 1));
// the group of steps a .. a+ahead-1 is drawn just before select(a-1), which needs the
// flip sets of step a for the base words a's scoring uses, and whose own slot is the
// one slot the group does not touch.  Per step: one scoring launch and one selection
// launch (which also forms the next step's base words).
mc3_status do_step_n(mc3_ctx* c, uint32_t step0, int64_t n, double beta0, double beta1, int64_t total,
                     const double* sched = nullptr) {
  if (n <= 0) return MC3_OK;
  const int64_t K = c->pl.ahead;
  MC3_TRY(propose_all(c, step0, (int)std::min<int64_t>(K, n), true));
  c->have_proposal = true;
  c->proposal_step = step0;
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t t = step0 + (uint32_t)i;
    const bool last = i + 1 == n;
    MC3_TRY(do_score(c, nullptr));
    if (!last && (i + 1) % K == 0) MC3_TRY(propose_all(c, t + 1u, (int)std::min<int64_t>(K, n - i - 1), false));
    MC3_TRY(select_in_run(c, t, beta_at(t, beta0, beta1, total), !last, sched));
  }
  MC3_TRY(flush_moves(c, step0 + (uint32_t)(n - 1)));
  c->have_proposal = false;
  return MC3_OK;
}

// Steps t0 .. t0+n-1 of mc3_step_n whose first group of proposals is already drawn.
mc3_status step_groups(mc3_ctx* c, uint32_t t0, int64_t n, double beta0, double beta1, int64_t total) {
  const int64_t K = c->pl.ahead;
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t t = t0 + (uint32_t)i;
    const bool last = i + 1 == n;
    MC3_TRY(do_score(c, nullptr));
    if (!last && (i + 1) % K == 0) MC3_TRY(propose_all(c, t + 1u, (int)std::min<int64_t>(K, n - i - 1), false));
    MC3_TRY(select_in_run(c, t, beta_at(t, beta0, beta1, total), !last, nullptr));
  }
  return n > 0 ? flush_moves(c, t0 + (uint32_t)(n - 1)) : MC3_OK;
}

int64_t gcd64(int64_t a, int64_t b) { return b ? gcd64(b, a % b) : a; }

// Body length of a replayed graph: a multiple of the proposal group (K), of the ring
// (nslots) and of 2 (the base words alternate), so that every captured launch finds
// its ring slots and base words at the same place on every replay.
int64_t graph_body(const Plan& pl) {
  const int64_t K = pl.ahead, S = pl.nslots;
  const int64_t KS = K / gcd64(K, S) * S;
  return KS % 2 ? 2 * KS : KS;
}

// Capture the body for steps a .. a+L-1 on the capture stream: per step the scoring,
// every K-th step the next group's proposals, the selection (always followed by a
// step: next_base), the means; then the clock advances by L.
mc3_status capture_body(mc3_ctx* c, uint32_t a, int64_t L, double beta0, double beta1, int64_t total) {
  const int64_t K = c->pl.ahead;
  const ClockArg ck{c->at<const uint32_t>(c->pl.clock), a, beta0, beta1, total};
  hipStream_t user = c->stream;
  const bool timing = c->timing;
  c->stream = c->cap;
  c->timing = false;
  hipGraph_t g = nullptr;
  mc3_status st = hip_ok(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal), "graph capture");
  if (st == MC3_OK) {
    for (int64_t j = 0; j < L && st == MC3_OK; ++j) {
      const uint32_t t = a + (uint32_t)j;
      c->proposal_step = t;
      st = do_score(c, nullptr);
      if (st == MC3_OK && (j + 1) % K == 0) st = propose_all(c, (uint32_t)(j + 1), (int)K, false, ck.clk);
      if (st == MC3_OK) st = launch_select(c, t, 0.0, true, 0, c->pl.total_chains, ck);
      if (st == MC3_OK && c->cfg.mean_steps > 0) st = flush_moves(c, t, ck);
      if (st == MC3_OK) st = launch_means(c, t, ck);
    }
    if (st == MC3_OK) {
      hipLaunchKernelGGL(mc3::k_clock, dim3(1), dim3(64), 0, c->stream, c->at<uint32_t>(c->pl.clock), (uint32_t)L, 1);
      st = check_launch(c, "clock kernel");
    }
    const hipError_t e = hipStreamEndCapture(c->cap, &g);
    if (st == MC3_OK) st = hip_ok(c, e, "graph capture");
  }
  c->stream = user;
  c->timing = timing;
  if (st == MC3_OK) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    st = hip_ok(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0), "graph instantiate");
  }
  if (g) (void)hipGraphDestroy(g);
  if (st != MC3_OK) {
    c->g_phase = -1;
    return st;
  }
  c->g_beta0 = beta0;
  c->g_beta1 = beta1;
  c->g_total = total;
  c->g_len = L;
  c->g_phase = (int64_t)(a % (uint32_t)L);
  return MC3_OK;
}

// mc3_step_n through a replayed graph: the first group's proposals, then R replays of
// the captured L-step body (captured once per schedule and step residue modulo L), then
// the remaining n - R L >= K steps launch by launch.  The same launches in the same
// order as do_step_n, so the same results.
mc3_status do_step_n_graph(mc3_ctx* c, uint32_t step0, int64_t n, double beta0, double beta1, int64_t total) {
  const Plan& pl = c->pl;
  const int64_t K = pl.ahead, L = graph_body(pl);
  const int64_t R = n >= L + K ? (n - K) / L : 0;
  // the periodic recompute is launched by the host between steps: not in a replay
  if (R == 0 || c->cfg.recompute_every > 0) return do_step_n(c, step0, n, beta0, beta1, total);
  MC3_TRY(propose_all(c, step0, (int)K, true));
  c->have_proposal = true;
  c->proposal_step = step0;
  if (!c->cap) MC3_TRY(hip_ok(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking), "capture stream"));
  if (!c->gexec || c->g_len != L || c->g_phase != (int64_t)(step0 % (uint32_t)L) || c->g_beta0 != beta0 ||
      c->g_beta1 != beta1 || c->g_total != total)
    MC3_TRY(capture_body(c, step0, L, beta0, beta1, total));
  // the body's launches take steps relative to its first; replay r starts at step0 + r L
  hipLaunchKernelGGL(mc3::k_clock, dim3(1), dim3(64), 0, c->stream, c->at<uint32_t>(pl.clock), step0, 0);
  MC3_TRY(check_launch(c, "clock kernel"));
  for (int64_t r = 0; r < R; ++r) MC3_TRY(hip_ok(c, hipGraphLaunch(c->gexec, c->stream), "graph launch"));
  const uint32_t t1 = step0 + (uint32_t)(R * L);
  c->steps_done += R * L;
  c->have_proposal = true;
  c->proposal_step = t1;
  c->have_scores = false;
  MC3_TRY(step_groups(c, t1, n - R * L, beta0, beta1, total));
  c->have_proposal = false;
  return MC3_OK;
}

// The same steps with one propose, one score and one select launch per instance,
// in instance order on the caller's stream: what running the instances one by one
// costs, against which the batched launches are measured.
mc3_status do_step_n_per_instance(mc3_ctx* c, uint32_t step0, int64_t n, double beta0, double beta1,
                                  int64_t total) {
  const Plan& pl = c->pl;
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t t = step0 + (uint32_t)i;
    const double beta = beta_at(t, beta0, beta1, total);
    c->proposal_step = t;
    for (const InstH& h : pl.inst) {
      MC3_TRY(launch_propose(c, t, 1, true, h.pblock_off, h.pblock_cnt));
      const ScoreLaunch one{pl.units_local_off + (size_t)h.unit_off * sizeof(mc3::Unit), h.unit_grid, h.cls};
      MC3_TRY(score_timed(c, &one, 1));
      MC3_TRY(launch_select(c, t, beta, false, h.chain0, h.desc.chains));
    }
    MC3_TRY(after_select(c, t, false));
  }
  if (n > 0) MC3_TRY(flush_moves(c, step0 + (uint32_t)(n - 1)));
  c->have_proposal = false;
  return MC3_OK;
}

// fixed_ws: the workspace is the library's own fixed array (its address is known to be
// device memory).
mc3_status create_impl(const mc3_batch_config* cfg, void* workspace, size_t bytes, void* stream, mc3_ctx** out,
                       bool fixed_ws = false) {
  if (!out) return MC3_E_ARG;
  *out = nullptr;
  if (validate_batch(cfg)) return MC3_E_ARG;
  size_t lds = 0;
  if (resolve_delta(*cfg, &lds) < 0) return MC3_E_UNSUPPORTED;
  Plan plan = make_plan(*cfg);
  if (!workspace || bytes < plan.total || ((uintptr_t)workspace % kAlign) != 0) return MC3_E_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MC3_E_DEVICE;
  hipPointerAttribute_t attr;
  if (!fixed_ws && (hipPointerGetAttributes(&attr, workspace) != hipSuccess || attr.type != hipMemoryTypeDevice)) {
    (void)hipGetLastError();
    return MC3_E_WORKSPACE;
  }
  mc3_ctx* c = new (std::nothrow) mc3_ctx();
  if (!c) return MC3_E_ARG;
  c->cfg = *cfg;
  c->descs.assign(cfg->instances, cfg->instances + cfg->n_instances);
  c->cfg.instances = c->descs.data();
  c->pl = std::move(plan);
  c->ws = (char*)workspace;
  c->stream = (hipStream_t)stream;
  c->device = dev;
  // Near ties: a fixed threshold when the caller gives one; otherwise 4 beta eps_E
  // per instance, eps_E = N 2^-24 the split path's bound on an energy's error (FP32
  // accumulation of N terms of a field of order one) and N 2^-40 the FP64 paths'.
  // A draw whose margin exceeds the largest change that errors of eps_E in every
  // energy can make to the cumulative weights (beta eps_E per unit of total weight)
  // picks the same node as exact arithmetic would.
  const bool split_scores = cfg->precision == MC3_SPLIT_BF16 && !c->pl.delta;
  c->tol = cfg->near_tie_tol >= 0.0 ? cfg->near_tie_tol : 0.0;
  for (InstH& h : c->pl.inst)
    h.tie_coef = cfg->near_tie_tol >= 0.0 ? 0.0 : 4.0 * h.desc.N * (split_scores ? 0x1.0p-24 : 0x1.0p-40);
  c->drift_tol = cfg->drift_tol >= 0.0 ? cfg->drift_tol : 1e-9;
  // the static tables
  const Plan& P = c->pl;
  auto up = [&](size_t off, const void* src, size_t n) {
    return n ? hipMemcpyAsync(c->at<char>(off), src, n, hipMemcpyHostToDevice, c->stream) : hipSuccess;
  };
  hipError_t e = up(P.chain_inst_off, P.chain_inst.data(), P.chain_inst.size() * 4);
  for (int k = 0; k < kClasses && e == hipSuccess; ++k)
    e = up(P.units_global_off[k], P.units_global[k].data(), P.units_global[k].size() * sizeof(mc3::Unit));
  if (e == hipSuccess) e = up(P.units_local_off, P.units_local.data(), P.units_local.size() * sizeof(mc3::Unit));
  if (e == hipSuccess) e = up(P.pblocks_off, P.pblocks.data(), P.pblocks.size() * sizeof(mc3::PBlock));
  if (e == hipSuccess) e = up(P.rec_units_off, P.rec_units.data(), P.rec_units.size() * sizeof(mc3::RecUnit));
  // log-priors: the line law's log C(M, v) = lgamma(M+1) - lgamma(v+1) - lgamma(M-v+1);
  // the table law's log q_v (q_v = 0: -infinity) and its cumulative weights
  std::vector<std::vector<double>> priors;
  std::vector<std::vector<uint64_t>> cdfs;
  size_t table_at = 0;
  for (const InstH& h : P.inst) {
    const int M = h.desc.M;
    if (!h.prior || e != hipSuccess) continue;
    priors.emplace_back(M + 1);
    if (cfg->law == MC3_LAW_TABLE) {
      cdfs.emplace_back();
      root_table(cfg->law_table + table_at, M, &cdfs.back());
      table_at += M + 1;
      for (int v = 0; v <= M; ++v) {
        const uint64_t q = cdfs.back()[v] - (v ? cdfs.back()[v - 1] : 0u);
        priors.back()[v] = q ? std::log((double)q) : -HUGE_VAL;
      }
      e = up(h.root_q, cdfs.back().data(), cdfs.back().size() * 8);
    } else {
      for (int v = 0; v <= M; ++v)
        priors.back()[v] =
            std::lgamma((double)M + 1.0) - std::lgamma((double)v + 1.0) - std::lgamma((double)(M - v) + 1.0);
    }
    if (e == hipSuccess) e = up(h.prior, priors.back().data(), priors.back().size() * 8);
  }
  c->cfg.law_table = nullptr;   // the caller's table is not kept
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess || upload_insts(c) != MC3_OK) {
    mc3_destroy(c);
    return MC3_E_DEVICE;
  }
  *out = c;
  return MC3_OK;
}

mc3_status pack_couplings(mc3_ctx* c, InstH& h, double scale);

mc3_status init_couplings_impl(mc3_ctx* c, int32_t instance, const double* J, int64_t ld, double scale) {
  MC3_TRY(usable(c));
  if (instance < 0 || instance >= (int32_t)c->pl.inst.size())
    return fail(c, MC3_E_ARG, "instance %d is not in the batch", instance);
  InstH& h = c->pl.inst[instance];
  const int N = h.desc.N, Np = h.Np;
  if (!J || ld < N) return fail(c, MC3_E_ARG, "J is NULL or ld < N");
  if (!std::isfinite(scale)) return fail(c, MC3_E_NUMERIC, "scale is not finite");
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j)
      if (!std::isfinite(J[(size_t)i * ld + j])) return fail(c, MC3_E_NUMERIC, "J[%d][%d] is not finite", i, j);
  double* J64 = c->at<double>(h.J64);
  MC3_TRY(hip_ok(c, hipMemsetAsync(J64, 0, (size_t)Np * Np * 8, c->stream), "clear J"));
  MC3_TRY(hip_ok(c, hipMemcpy2DAsync(J64, (size_t)Np * 8, J, (size_t)ld * 8, (size_t)N * 8, N, hipMemcpyHostToDevice,
                                     c->stream), "upload J"));
  const long long n = (long long)Np * Np;
  hipLaunchKernelGGL(mc3::k_mirror_upper, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, J64, Np);
  MC3_TRY(check_launch(c, "mirror kernel"));
  return pack_couplings(c, h, scale);
}

// The scorer's packed copy of an instance's J64 (three BF16 terms or FP64 fragments),
// then the instance's scale and tables.
mc3_status pack_couplings(mc3_ctx* c, InstH& h, double scale) {
  const int Np = h.Np;
  const double* J64 = c->at<const double>(h.J64);
  if (c->cfg.precision == MC3_SPLIT_BF16) {
    const long long n = (long long)(Np / 32) * (Np / 16) * 64;
    hipLaunchKernelGGL(mc3::k_pack_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       c->at<uint4>(h.Jpack), J64, Np);
  } else {
    const long long n = (long long)(Np / 16) * (Np / 4) * 64;
    hipLaunchKernelGGL(mc3::k_pack_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       c->at<double>(h.Jpack), J64, Np);
  }
  MC3_TRY(check_launch(c, "pack kernel"));
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "init_couplings sync"));
  h.scale = scale;
  h.have_J = true;
  c->have_chains = false;
  return upload_insts(c);
}

// Clear what a fresh chain state needs cleared: flip-set padding columns and the zero
// base row (must read as zero), counters, move flags, margins, the record and means
// rings.
mc3_status reset_buffers(mc3_ctx* c) {
  const Plan& pl = c->pl;
  const size_t C = (size_t)pl.total_chains;
  for (const InstH& h : pl.inst) {
    MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(h.flips), 0, (size_t)pl.nslots * h.flip_slot, c->stream), "clear"));
    for (int q = 0; q < 2; ++q)
      MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(h.base[q]), 0, (size_t)(h.desc.chains + 1) * h.W * 4, c->stream),
                     "clear"));
  }
  MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(pl.moves), 0, C * 8, c->stream), "clear"));
  MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(pl.near), 0, C * 8, c->stream), "clear"));
  MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(pl.drift), 0, C * 8, c->stream), "clear"));
  MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(pl.drift_ev), 0, C * 8, c->stream), "clear"));
  // no move's difference is pending (the selection adds a flagged chain's first); the
  // field-update path has no move buffers
  if (!pl.delta) MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(pl.mflag), 0, C * 4, c->stream), "clear"));
  c->recomputes = 0;
  {
    std::vector<double> big(C, HUGE_VAL);
    MC3_TRY(hip_ok(c, hipMemcpyAsync(c->at<double>(pl.minm), big.data(), big.size() * 8, hipMemcpyHostToDevice,
                                     c->stream), "init margins"));
    MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "init_chains sync"));
  }
  if (c->cfg.trace_steps > 0) {
    std::vector<mc3::Record> ring((size_t)c->cfg.trace_steps * C);
    for (auto& r : ring) {
      std::memset(&r, 0, sizeof r);
      r.step = 0xFFFFFFFFu;
    }
    MC3_TRY(hip_ok(c, hipMemcpyAsync(c->at<mc3::Record>(pl.ring), ring.data(), ring.size() * sizeof(mc3::Record),
                                     hipMemcpyHostToDevice, c->stream), "clear ring"));
    MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "init_chains sync"));
  }
  if (c->cfg.mean_steps > 0) {
    std::vector<double> tr((size_t)c->cfg.mean_steps * 3, -1.0);
    MC3_TRY(hip_ok(c, hipMemcpyAsync(c->at<double>(pl.means), tr.data(), tr.size() * 8, hipMemcpyHostToDevice,
                                     c->stream), "clear means"));
    MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "init_chains sync"));
  }
  return MC3_OK;
}


// Upload per-instance schedules (beta0, beta1, total) to the workspace table; waits for
// the stream first, so that no launch still reading the previous table is overtaken.
mc3_status upload_sched(mc3_ctx* c, const std::vector<double>& tab) {
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "schedule sync"));
  c->sched_host = tab;
  return hip_ok(c, hipMemcpyAsync(c->at<double>(c->pl.sched), c->sched_host.data(), tab.size() * 8,
                                  hipMemcpyHostToDevice, c->stream), "upload schedules");
}

mc3_status step_args(mc3_ctx* c, uint32_t step0, int64_t n, double beta0, double beta1) {
  MC3_TRY(usable(c));
  if (!c->have_chains) return fail(c, MC3_E_STATE, "step_n before init_chains");
  if (n < 0 || (uint64_t)step0 + (uint64_t)n > 0x100000000ull) return fail(c, MC3_E_ARG, "bad step range");
  if (!std::isfinite(beta0) || !std::isfinite(beta1) || beta0 < 0.0 || beta1 < 0.0)
    return fail(c, MC3_E_ARG, "beta must be finite and >= 0");
  return MC3_OK;
}

}  // namespace

extern "C" {

const char* mc3_version(void) { return "mc3 0.2 (gfx950)"; }

mc3_status mc3_batch_workspace_size(const mc3_batch_config* cfg, size_t* bytes) {
  if (validate_batch(cfg) || !bytes) return MC3_E_ARG;
  size_t lds = 0;
  if (resolve_delta(*cfg, &lds) < 0) return MC3_E_UNSUPPORTED;
  *bytes = make_plan(*cfg).total;
  return MC3_OK;
}

mc3_status mc3_workspace_size(const mc3_config* cfg, size_t* bytes) {
  if (!cfg) return MC3_E_ARG;
  mc3_instance_desc one;
  const mc3_batch_config b = single_to_batch(cfg, &one);
  return mc3_batch_workspace_size(&b, bytes);
}

mc3_status mc3_batch_create(const mc3_batch_config* cfg, void* workspace, size_t bytes, void* stream,
                            mc3_ctx** out) {
  return create_impl(cfg, workspace, bytes, stream, out);
}

mc3_status mc3_create(const mc3_config* cfg, void* workspace, size_t bytes, void* stream, mc3_ctx** out) {
  if (out) *out = nullptr;
  if (!cfg) return MC3_E_ARG;
  mc3_instance_desc one;
  const mc3_batch_config b = single_to_batch(cfg, &one);
  return create_impl(&b, workspace, bytes, stream, out);
}

mc3_status mc3_create_noalloc(const mc3_config* cfg, void* stream, mc3_ctx** out) {
  if (out) *out = nullptr;
  if (!cfg || !out) return MC3_E_ARG;
  mc3_instance_desc one;
  const mc3_batch_config b = single_to_batch(cfg, &one);
  if (validate_batch(&b)) return MC3_E_ARG;
  size_t lds = 0;
  if (resolve_delta(b, &lds) < 0) return MC3_E_UNSUPPORTED;
  if (make_plan(b).total > (size_t)MC3_NOALLOC_BYTES) return MC3_E_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MC3_E_DEVICE;
  void* ws = nullptr;
  MC3_TRY(reserve_scratch(dev, &ws));
  const mc3_status st = create_impl(&b, ws, (size_t)MC3_NOALLOC_BYTES, stream, out, true);
  if (st != MC3_OK) {
    release_scratch(dev);
    return st;
  }
  (*out)->noalloc = true;
  return MC3_OK;
}

mc3_status mc3_destroy(mc3_ctx* ctx) {
  if (!ctx) return MC3_E_ARG;
  if (ctx->noalloc) {
    (void)hipStreamSynchronize(ctx->stream);   // the array is free once its last kernel ends
    release_scratch(ctx->device);
  }
  for (hipEvent_t e : ctx->t_start) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->t_stop) (void)hipEventDestroy(e);
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  delete ctx;
  return MC3_OK;
}

mc3_status mc3_generate_couplings(mc3_ctx* c, int32_t instance, int32_t kind, uint64_t seed) {
  MC3_TRY(usable(c));
  if (instance < 0 || instance >= (int32_t)c->pl.inst.size())
    return fail(c, MC3_E_ARG, "instance %d is not in the batch", instance);
  if (kind != MC3_J_PM1 && kind != MC3_J_GAUSS) return fail(c, MC3_E_ARG, "unknown coupling kind %d", kind);
  InstH& h = c->pl.inst[instance];
  const int N = h.desc.N, Np = h.Np;
  const double inv_sqrt_n = 1.0 / std::sqrt((double)N);
  const long long n = (long long)Np * Np;
  hipLaunchKernelGGL(mc3::k_gen_couplings, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                     c->at<double>(h.J64), N, Np, (int)kind, mc3::Key{(uint32_t)seed, (uint32_t)(seed >> 32)},
                     inv_sqrt_n);
  MC3_TRY(check_launch(c, "coupling generator"));
  return pack_couplings(c, h, kind == MC3_J_PM1 ? inv_sqrt_n : 1.0);
}

mc3_status mc3_init_couplings(mc3_ctx* c, const double* J, int64_t ld, double scale) {
  return init_couplings_impl(c, 0, J, ld, scale);
}

mc3_status mc3_init_couplings_instance(mc3_ctx* c, int32_t instance, const double* J, int64_t ld, double scale) {
  return init_couplings_impl(c, instance, J, ld, scale);
}

mc3_status mc3_init_chains(mc3_ctx* c, const int8_t* spins) {
  MC3_TRY(usable(c));
  if (!c->all_J()) return fail(c, MC3_E_STATE, "init_chains before init_couplings of every instance");
  const Plan& pl = c->pl;
  if (spins) {
    size_t off = 0;
    std::vector<uint32_t> bits;
    for (const InstH& h : pl.inst) {
      bits.assign((size_t)h.desc.chains * h.W, 0u);
      for (int ch = 0; ch < h.desc.chains; ++ch)
        for (int i = 0; i < h.desc.N; ++i) {
          const int8_t v = spins[off + (size_t)ch * h.desc.N + i];
          if (v != 1 && v != -1) return fail(c, MC3_E_ARG, "spin [%d][%d] is not +-1", h.chain0 + ch, i);
          if (v == -1) bits[(size_t)ch * h.W + i / 32] |= 1u << mc3::site_bit(i % 32);
        }
      off += (size_t)h.desc.chains * h.desc.N;
      MC3_TRY(hip_ok(c, hipMemcpyAsync(c->at<uint32_t>(h.spins), bits.data(), bits.size() * 4,
                                       hipMemcpyHostToDevice, c->stream), "upload spins"));
      MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "init_chains sync"));
    }
  } else {
    hipLaunchKernelGGL(mc3::k_init_spins, dim3((pl.Wmax + 63) / 64, pl.total_chains), dim3(64), 0, c->stream, c->ws,
                       c->insts(), c->chain_inst(), pl.total_chains, c->key(), c->cfg.chain_base);
    MC3_TRY(check_launch(c, "init spins kernel"));
  }
  MC3_TRY(launch_recompute(c, 0));
  MC3_TRY(reset_buffers(c));
  c->have_chains = true;
  c->have_proposal = c->have_scores = false;
  c->steps_done = 0;
  return MC3_OK;
}

mc3_status mc3_propose(mc3_ctx* c, uint32_t step) {
  MC3_TRY(usable(c));
  if (!c->have_chains) return fail(c, MC3_E_STATE, "propose before init_chains");
  MC3_TRY(no_delta(c, "mc3_propose"));
  MC3_TRY(propose_all(c, step, 1, true));
  c->have_proposal = true;
  c->have_scores = false;
  c->proposal_step = step;
  return MC3_OK;
}

mc3_status mc3_score_candidates(mc3_ctx* c, double* E_out) {
  MC3_TRY(usable(c));
  MC3_TRY(no_delta(c, "mc3_score_candidates"));
  if (!c->have_proposal) return fail(c, MC3_E_STATE, "score_candidates before propose");
  return do_score(c, E_out);
}

mc3_status mc3_select(mc3_ctx* c, uint32_t step, double beta) {
  MC3_TRY(usable(c));
  MC3_TRY(no_delta(c, "mc3_select"));
  if (!c->have_scores) return fail(c, MC3_E_STATE, "select before score_candidates");
  if (step != c->proposal_step)
    return fail(c, MC3_E_ARG, "select step %u differs from propose step %u", step, c->proposal_step);
  if (!std::isfinite(beta) || beta < 0.0) return fail(c, MC3_E_ARG, "beta must be finite and >= 0");
  return do_select(c, step, beta);
}

mc3_status mc3_select_betas(mc3_ctx* c, uint32_t step, const double* beta) {
  MC3_TRY(usable(c));
  MC3_TRY(no_delta(c, "mc3_select_betas"));
  if (!beta) return fail(c, MC3_E_ARG, "beta is NULL");
  if (!c->have_scores) return fail(c, MC3_E_STATE, "select before score_candidates");
  if (step != c->proposal_step)
    return fail(c, MC3_E_ARG, "select step %u differs from propose step %u", step, c->proposal_step);
  const size_t n = c->pl.inst.size();
  std::vector<double> tab(3 * n);
  for (size_t i = 0; i < n; ++i) {
    if (!std::isfinite(beta[i]) || beta[i] < 0.0) return fail(c, MC3_E_ARG, "beta[%zu] must be finite and >= 0", i);
    tab[3 * i] = beta[i];
    tab[3 * i + 1] = beta[i];
    tab[3 * i + 2] = 1.0;
  }
  MC3_TRY(upload_sched(c, tab));
  return do_select(c, step, 0.0, false, c->at<const double>(c->pl.sched));
}

mc3_status mc3_step_n_schedules(mc3_ctx* c, uint32_t step0, int64_t n, const mc3_schedule* sched) {
  MC3_TRY(step_args(c, step0, n, 0.0, 0.0));
  if (!sched) return fail(c, MC3_E_ARG, "sched is NULL");
  const size_t ni = c->pl.inst.size();
  std::vector<double> tab(3 * ni);
  for (size_t i = 0; i < ni; ++i) {
    const mc3_schedule& q = sched[i];
    if (!std::isfinite(q.beta0) || !std::isfinite(q.beta1) || q.beta0 < 0.0 || q.beta1 < 0.0)
      return fail(c, MC3_E_ARG, "schedule %zu: beta must be finite and >= 0", i);
    if (q.total < 0 || q.total > (int64_t(1) << 53)) return fail(c, MC3_E_ARG, "schedule %zu: bad total", i);
    tab[3 * i] = q.beta0;
    tab[3 * i + 1] = q.beta1;
    tab[3 * i + 2] = (double)q.total;
  }
  MC3_TRY(upload_sched(c, tab));
  const double* dev = c->at<const double>(c->pl.sched);
  if (c->pl.delta) return do_step_n_delta(c, step0, n, 0.0, 0.0, 1, dev);
  return do_step_n(c, step0, n, 0.0, 0.0, 1, dev);
}

mc3_status mc3_step_n(mc3_ctx* c, uint32_t step0, int64_t n, double beta0, double beta1, int64_t total) {
  MC3_TRY(step_args(c, step0, n, beta0, beta1));
  if (c->pl.delta) return do_step_n_delta(c, step0, n, beta0, beta1, total);
  return do_step_n(c, step0, n, beta0, beta1, total);
}

mc3_status mc3_step_n_graph(mc3_ctx* c, uint32_t step0, int64_t n, double beta0, double beta1, int64_t total) {
  MC3_TRY(step_args(c, step0, n, beta0, beta1));
  if (c->pl.delta) return do_step_n_delta(c, step0, n, beta0, beta1, total);
  return do_step_n_graph(c, step0, n, beta0, beta1, total);
}

mc3_status mc3_step_n_per_instance(mc3_ctx* c, uint32_t step0, int64_t n, double beta0, double beta1,
                                   int64_t total) {
  MC3_TRY(step_args(c, step0, n, beta0, beta1));
  MC3_TRY(no_delta(c, "mc3_step_n_per_instance"));
  return do_step_n_per_instance(c, step0, n, beta0, beta1, total);
}

mc3_status mc3_recompute(mc3_ctx* c) {
  MC3_TRY(usable(c));
  if (!c->have_chains) return fail(c, MC3_E_STATE, "recompute before init_chains");
  MC3_TRY(launch_recompute(c, 1));
  return hip_ok(c, hipStreamSynchronize(c->stream), "recompute sync");
}

mc3_status mc3_measure(mc3_ctx* c, double* e_cur, uint32_t* spin_bits, mc3_summary* summary) {
  MC3_TRY(usable(c));
  if (!c->have_chains) return fail(c, MC3_E_STATE, "measure before init_chains");
  const Plan& pl = c->pl;
  const size_t C = (size_t)pl.total_chains;
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "measure sync"));
  if (e_cur)
    MC3_TRY(hip_ok(c, hipMemcpy(e_cur, c->at<double>(pl.e_cur), C * 8, hipMemcpyDeviceToHost), "read energies"));
  if (spin_bits) {
    std::memset(spin_bits, 0, C * pl.Wn_max * 4);
    std::vector<uint32_t> b;
    for (const InstH& h : pl.inst) {
      b.resize((size_t)h.desc.chains * h.W);
      MC3_TRY(hip_ok(c, hipMemcpy(b.data(), c->at<uint32_t>(h.spins), b.size() * 4, hipMemcpyDeviceToHost),
                     "read spins"));
      for (int ch = 0; ch < h.desc.chains; ++ch)
        for (int w = 0; w < h.Wn; ++w)
          spin_bits[(size_t)(h.chain0 + ch) * pl.Wn_max + w] = mc3::natural_word(b[(size_t)ch * h.W + w]);
    }
  }
  if (summary) {
    std::vector<unsigned long long> mv(C), nt(C), de(C);
    std::vector<double> mm(C), dr(C);
    MC3_TRY(hip_ok(c, hipMemcpy(de.data(), c->at<char>(pl.drift_ev), C * 8, hipMemcpyDeviceToHost), "read"));
    MC3_TRY(hip_ok(c, hipMemcpy(mv.data(), c->at<char>(pl.moves), C * 8, hipMemcpyDeviceToHost), "read"));
    MC3_TRY(hip_ok(c, hipMemcpy(nt.data(), c->at<char>(pl.near), C * 8, hipMemcpyDeviceToHost), "read"));
    MC3_TRY(hip_ok(c, hipMemcpy(mm.data(), c->at<char>(pl.minm), C * 8, hipMemcpyDeviceToHost), "read"));
    MC3_TRY(hip_ok(c, hipMemcpy(dr.data(), c->at<char>(pl.drift), C * 8, hipMemcpyDeviceToHost), "read"));
    summary->steps_done = c->steps_done;
    summary->moves = 0;
    summary->near_ties = 0;
    summary->min_margin = HUGE_VAL;
    summary->max_drift = 0.0;
    summary->recomputes = c->recomputes;
    summary->drift_events = 0;
    for (size_t i = 0; i < C; ++i) {
      summary->moves += (int64_t)mv[i];
      summary->near_ties += (int64_t)nt[i];
      if (mm[i] < summary->min_margin) summary->min_margin = mm[i];
      if (!(dr[i] <= summary->max_drift)) summary->max_drift = dr[i];
      summary->drift_events += (int64_t)de[i];
    }
  }
  return MC3_OK;
}

mc3_status mc3_read_records(mc3_ctx* c, uint32_t first, int32_t n, mc3_record* out) {
  MC3_TRY(usable(c));
  const size_t C = (size_t)c->pl.total_chains;
  if (n < 0 || !out) return fail(c, MC3_E_ARG, "bad arguments");
  if (n > c->cfg.trace_steps) return fail(c, MC3_E_ARG, "more steps than the ring holds");
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "read_records sync"));
  static_assert(sizeof(mc3_record) == sizeof(mc3::Record), "record layout");
  for (int32_t i = 0; i < n; ++i) {
    const uint32_t st = first + (uint32_t)i;
    const size_t slot = (size_t)(st % (uint32_t)c->cfg.trace_steps);
    MC3_TRY(hip_ok(c, hipMemcpy(out + (size_t)i * C, c->at<mc3::Record>(c->pl.ring) + slot * C,
                                C * sizeof(mc3_record), hipMemcpyDeviceToHost), "read ring"));
    for (size_t ch = 0; ch < C; ++ch)
      if (out[(size_t)i * C + ch].step != st) return fail(c, MC3_E_ARG, "step %u is not in the ring", st);
  }
  return MC3_OK;
}

mc3_status mc3_read_candidates(mc3_ctx* c, uint32_t* bits, int32_t* roots) {
  MC3_TRY(usable(c));
  MC3_TRY(no_delta(c, "mc3_read_candidates"));
  if (!c->have_proposal) return fail(c, MC3_E_STATE, "no proposal to read");
  if (c->pl.inst.size() != 1) return fail(c, MC3_E_UNSUPPORTED, "read_candidates needs a single-instance context");
  const InstH& h = c->pl.inst[0];
  const uint32_t st = c->proposal_step;
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "read_candidates sync"));
  if (bits) {
    hipLaunchKernelGGL(mc3::k_build_candidates, dim3(h.Bp / 256, h.W), dim3(256), 0, c->stream,
                       c->at<uint32_t>(c->pl.candT), c->at<const uint32_t>(h.flips + c->slot(st) * h.flip_slot),
                       c->at<const uint32_t>(h.base[st & 1u]), c->roots(st) + h.chain0, h.desc.chains, h.desc.M, h.W,
                       h.Bp);
    MC3_TRY(check_launch(c, "candidate kernel"));
    MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "read_candidates sync"));
    std::vector<uint32_t> t((size_t)h.W * h.Bp);
    MC3_TRY(hip_ok(c, hipMemcpy(t.data(), c->at<uint32_t>(c->pl.candT), t.size() * 4, hipMemcpyDeviceToHost),
                   "read"));
    for (int col = 0; col < h.B; ++col)
      for (int w = 0; w < h.Wn; ++w) bits[(size_t)col * h.Wn + w] = mc3::natural_word(t[(size_t)w * h.Bp + col]);
  }
  if (roots)
    MC3_TRY(hip_ok(c, hipMemcpy(roots, c->roots(st) + h.chain0, (size_t)h.desc.chains * 4, hipMemcpyDeviceToHost),
                   "read roots"));
  return MC3_OK;
}

mc3_status mc3_timing_enable(mc3_ctx* c, int32_t on) {
  MC3_TRY(usable(c));
  if (on < 0) return fail(c, MC3_E_ARG, "timing period must be >= 0");
  if (on && c->t_start.empty()) {
    const size_t n = 256;
    c->t_start.assign(n, nullptr);
    c->t_stop.assign(n, nullptr);
    c->t_pending.assign(n, 0);
    for (size_t i = 0; i < n; ++i) {
      // timestamps only: no system-scope cache writeback and invalidation at each record
      MC3_TRY(hip_ok(c, hipEventCreateWithFlags(&c->t_start[i], hipEventDisableSystemFence), "timing events"));
      MC3_TRY(hip_ok(c, hipEventCreateWithFlags(&c->t_stop[i], hipEventDisableSystemFence), "timing events"));
    }
  }
  if (on) {
    for (size_t i = 0; i < c->t_pending.size(); ++i) c->t_pending[i] = 0;
    c->t_total_ms = 0.0;
    c->t_count = 0;
    c->t_every = on;
    c->t_seen = 0;
  }
  c->timing = on != 0;
  return MC3_OK;
}

mc3_status mc3_timing_read(mc3_ctx* c, double* total_ms, int64_t* launches) {
  MC3_TRY(usable(c));
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "timing sync"));
  for (size_t i = 0; i < c->t_pending.size(); ++i) MC3_TRY(timing_collect(c, i));
  if (total_ms) *total_ms = c->t_total_ms;
  if (launches) *launches = c->t_count;
  return MC3_OK;
}

mc3_status mc3_read_means(mc3_ctx* c, uint32_t first, int32_t n, double* out) {
  MC3_TRY(usable(c));
  if (n < 0 || !out) return fail(c, MC3_E_ARG, "bad arguments");
  if (n > c->cfg.mean_steps) return fail(c, MC3_E_ARG, "more steps than the trace holds");
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "read_means sync"));
  std::vector<double> buf((size_t)c->cfg.mean_steps * 3);
  MC3_TRY(hip_ok(c, hipMemcpy(buf.data(), c->at<double>(c->pl.means), buf.size() * 8, hipMemcpyDeviceToHost),
                 "read means"));
  for (int32_t i = 0; i < n; ++i) {
    const uint32_t st = first + (uint32_t)i;
    const size_t slot = st % (uint32_t)c->cfg.mean_steps;
    if (buf[3 * slot] != (double)st) return fail(c, MC3_E_ARG, "step %u is not in the trace", st);
    out[2 * (size_t)i] = buf[3 * slot + 1];
    out[2 * (size_t)i + 1] = buf[3 * slot + 2];
  }
  return MC3_OK;
}

// Checkpoint layout: header, one shape record per instance, then the arrays in a
// fixed order (see checkpoint_items).
struct CkHeader {
  char magic[8];
  uint32_t version;
  int32_t n_instances, total_chains, delta;
  int64_t steps_done, recomputes;
  uint64_t payload;
};
struct CkShape {
  int32_t N, M, chains, W;
};

}  // extern "C"

namespace {

// (device pointer, bytes) of every array a checkpoint carries, in order.
std::vector<std::pair<char*, size_t>> checkpoint_items(mc3_ctx* c) {
  const Plan& pl = c->pl;
  const size_t C = (size_t)pl.total_chains;
  std::vector<std::pair<char*, size_t>> it;
  it.emplace_back(c->at<char>(pl.e_cur), C * 8);
  it.emplace_back(c->at<char>(pl.u_cur), C * 8);
  it.emplace_back(c->at<char>(pl.drift_ev), C * 8);
  it.emplace_back(c->at<char>(pl.moves), C * 8);
  it.emplace_back(c->at<char>(pl.near), C * 8);
  it.emplace_back(c->at<char>(pl.minm), C * 8);
  it.emplace_back(c->at<char>(pl.drift), C * 8);
  for (const InstH& h : pl.inst) {
    it.emplace_back(c->at<char>(h.spins), (size_t)h.desc.chains * h.W * 4);
    if (pl.delta) it.emplace_back(c->at<char>(h.field), (size_t)h.desc.chains * h.Np * 8);
  }
  return it;
}

size_t checkpoint_bytes(mc3_ctx* c) {
  size_t n = sizeof(CkHeader) + c->pl.inst.size() * sizeof(CkShape);
  for (const auto& x : checkpoint_items(c)) n += x.second;
  return n;
}

}  // namespace

extern "C" {

mc3_status mc3_checkpoint_save(mc3_ctx* c, void* buf, size_t* bytes) {
  MC3_TRY(usable(c));
  if (!bytes) return fail(c, MC3_E_ARG, "bytes is NULL");
  const size_t need = checkpoint_bytes(c);
  if (!buf) {
    *bytes = need;
    return MC3_OK;
  }
  if (*bytes < need) return fail(c, MC3_E_ARG, "checkpoint needs %zu bytes", need);
  if (!c->have_chains) return fail(c, MC3_E_STATE, "checkpoint_save before init_chains");
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "checkpoint sync"));
  char* p = (char*)buf;
  CkHeader hd;
  std::memset(&hd, 0, sizeof hd);
  std::memcpy(hd.magic, "MC3CKPT1", 8);
  hd.version = 2;
  hd.n_instances = (int32_t)c->pl.inst.size();
  hd.total_chains = c->pl.total_chains;
  hd.delta = c->pl.delta ? 1 : 0;
  hd.steps_done = c->steps_done;
  hd.recomputes = c->recomputes;
  hd.payload = need - sizeof hd;
  std::memcpy(p, &hd, sizeof hd);
  p += sizeof hd;
  for (const InstH& h : c->pl.inst) {
    const CkShape sh{h.desc.N, h.desc.M, h.desc.chains, h.W};
    std::memcpy(p, &sh, sizeof sh);
    p += sizeof sh;
  }
  for (const auto& x : checkpoint_items(c)) {
    MC3_TRY(hip_ok(c, hipMemcpy(p, x.first, x.second, hipMemcpyDeviceToHost), "checkpoint read"));
    p += x.second;
  }
  *bytes = need;
  return MC3_OK;
}

mc3_status mc3_checkpoint_load(mc3_ctx* c, const void* buf, size_t bytes) {
  MC3_TRY(usable(c));
  if (!buf) return fail(c, MC3_E_ARG, "buf is NULL");
  if (!c->all_J()) return fail(c, MC3_E_STATE, "checkpoint_load before init_couplings of every instance");
  const size_t need = checkpoint_bytes(c);
  if (bytes < need) return fail(c, MC3_E_ARG, "checkpoint is %zu bytes, this context needs %zu", bytes, need);
  const char* p = (const char*)buf;
  CkHeader hd;
  std::memcpy(&hd, p, sizeof hd);
  p += sizeof hd;
  if (std::memcmp(hd.magic, "MC3CKPT1", 8) != 0 || hd.version != 2) return fail(c, MC3_E_ARG, "not a checkpoint");
  if (hd.n_instances != (int32_t)c->pl.inst.size() || hd.total_chains != c->pl.total_chains ||
      hd.delta != (c->pl.delta ? 1 : 0) || hd.payload != need - sizeof hd)
    return fail(c, MC3_E_ARG, "checkpoint of a different batch shape or scorer");
  for (const InstH& h : c->pl.inst) {
    CkShape sh;
    std::memcpy(&sh, p, sizeof sh);
    p += sizeof sh;
    if (sh.N != h.desc.N || sh.M != h.desc.M || sh.chains != h.desc.chains || sh.W != h.W)
      return fail(c, MC3_E_ARG, "checkpoint of a different instance shape");
  }
  MC3_TRY(reset_buffers(c));
  for (const auto& x : checkpoint_items(c)) {
    MC3_TRY(hip_ok(c, hipMemcpy(x.first, p, x.second, hipMemcpyHostToDevice), "checkpoint write"));
    p += x.second;
  }
  c->have_chains = true;
  c->have_proposal = c->have_scores = false;
  c->steps_done = hd.steps_done;
  c->recomputes = hd.recomputes;
  return MC3_OK;
}

mc3_status mc3_sync(mc3_ctx* c) {
  MC3_TRY(usable(c));
  return hip_ok(c, hipStreamSynchronize(c->stream), "sync");
}

const char* mc3_last_error(const mc3_ctx* c) { return c ? c->err.c_str() : "context is NULL"; }

mc3_status mc3_set_generation(const double* G, int32_t n, int32_t n_sets, double* out, const double* peq,
                              double* psub, double* peq_set, void* stream) {
  if (!G || !out || n < 1 || n > 20 || n_sets < 1 || ((int64_t)n_sets << n) > (int64_t(1) << 28)) return MC3_E_ARG;
  if ((peq != nullptr) != (psub != nullptr) || (peq != nullptr) != (peq_set != nullptr)) return MC3_E_ARG;
  for (const void* ptr : {(const void*)G, (const void*)out, (const void*)peq, (const void*)psub,
                          (const void*)peq_set}) {
    if (!ptr) continue;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, ptr) != hipSuccess || attr.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      return MC3_E_ARG;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  const unsigned masks = (1u << n);
  const dim3 grid((masks + 255) / 256, (unsigned)n_sets);
  auto binom = [](int b, int j) {
    uint64_t c = 1;
    for (int i = 0; i < j; ++i) c = c * (uint64_t)(b - i) / (uint64_t)(i + 1);
    return (unsigned)c;
  };
  if (n <= mc3::kSetLdsMax) {
    hipLaunchKernelGGL(mc3::k_set_gen_lds, dim3((unsigned)n_sets), dim3(256), 0, st, G, out, n);
  } else {
    hipLaunchKernelGGL(mc3::k_set_gen_ends, dim3((n_sets + 255) / 256), dim3(256), 0, st, out, n, n_sets);
    for (int k = n - 1; k >= 1; --k)
      hipLaunchKernelGGL(mc3::k_set_gen_level, dim3((binom(n, k) + 255) / 256, (unsigned)n_sets), dim3(256), 0, st,
                         G, out, n, k);
  }
  if (peq) {
    hipLaunchKernelGGL(mc3::k_set_peq, dim3((unsigned)n_sets), dim3(256), 0, st, peq, out, peq_set, n);
    hipLaunchKernelGGL(mc3::k_set_psub, grid, dim3(256), 0, st, peq, out, peq_set, psub, n);
  }
  return hipGetLastError() == hipSuccess ? MC3_OK : MC3_E_DEVICE;
}

}  // extern "C"
