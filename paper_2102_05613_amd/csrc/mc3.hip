// mc3.hip -- C ABI of the MI355X MCMCMC hot path for the SK spin glass.
// The declarations and their contracts are in include/mc3.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mc3.h"
#include "kernels.hpp"

namespace {

constexpr size_t kAlign = 256;
constexpr int kColTile = 512;  // candidate columns are padded to this (split tile width)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Dims {
  int N, M, chains, Np, W, Wn, B, Bp, NB, P;
};

Dims dims_of(const mc3_config& c) {
  Dims d;
  d.N = c.N;
  d.M = c.M;
  d.chains = c.chains;
  d.Np = (c.N + mc3::kRowBlock - 1) / mc3::kRowBlock * mc3::kRowBlock;
  d.W = d.Np / 32;
  d.Wn = (c.N + 31) / 32;
  d.B = c.chains * c.M;
  d.Bp = (d.B + kColTile - 1) / kColTile * kColTile;
  d.NB = d.Np / mc3::kRowBlock;
  d.P = (d.NB + 1) / 2;
  return d;
}

struct Layout {
  size_t J64, Jpack, spins, e_cur, e_bar, flips, roots, base, candT, partial, Ecol, ring, means, moves, near, minm,
      drift, erecomp, total;
};

Layout layout_of(const mc3_config& c) {
  const Dims d = dims_of(c);
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, kAlign);
    return at;
  };
  L.J64 = take((size_t)d.Np * d.Np * sizeof(double));
  if (c.precision == MC3_SPLIT_BF16)
    L.Jpack = take((size_t)d.Np * d.Np * 3 * sizeof(uint16_t));
  else
    L.Jpack = take((size_t)d.Np * d.Np * sizeof(double));
  L.spins = take((size_t)d.chains * d.W * 4);
  L.e_cur = take((size_t)d.chains * 8);
  L.e_bar = take((size_t)d.chains * 8);
  L.flips = take((size_t)2 * d.W * d.Bp * 4);           // two steps (by parity)
  L.roots = take((size_t)2 * d.chains * 4);
  L.base = take((size_t)2 * (d.chains + 1) * d.W * 4);
  L.candT = take((size_t)d.W * d.Bp * 4);
  L.partial = take((size_t)d.P * d.Bp * 8);
  L.Ecol = take((size_t)d.Bp * 8);
  L.ring = take((size_t)(c.trace_steps > 0 ? c.trace_steps : 0) * d.chains * sizeof(mc3::Record));
  L.means = take((size_t)(c.mean_steps > 0 ? c.mean_steps : 0) * 3 * sizeof(double));
  L.moves = take((size_t)d.chains * 8);
  L.near = take((size_t)d.chains * 8);
  L.minm = take((size_t)d.chains * 8);
  L.drift = take((size_t)d.chains * 8);
  L.erecomp = take((size_t)d.chains * 8);
  L.total = o;
  return L;
}

const char* validate(const mc3_config* c) {
  if (!c) return "config is NULL";
  if (c->N < 2 || c->N > 8192) return "N must be in [2, 8192]";
  if (c->M < 1 || c->M > 4000) return "M must be in [1, 4000]";
  if (c->chains < 1) return "chains must be >= 1";
  if ((long long)c->chains * c->M > (1ll << 24)) return "chains * M must be <= 2^24";
  if ((long long)c->chains + c->chain_base > (1ll << 28)) return "chain_base + chains must be <= 2^28";
  if (c->kmin < 1 || c->kmax < c->kmin || c->kmax > c->N) return "need 1 <= kmin <= kmax <= N";
  if (c->precision != MC3_FP64 && c->precision != MC3_SPLIT_BF16) return "unknown precision";
  if (c->rule != MC3_RULE_MCMCMC && c->rule != MC3_RULE_METROPOLIS) return "unknown rule";
  if (c->rule == MC3_RULE_METROPOLIS && c->M != 1) return "rule METROPOLIS requires M == 1";
  if (c->trace_steps < 0) return "trace_steps must be >= 0";
  if (c->mean_steps < 0) return "mean_steps must be >= 0";
  if (!(c->near_tie_tol == c->near_tie_tol)) return "near_tie_tol is NaN";
  return nullptr;
}

}  // namespace

struct mc3_ctx {
  mc3_config cfg;
  Dims d;
  Layout L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t aux = nullptr;          // proposals of the next step run here, overlapping scoring
  hipEvent_t ev_prop[2] = {nullptr, nullptr}, ev_sel[2] = {nullptr, nullptr};
  int device = 0;
  bool have_J = false, have_chains = false, have_proposal = false, have_scores = false, poisoned = false;
  uint32_t proposal_step = 0;
  double scale = 1.0;
  double tol = 0.0;
  int64_t steps_done = 0;
  int split_cf = 2;  // split scoring tile: 32*split_cf columns per wave (2 or 4)
  // optional HIP-event timing of the scoring launches
  bool timing = false;
  std::vector<hipEvent_t> t_start, t_stop;
  std::vector<char> t_pending;
  size_t t_next = 0;
  double t_total_ms = 0.0;
  int64_t t_count = 0;
  std::string err;

  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  uint32_t* flips(uint32_t step) const { return at<uint32_t>(L.flips) + (size_t)(step & 1u) * d.W * d.Bp; }
  int32_t* roots(uint32_t step) const { return at<int32_t>(L.roots) + (size_t)(step & 1u) * d.chains; }
  uint32_t* base(uint32_t step) const { return at<uint32_t>(L.base) + (size_t)(step & 1u) * (d.chains + 1) * d.W; }
  mc3::Key key() const { return mc3::Key{(uint32_t)cfg.seed, (uint32_t)(cfg.seed >> 32)}; }
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

#define MC3_TRY(expr)              \
  do {                             \
    mc3_status _s = (expr);        \
    if (_s != MC3_OK) return _s;   \
  } while (0)

mc3_status usable(mc3_ctx* c) {
  if (!c) return MC3_E_ARG;
  if (c->poisoned) return fail(c, MC3_E_STATE, "context poisoned by an earlier device error");
  c->err.clear();
  return MC3_OK;
}

mc3_status launch_energy(mc3_ctx* c, double* out) {
  hipLaunchKernelGGL(mc3::k_energy_f64, dim3(c->d.chains), dim3(256), 0, c->stream, out,
                     c->at<uint32_t>(c->L.spins), c->at<double>(c->L.J64), c->d.N, c->d.Np, c->d.W, c->scale);
  return check_launch(c, "energy kernel");
}

mc3_status launch_propose(mc3_ctx* c, uint32_t step, hipStream_t st, bool write_base) {
  const Dims& d = c->d;
  int stride = d.W + 1;
  int T = (int)(65536 / ((size_t)stride * 4));
  if (T < 64) {
    stride = d.W;
    T = (int)(65536 / ((size_t)stride * 4));
  }
  if (T > 256) T = 256;
  T = (T / 64) * 64;
  const size_t lds = (size_t)T * stride * 4;
  const long long total = (long long)d.chains * d.M;
  const int blocks = (int)((total + T - 1) / T);
  hipLaunchKernelGGL(mc3::k_propose, dim3(blocks), dim3(T), lds, st, c->flips(step), c->roots(step), c->base(step),
                     c->at<const uint32_t>(c->L.spins), write_base ? 1 : 0, d.chains, d.M, d.N, d.W, d.Bp, stride,
                     c->cfg.kmin, c->cfg.kmax, c->cfg.rule == MC3_RULE_METROPOLIS ? 1 : 0, c->key(),
                     c->cfg.chain_base, step);
  return check_launch(c, "propose kernel");
}

mc3_status do_propose(mc3_ctx* c, uint32_t step) {
  MC3_TRY(launch_propose(c, step, c->stream, true));
  c->have_proposal = true;
  c->have_scores = false;
  c->proposal_step = step;
  return MC3_OK;
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

mc3_status launch_score_kernel(mc3_ctx* c);

mc3_status do_score(mc3_ctx* c, double* E_out) {
  const Dims& d = c->d;
  if (c->timing) {
    const size_t i = c->t_next;
    c->t_next = (c->t_next + 1) % c->t_start.size();
    MC3_TRY(timing_collect(c, i));
    MC3_TRY(hip_ok(c, hipEventRecord(c->t_start[i], c->stream), "timing event"));
    MC3_TRY(launch_score_kernel(c));
    MC3_TRY(hip_ok(c, hipEventRecord(c->t_stop[i], c->stream), "timing event"));
    c->t_pending[i] = 1;
  } else {
    MC3_TRY(launch_score_kernel(c));
  }
  if (E_out) {
    hipLaunchKernelGGL(mc3::k_column_energies, dim3((d.B + 255) / 256), dim3(256), 0, c->stream,
                       c->at<double>(c->L.Ecol), c->at<const double>(c->L.partial), d.P, d.Bp, d.B, c->scale);
    MC3_TRY(check_launch(c, "column energy kernel"));
    MC3_TRY(hip_ok(c, hipMemcpyAsync(E_out, c->at<double>(c->L.Ecol), (size_t)d.B * 8, hipMemcpyDeviceToDevice,
                                     c->stream), "copy energies"));
  }
  c->have_scores = true;
  return MC3_OK;
}

mc3_status launch_score_kernel(mc3_ctx* c) {
  const Dims& d = c->d;
  const uint32_t t = c->proposal_step;
  if (c->cfg.precision == MC3_SPLIT_BF16) {
    const int TN = 128 * c->split_cf;
    const int CT = d.Bp / TN;
    const int U = d.P * CT;
    const int grid = 8 * ((U + 7) / 8);
    if (c->split_cf == 4)
      hipLaunchKernelGGL(mc3::k_score_split<4>, dim3(grid), dim3(256), 0, c->stream, c->at<const uint4>(c->L.Jpack),
                         c->flips(t), c->base(t), c->roots(t), c->at<double>(c->L.partial), d.chains, d.M, d.Np,
                         d.Bp, d.NB, d.P, CT);
    else
      hipLaunchKernelGGL(mc3::k_score_split<2>, dim3(grid), dim3(256), 0, c->stream, c->at<const uint4>(c->L.Jpack),
                         c->flips(t), c->base(t), c->roots(t), c->at<double>(c->L.partial), d.chains, d.M, d.Np,
                         d.Bp, d.NB, d.P, CT);
  } else {
    const int CT = d.Bp / 128;
    const int U = d.P * CT;
    const int grid = 8 * ((U + 7) / 8);
    hipLaunchKernelGGL(mc3::k_score_f64, dim3(grid), dim3(256), 0, c->stream, c->at<const double>(c->L.Jpack),
                       c->flips(t), c->base(t), c->roots(t), c->at<double>(c->L.partial), d.chains, d.M, d.Np, d.Bp,
                       d.NB, d.P, CT);
  }
  return check_launch(c, "score kernel");
}

// Selection of step `step`; with next_base, also the base words of step+1 (whose
// flip sets and roots must already be proposed).
mc3_status do_select(mc3_ctx* c, uint32_t step, double beta, bool next_base = false) {
  const Dims& d = c->d;
  const size_t lds = (size_t)(d.M + 1) * 16 + (size_t)d.W * 4;
  hipLaunchKernelGGL(mc3::k_select, dim3(d.chains), dim3(256), lds, c->stream, c->at<uint32_t>(c->L.spins),
                     c->at<double>(c->L.e_cur), c->flips(step), c->base(step), c->at<const double>(c->L.partial), d.P,
                     c->scale, c->roots(step), c->at<mc3::Record>(c->L.ring), c->at<unsigned long long>(c->L.moves),
                     c->at<unsigned long long>(c->L.near), c->at<double>(c->L.minm), c->at<double>(c->L.e_bar),
                     d.chains, d.M, d.W, d.Bp, c->cfg.rule == MC3_RULE_METROPOLIS ? 1 : 0, beta, c->tol, c->key(),
                     c->cfg.chain_base, step, c->cfg.trace_steps, next_base ? 1 : 0, c->flips(step + 1u),
                     c->roots(step + 1u), c->base(step + 1u));
  MC3_TRY(check_launch(c, "select kernel"));
  if (c->cfg.mean_steps > 0) {
    hipLaunchKernelGGL(mc3::k_chain_means, dim3(1), dim3(256), 0, c->stream, c->at<double>(c->L.means),
                       c->at<const double>(c->L.e_cur), c->at<const double>(c->L.e_bar), d.chains,
                       step % (uint32_t)c->cfg.mean_steps, step);
    MC3_TRY(check_launch(c, "means kernel"));
  }
  c->have_proposal = next_base;
  c->have_scores = false;
  if (next_base) c->proposal_step = step + 1u;
  c->steps_done += 1;
  return MC3_OK;
}

double beta_at(uint32_t t, double beta0, double beta1, int64_t total) {
  if (total <= 1) return beta0;
  return beta0 + (beta1 - beta0) * ((double)t / (double)(total - 1));
}

// n steps with the proposal of step t+1 on the auxiliary stream, overlapping the
// scoring of step t; the selection of step t also forms the base words of step t+1.
// Flip sets, roots and base words are double-buffered by step parity: propose(t+1)
// waits for select(t-1) (the last reader of its buffers); select(t) waits for
// propose(t+1).  Everything joins back into the caller's stream.
mc3_status do_step_n(mc3_ctx* c, uint32_t step0, int64_t n, double beta0, double beta1, int64_t total) {
  if (n <= 0) return MC3_OK;
  MC3_TRY(hip_ok(c, hipEventRecord(c->ev_sel[0], c->stream), "event"));
  MC3_TRY(hip_ok(c, hipEventRecord(c->ev_sel[1], c->stream), "event"));
  MC3_TRY(hip_ok(c, hipStreamWaitEvent(c->aux, c->ev_sel[step0 & 1u], 0), "wait"));
  MC3_TRY(launch_propose(c, step0, c->aux, true));
  MC3_TRY(hip_ok(c, hipEventRecord(c->ev_prop[step0 & 1u], c->aux), "event"));
  MC3_TRY(hip_ok(c, hipStreamWaitEvent(c->stream, c->ev_prop[step0 & 1u], 0), "wait"));
  c->have_proposal = true;
  c->proposal_step = step0;
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t t = step0 + (uint32_t)i;
    const bool last = i + 1 == n;
    if (!last) {
      const uint32_t t1 = t + 1u;
      MC3_TRY(hip_ok(c, hipStreamWaitEvent(c->aux, c->ev_sel[t1 & 1u], 0), "wait"));
      MC3_TRY(launch_propose(c, t1, c->aux, false));
      MC3_TRY(hip_ok(c, hipEventRecord(c->ev_prop[t1 & 1u], c->aux), "event"));
    }
    MC3_TRY(do_score(c, nullptr));
    if (!last) MC3_TRY(hip_ok(c, hipStreamWaitEvent(c->stream, c->ev_prop[(t + 1u) & 1u], 0), "wait"));
    MC3_TRY(do_select(c, t, beta_at(t, beta0, beta1, total), !last));
    MC3_TRY(hip_ok(c, hipEventRecord(c->ev_sel[t & 1u], c->stream), "event"));
  }
  c->have_proposal = false;
  return MC3_OK;
}

}  // namespace

extern "C" {

const char* mc3_version(void) { return "mc3 0.1 (gfx950)"; }

mc3_status mc3_workspace_size(const mc3_config* cfg, size_t* bytes) {
  if (validate(cfg) || !bytes) return MC3_E_ARG;
  *bytes = layout_of(*cfg).total;
  return MC3_OK;
}

mc3_status mc3_create(const mc3_config* cfg, void* workspace, size_t bytes, void* stream, mc3_ctx** out) {
  if (!out) return MC3_E_ARG;
  *out = nullptr;
  if (validate(cfg)) return MC3_E_ARG;
  const Layout L = layout_of(*cfg);
  if (!workspace || bytes < L.total || ((uintptr_t)workspace % kAlign) != 0) return MC3_E_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MC3_E_DEVICE;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, workspace) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return MC3_E_WORKSPACE;
  }
  mc3_ctx* c = new (std::nothrow) mc3_ctx();
  if (!c) return MC3_E_ARG;
  c->cfg = *cfg;
  c->d = dims_of(*cfg);
  c->L = L;
  c->ws = (char*)workspace;
  c->stream = (hipStream_t)stream;
  c->device = dev;
  bool ok = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i < 2 && ok; ++i) {
    ok = hipEventCreateWithFlags(&c->ev_prop[i], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&c->ev_sel[i], hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    mc3_destroy(c);
    return MC3_E_DEVICE;
  }
  if (const char* e = std::getenv("MC3_SPLIT_CF")) {
    if (std::strcmp(e, "4") == 0) c->split_cf = 4;
  }
  if (cfg->near_tie_tol >= 0.0)
    c->tol = cfg->near_tie_tol;
  else
    c->tol = cfg->precision == MC3_SPLIT_BF16 ? 1e-4 : 1e-9;
  *out = c;
  return MC3_OK;
}

mc3_status mc3_destroy(mc3_ctx* ctx) {
  if (!ctx) return MC3_E_ARG;
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  for (int i = 0; i < 2; ++i) {
    if (ctx->ev_prop[i]) (void)hipEventDestroy(ctx->ev_prop[i]);
    if (ctx->ev_sel[i]) (void)hipEventDestroy(ctx->ev_sel[i]);
  }
  for (hipEvent_t e : ctx->t_start) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->t_stop) (void)hipEventDestroy(e);
  delete ctx;
  return MC3_OK;
}

mc3_status mc3_init_couplings(mc3_ctx* c, const double* J, int64_t ld, double scale) {
  MC3_TRY(usable(c));
  const Dims& d = c->d;
  if (!J || ld < d.N) return fail(c, MC3_E_ARG, "J is NULL or ld < N");
  if (!std::isfinite(scale)) return fail(c, MC3_E_NUMERIC, "scale is not finite");
  for (int i = 0; i < d.N; ++i)
    for (int j = i + 1; j < d.N; ++j)
      if (!std::isfinite(J[(size_t)i * ld + j])) return fail(c, MC3_E_NUMERIC, "J[%d][%d] is not finite", i, j);
  double* J64 = c->at<double>(c->L.J64);
  MC3_TRY(hip_ok(c, hipMemsetAsync(J64, 0, (size_t)d.Np * d.Np * 8, c->stream), "clear J"));
  MC3_TRY(hip_ok(c, hipMemcpy2DAsync(J64, (size_t)d.Np * 8, J, (size_t)ld * 8, (size_t)d.N * 8, d.N,
                                     hipMemcpyHostToDevice, c->stream), "upload J"));
  if (c->cfg.precision == MC3_SPLIT_BF16) {
    const long long n = (long long)(d.Np / 32) * (d.Np / 16) * 64;
    hipLaunchKernelGGL(mc3::k_pack_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       c->at<uint4>(c->L.Jpack), J64, d.Np);
  } else {
    const long long n = (long long)(d.Np / 16) * (d.Np / 4) * 64;
    hipLaunchKernelGGL(mc3::k_pack_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       c->at<double>(c->L.Jpack), J64, d.Np);
  }
  MC3_TRY(check_launch(c, "pack kernel"));
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "init_couplings sync"));
  c->scale = scale;
  c->have_J = true;
  c->have_chains = false;
  return MC3_OK;
}

mc3_status mc3_init_chains(mc3_ctx* c, const int8_t* spins) {
  MC3_TRY(usable(c));
  if (!c->have_J) return fail(c, MC3_E_STATE, "init_chains before init_couplings");
  const Dims& d = c->d;
  uint32_t* sp = c->at<uint32_t>(c->L.spins);
  if (spins) {
    std::vector<uint32_t> bits((size_t)d.chains * d.W, 0u);
    for (int ch = 0; ch < d.chains; ++ch)
      for (int i = 0; i < d.N; ++i) {
        const int8_t v = spins[(size_t)ch * d.N + i];
        if (v != 1 && v != -1) return fail(c, MC3_E_ARG, "spin [%d][%d] is not +-1", ch, i);
        if (v == -1) bits[(size_t)ch * d.W + i / 32] |= 1u << (i % 32);
      }
    MC3_TRY(hip_ok(c, hipMemcpyAsync(sp, bits.data(), bits.size() * 4, hipMemcpyHostToDevice, c->stream),
                   "upload spins"));
    MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "init_chains sync"));
  } else {
    hipLaunchKernelGGL(mc3::k_init_spins, dim3((d.W + 63) / 64, d.chains), dim3(64), 0, c->stream, sp, d.chains, d.N,
                       d.W, c->key(), c->cfg.chain_base);
    MC3_TRY(check_launch(c, "init spins kernel"));
  }
  MC3_TRY(launch_energy(c, c->at<double>(c->L.e_cur)));
  // flip-set padding columns and the zero base row must read as zero
  MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(c->L.flips), 0, (size_t)2 * d.W * d.Bp * 4, c->stream), "clear"));
  MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(c->L.base), 0, (size_t)2 * (d.chains + 1) * d.W * 4, c->stream),
                 "clear"));
  MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(c->L.moves), 0, (size_t)d.chains * 8, c->stream), "clear"));
  MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(c->L.near), 0, (size_t)d.chains * 8, c->stream), "clear"));
  MC3_TRY(hip_ok(c, hipMemsetAsync(c->at<char>(c->L.drift), 0, (size_t)d.chains * 8, c->stream), "clear"));
  {
    std::vector<double> big((size_t)d.chains, HUGE_VAL);
    MC3_TRY(hip_ok(c, hipMemcpyAsync(c->at<double>(c->L.minm), big.data(), big.size() * 8, hipMemcpyHostToDevice,
                                     c->stream), "init margins"));
    MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "init_chains sync"));
  }
  if (c->cfg.trace_steps > 0) {
    std::vector<mc3::Record> ring((size_t)c->cfg.trace_steps * d.chains);
    for (auto& r : ring) {
      std::memset(&r, 0, sizeof r);
      r.step = 0xFFFFFFFFu;
    }
    MC3_TRY(hip_ok(c, hipMemcpyAsync(c->at<mc3::Record>(c->L.ring), ring.data(), ring.size() * sizeof(mc3::Record),
                                     hipMemcpyHostToDevice, c->stream), "clear ring"));
    MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "init_chains sync"));
  }
  if (c->cfg.mean_steps > 0) {
    std::vector<double> tr((size_t)c->cfg.mean_steps * 3, -1.0);
    MC3_TRY(hip_ok(c, hipMemcpyAsync(c->at<double>(c->L.means), tr.data(), tr.size() * 8, hipMemcpyHostToDevice,
                                     c->stream), "clear means"));
    MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "init_chains sync"));
  }
  c->have_chains = true;
  c->have_proposal = c->have_scores = false;
  c->steps_done = 0;
  return MC3_OK;
}

mc3_status mc3_propose(mc3_ctx* c, uint32_t step) {
  MC3_TRY(usable(c));
  if (!c->have_chains) return fail(c, MC3_E_STATE, "propose before init_chains");
  return do_propose(c, step);
}

mc3_status mc3_score_candidates(mc3_ctx* c, double* E_out) {
  MC3_TRY(usable(c));
  if (!c->have_proposal) return fail(c, MC3_E_STATE, "score_candidates before propose");
  return do_score(c, E_out);
}

mc3_status mc3_select(mc3_ctx* c, uint32_t step, double beta) {
  MC3_TRY(usable(c));
  if (!c->have_scores) return fail(c, MC3_E_STATE, "select before score_candidates");
  if (step != c->proposal_step) return fail(c, MC3_E_ARG, "select step %u differs from propose step %u", step,
                                            c->proposal_step);
  if (!std::isfinite(beta) || beta < 0.0) return fail(c, MC3_E_ARG, "beta must be finite and >= 0");
  return do_select(c, step, beta);
}

mc3_status mc3_step_n(mc3_ctx* c, uint32_t step0, int64_t n, double beta0, double beta1, int64_t total) {
  MC3_TRY(usable(c));
  if (!c->have_chains) return fail(c, MC3_E_STATE, "step_n before init_chains");
  if (n < 0 || (uint64_t)step0 + (uint64_t)n > 0x100000000ull) return fail(c, MC3_E_ARG, "bad step range");
  if (!std::isfinite(beta0) || !std::isfinite(beta1) || beta0 < 0.0 || beta1 < 0.0)
    return fail(c, MC3_E_ARG, "beta must be finite and >= 0");
  return do_step_n(c, step0, n, beta0, beta1, total);
}

mc3_status mc3_recompute(mc3_ctx* c) {
  MC3_TRY(usable(c));
  if (!c->have_chains) return fail(c, MC3_E_STATE, "recompute before init_chains");
  const Dims& d = c->d;
  MC3_TRY(launch_energy(c, c->at<double>(c->L.erecomp)));
  std::vector<double> er(d.chains), ec(d.chains), dr(d.chains);
  MC3_TRY(hip_ok(c, hipMemcpyAsync(er.data(), c->at<double>(c->L.erecomp), (size_t)d.chains * 8,
                                   hipMemcpyDeviceToHost, c->stream), "read energies"));
  MC3_TRY(hip_ok(c, hipMemcpyAsync(ec.data(), c->at<double>(c->L.e_cur), (size_t)d.chains * 8, hipMemcpyDeviceToHost,
                                   c->stream), "read energies"));
  MC3_TRY(hip_ok(c, hipMemcpyAsync(dr.data(), c->at<double>(c->L.drift), (size_t)d.chains * 8, hipMemcpyDeviceToHost,
                                   c->stream), "read drift"));
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "recompute sync"));
  for (int i = 0; i < d.chains; ++i) {
    const double x = std::fabs(ec[i] - er[i]);
    if (x > dr[i]) dr[i] = x;
  }
  MC3_TRY(hip_ok(c, hipMemcpyAsync(c->at<double>(c->L.drift), dr.data(), (size_t)d.chains * 8, hipMemcpyHostToDevice,
                                   c->stream), "write drift"));
  MC3_TRY(hip_ok(c, hipMemcpyAsync(c->at<double>(c->L.e_cur), er.data(), (size_t)d.chains * 8, hipMemcpyHostToDevice,
                                   c->stream), "write energies"));
  return hip_ok(c, hipStreamSynchronize(c->stream), "recompute sync");
}

mc3_status mc3_measure(mc3_ctx* c, double* e_cur, uint32_t* spin_bits, mc3_summary* summary) {
  MC3_TRY(usable(c));
  if (!c->have_chains) return fail(c, MC3_E_STATE, "measure before init_chains");
  const Dims& d = c->d;
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "measure sync"));
  if (e_cur)
    MC3_TRY(hip_ok(c, hipMemcpy(e_cur, c->at<double>(c->L.e_cur), (size_t)d.chains * 8, hipMemcpyDeviceToHost),
                   "read energies"));
  if (spin_bits) {
    std::vector<uint32_t> b((size_t)d.chains * d.W);
    MC3_TRY(hip_ok(c, hipMemcpy(b.data(), c->at<uint32_t>(c->L.spins), b.size() * 4, hipMemcpyDeviceToHost),
                   "read spins"));
    for (int ch = 0; ch < d.chains; ++ch)
      std::memcpy(spin_bits + (size_t)ch * d.Wn, b.data() + (size_t)ch * d.W, (size_t)d.Wn * 4);
  }
  if (summary) {
    std::vector<unsigned long long> mv(d.chains), nt(d.chains);
    std::vector<double> mm(d.chains), dr(d.chains);
    MC3_TRY(hip_ok(c, hipMemcpy(mv.data(), c->at<char>(c->L.moves), (size_t)d.chains * 8, hipMemcpyDeviceToHost), "read"));
    MC3_TRY(hip_ok(c, hipMemcpy(nt.data(), c->at<char>(c->L.near), (size_t)d.chains * 8, hipMemcpyDeviceToHost), "read"));
    MC3_TRY(hip_ok(c, hipMemcpy(mm.data(), c->at<char>(c->L.minm), (size_t)d.chains * 8, hipMemcpyDeviceToHost), "read"));
    MC3_TRY(hip_ok(c, hipMemcpy(dr.data(), c->at<char>(c->L.drift), (size_t)d.chains * 8, hipMemcpyDeviceToHost), "read"));
    summary->steps_done = c->steps_done;
    summary->moves = 0;
    summary->near_ties = 0;
    summary->min_margin = HUGE_VAL;
    summary->max_drift = 0.0;
    for (int i = 0; i < d.chains; ++i) {
      summary->moves += (int64_t)mv[i];
      summary->near_ties += (int64_t)nt[i];
      if (mm[i] < summary->min_margin) summary->min_margin = mm[i];
      if (dr[i] > summary->max_drift) summary->max_drift = dr[i];
    }
  }
  return MC3_OK;
}

mc3_status mc3_read_records(mc3_ctx* c, uint32_t first, int32_t n, mc3_record* out) {
  MC3_TRY(usable(c));
  const Dims& d = c->d;
  if (n < 0 || !out) return fail(c, MC3_E_ARG, "bad arguments");
  if (n > c->cfg.trace_steps) return fail(c, MC3_E_ARG, "more steps than the ring holds");
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "read_records sync"));
  static_assert(sizeof(mc3_record) == sizeof(mc3::Record), "record layout");
  for (int32_t i = 0; i < n; ++i) {
    const uint32_t st = first + (uint32_t)i;
    const size_t slot = (size_t)(st % (uint32_t)c->cfg.trace_steps);
    MC3_TRY(hip_ok(c, hipMemcpy(out + (size_t)i * d.chains, c->at<mc3::Record>(c->L.ring) + slot * d.chains,
                                (size_t)d.chains * sizeof(mc3_record), hipMemcpyDeviceToHost), "read ring"));
    for (int ch = 0; ch < d.chains; ++ch)
      if (out[(size_t)i * d.chains + ch].step != st)
        return fail(c, MC3_E_ARG, "step %u is not in the ring", st);
  }
  return MC3_OK;
}

mc3_status mc3_read_candidates(mc3_ctx* c, uint32_t* bits, int32_t* roots) {
  MC3_TRY(usable(c));
  if (!c->have_proposal) return fail(c, MC3_E_STATE, "no proposal to read");
  const Dims& d = c->d;
  MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "read_candidates sync"));
  if (bits) {
    const uint32_t st = c->proposal_step;
    hipLaunchKernelGGL(mc3::k_build_candidates, dim3(d.Bp / 256, d.W), dim3(256), 0, c->stream,
                       c->at<uint32_t>(c->L.candT), c->flips(st), c->base(st), c->roots(st), d.chains, d.M, d.W, d.Bp);
    MC3_TRY(check_launch(c, "candidate kernel"));
    MC3_TRY(hip_ok(c, hipStreamSynchronize(c->stream), "read_candidates sync"));
    std::vector<uint32_t> t((size_t)d.W * d.Bp);
    MC3_TRY(hip_ok(c, hipMemcpy(t.data(), c->at<uint32_t>(c->L.candT), t.size() * 4, hipMemcpyDeviceToHost), "read"));
    for (int col = 0; col < d.B; ++col)
      for (int w = 0; w < d.Wn; ++w) bits[(size_t)col * d.Wn + w] = t[(size_t)w * d.Bp + col];
  }
  if (roots)
    MC3_TRY(hip_ok(c, hipMemcpy(roots, c->roots(c->proposal_step), (size_t)d.chains * 4, hipMemcpyDeviceToHost),
                   "read roots"));
  return MC3_OK;
}

mc3_status mc3_timing_enable(mc3_ctx* c, int32_t on) {
  MC3_TRY(usable(c));
  if (on && c->t_start.empty()) {
    const size_t n = 256;
    c->t_start.assign(n, nullptr);
    c->t_stop.assign(n, nullptr);
    c->t_pending.assign(n, 0);
    for (size_t i = 0; i < n; ++i) {
      MC3_TRY(hip_ok(c, hipEventCreate(&c->t_start[i]), "timing events"));
      MC3_TRY(hip_ok(c, hipEventCreate(&c->t_stop[i]), "timing events"));
    }
  }
  if (on) {
    for (size_t i = 0; i < c->t_pending.size(); ++i) c->t_pending[i] = 0;
    c->t_total_ms = 0.0;
    c->t_count = 0;
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
  MC3_TRY(hip_ok(c, hipMemcpy(buf.data(), c->at<double>(c->L.means), buf.size() * 8, hipMemcpyDeviceToHost),
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

mc3_status mc3_sync(mc3_ctx* c) {
  MC3_TRY(usable(c));
  return hip_ok(c, hipStreamSynchronize(c->stream), "sync");
}

const char* mc3_last_error(const mc3_ctx* c) { return c ? c->err.c_str() : "context is NULL"; }

}  // extern "C"
