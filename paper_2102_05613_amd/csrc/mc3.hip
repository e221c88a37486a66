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
  size_t J64, Jpack, spins, e_cur, flips, roots, candT, partial, Ecol, ring, moves, near, minm, drift, erecomp,
      total;
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
  L.flips = take((size_t)d.chains * d.M * d.W * 4);
  L.roots = take((size_t)d.chains * 4);
  L.candT = take((size_t)d.W * d.Bp * 4);
  L.partial = take((size_t)d.P * d.Bp * 8);
  L.Ecol = take((size_t)d.Bp * 8);
  L.ring = take((size_t)(c.trace_steps > 0 ? c.trace_steps : 0) * d.chains * sizeof(mc3::Record));
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
  if (c->M < 1 || c->M > 4096) return "M must be in [1, 4096]";
  if (c->chains < 1) return "chains must be >= 1";
  if ((long long)c->chains * c->M > (1ll << 24)) return "chains * M must be <= 2^24";
  if ((long long)c->chains + c->chain_base > (1ll << 28)) return "chain_base + chains must be <= 2^28";
  if (c->kmin < 1 || c->kmax < c->kmin || c->kmax > c->N) return "need 1 <= kmin <= kmax <= N";
  if (c->precision != MC3_FP64 && c->precision != MC3_SPLIT_BF16) return "unknown precision";
  if (c->rule != MC3_RULE_MCMCMC && c->rule != MC3_RULE_METROPOLIS) return "unknown rule";
  if (c->rule == MC3_RULE_METROPOLIS && c->M != 1) return "rule METROPOLIS requires M == 1";
  if (c->trace_steps < 0) return "trace_steps must be >= 0";
  if (c->reserved != 0) return "reserved must be 0";
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
  int device = 0;
  bool have_J = false, have_chains = false, have_proposal = false, have_scores = false, poisoned = false;
  uint32_t proposal_step = 0;
  double scale = 1.0;
  double tol = 0.0;
  int64_t steps_done = 0;
  int split_cf = 2;  // split scoring tile: 32*split_cf columns per wave (2 or 4)
  std::string err;

  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
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

mc3_status do_propose(mc3_ctx* c, uint32_t step) {
  const Dims& d = c->d;
  const size_t wbytes = (size_t)d.W * 4;
  int T = (int)(65536 / wbytes);
  if (T > 256) T = 256;
  T = (T / 64) * 64;
  if (T < 64) T = 64;
  const size_t lds = (size_t)T * wbytes;
  const long long total = (long long)d.chains * d.M;
  const int blocks = (int)((total + T - 1) / T);
  hipLaunchKernelGGL(mc3::k_propose, dim3(blocks), dim3(T), lds, c->stream, c->at<uint32_t>(c->L.flips),
                     c->at<int32_t>(c->L.roots), d.chains, d.M, d.N, d.W, c->cfg.kmin, c->cfg.kmax,
                     c->cfg.rule == MC3_RULE_METROPOLIS ? 1 : 0, c->key(), c->cfg.chain_base, step);
  MC3_TRY(check_launch(c, "propose kernel"));
  hipLaunchKernelGGL(mc3::k_build_candidates, dim3(d.Bp / 256, d.W), dim3(256), 0, c->stream,
                     c->at<uint32_t>(c->L.candT), c->at<uint32_t>(c->L.spins), c->at<uint32_t>(c->L.flips),
                     c->at<int32_t>(c->L.roots), d.chains, d.M, d.W, d.Bp);
  MC3_TRY(check_launch(c, "candidate kernel"));
  c->have_proposal = true;
  c->have_scores = false;
  c->proposal_step = step;
  return MC3_OK;
}

mc3_status do_score(mc3_ctx* c, double* E_out) {
  const Dims& d = c->d;
  if (c->cfg.precision == MC3_SPLIT_BF16) {
    const int TN = 128 * c->split_cf;
    const int CT = d.Bp / TN;
    const int U = d.P * CT;
    const int grid = 8 * ((U + 7) / 8);
    if (c->split_cf == 4)
      hipLaunchKernelGGL(mc3::k_score_split<4>, dim3(grid), dim3(256), 0, c->stream,
                         c->at<const uint4>(c->L.Jpack), c->at<const uint32_t>(c->L.candT),
                         c->at<double>(c->L.partial), d.Np, d.Bp, d.NB, d.P, CT);
    else
      hipLaunchKernelGGL(mc3::k_score_split<2>, dim3(grid), dim3(256), 0, c->stream,
                         c->at<const uint4>(c->L.Jpack), c->at<const uint32_t>(c->L.candT),
                         c->at<double>(c->L.partial), d.Np, d.Bp, d.NB, d.P, CT);
  } else {
    const int CT = d.Bp / 128;
    const int U = d.P * CT;
    const int grid = 8 * ((U + 7) / 8);
    hipLaunchKernelGGL(mc3::k_score_f64, dim3(grid), dim3(256), 0, c->stream, c->at<const double>(c->L.Jpack),
                       c->at<const uint32_t>(c->L.candT), c->at<double>(c->L.partial), d.Np, d.Bp, d.NB, d.P, CT);
  }
  MC3_TRY(check_launch(c, "score kernel"));
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

mc3_status do_select(mc3_ctx* c, uint32_t step, double beta) {
  const Dims& d = c->d;
  hipLaunchKernelGGL(mc3::k_select, dim3((d.chains + 3) / 4), dim3(256), 0, c->stream, c->at<uint32_t>(c->L.spins),
                     c->at<double>(c->L.e_cur), c->at<const uint32_t>(c->L.candT),
                     c->at<const double>(c->L.partial), d.P, c->scale, c->at<double>(c->L.Ecol),
                     c->at<const int32_t>(c->L.roots), c->at<mc3::Record>(c->L.ring),
                     c->at<unsigned long long>(c->L.moves), c->at<unsigned long long>(c->L.near),
                     c->at<double>(c->L.minm), d.chains, d.M, d.W, d.Bp, c->cfg.rule == MC3_RULE_METROPOLIS ? 1 : 0,
                     beta, c->tol, c->key(), c->cfg.chain_base, step, c->cfg.trace_steps);
  MC3_TRY(check_launch(c, "select kernel"));
  c->have_proposal = false;
  c->have_scores = false;
  c->steps_done += 1;
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
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t t = step0 + (uint32_t)i;
    double beta = beta0;
    if (total > 1) beta = beta0 + (beta1 - beta0) * ((double)t / (double)(total - 1));
    MC3_TRY(do_propose(c, t));
    MC3_TRY(do_score(c, nullptr));
    MC3_TRY(do_select(c, t, beta));
  }
  return MC3_OK;
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
    std::vector<uint32_t> t((size_t)d.W * d.Bp);
    MC3_TRY(hip_ok(c, hipMemcpy(t.data(), c->at<uint32_t>(c->L.candT), t.size() * 4, hipMemcpyDeviceToHost), "read"));
    for (int col = 0; col < d.B; ++col)
      for (int w = 0; w < d.Wn; ++w) bits[(size_t)col * d.Wn + w] = t[(size_t)w * d.Bp + col];
  }
  if (roots)
    MC3_TRY(hip_ok(c, hipMemcpy(roots, c->at<int32_t>(c->L.roots), (size_t)d.chains * 4, hipMemcpyDeviceToHost),
                   "read roots"));
  return MC3_OK;
}

mc3_status mc3_sync(mc3_ctx* c) {
  MC3_TRY(usable(c));
  return hip_ok(c, hipStreamSynchronize(c->stream), "sync");
}

const char* mc3_last_error(const mc3_ctx* c) { return c ? c->err.c_str() : "context is NULL"; }

}  // extern "C"
