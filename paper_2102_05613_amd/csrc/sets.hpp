// sets.hpp -- the set variant's generation probabilities and subset-visit
// probabilities (App. "Markov chain of sets of configurations"; Sec. "Stochastic
// generation of the set"; Sec. "Recursive exponential formula for the generation
// probability").
//
// S = {0..n-1}; a subset is a bitmask X.  A set grows from a nonempty subset by
// additions: a parent chosen uniformly among the current elements generates the new
// element e with probability G[e][parent]; S is reached from X when the n - |X|
// additions bring exactly the elements of S \ X.  Conditioning on the first addition
// gives, with out[X] = P_gen(S | X):
//   out[S] = 1, out[0] = 0,
//   out[X] = (1/|X|) sum_{e not in X} A(X, e) out[X + e],  A(X, e) = sum_{p in X} G[e][p],
// so the subsets are processed by decreasing popcount: every subset of a level in
// parallel, one level per launch (k_set_gen_level), or for small sets all levels of a
// set in one block's LDS (k_set_gen_lds).  (The printed recursion, indexed by the added
// elements S' = S \ X, carries 1/(|S'| |S \ S'|) and, for one element, 1/|S|; the
// sum over insertion orders fixes the factor 1/|S \ S'| = 1/|X| used here.)
#pragma once
#include "common.hpp"

namespace mc3 {

// out[S] = 1 and out[0] = 0 for every set of the batch (grid.x over sets).
__global__ void k_set_gen_ends(double* __restrict__ out, int n, int n_sets) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sets) return;
  double* o = out + ((size_t)s << n);
  o[0] = 0.0;
  o[((size_t)1 << n) - 1] = 1.0;
}

constexpr int kSetMaxN = 20;    // largest set
constexpr int kSetLdsMax = 12;  // largest set held in one block's LDS

// Binomial coefficients C(b, j), 0 <= j <= b <= 20, from Pascal's rule at compile time.
struct BinomTable {
  uint32_t c[kSetMaxN + 1][kSetMaxN + 1];
};
constexpr BinomTable make_binom() {
  BinomTable t{};
  for (int b = 0; b <= kSetMaxN; ++b)
    for (int j = 0; j <= b; ++j) t.c[b][j] = (j == 0 || j == b) ? 1u : t.c[b - 1][j - 1] + t.c[b - 1][j];
  return t;
}
__constant__ BinomTable kBinom = make_binom();

__device__ __forceinline__ uint32_t binom(int b, int j) {
  return (j < 0 || j > b) ? 0u : kBinom.c[b][j];
}

// The subset of {0..n-1} of size k with rank i in the combinatorial number system
// (bits taken from the top: bit b is in when C(b, remaining) <= the remaining rank).
__device__ __forceinline__ uint32_t unrank_subset(uint32_t i, int n, int k) {
  uint32_t X = 0u;
  for (int b = n - 1; b >= 0 && k > 0; --b) {
    const uint32_t c = binom(b, k);
    if (c <= i) {
      X |= 1u << b;
      i -= c;
      --k;
    }
  }
  return X;
}

// out[X] for one subset X of size k from the values of the subsets one larger:
// a[e] = sum_{p in X} G[e][p] accumulated over X's elements in increasing order, then
// (1/k) sum_{e not in X, increasing} a[e] out[X + e].  NMAX bounds n (registers).
template <int NMAX, class GetG, class GetP>
__device__ __forceinline__ double set_gen_value(uint32_t X, int n, int k, GetG g, GetP pv) {
  double a[NMAX];
#pragma unroll
  for (int e = 0; e < NMAX; ++e) a[e] = 0.0;
  for (uint32_t m = X; m; m &= m - 1u) {
    const int p = __ffs(m) - 1;
#pragma unroll
    for (int e = 0; e < NMAX; ++e)
      if (e < n) a[e] += g(e, p);
  }
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < NMAX; ++e)
    if (e < n && !((X >> e) & 1u)) acc += a[e] * pv(X | (1u << e));
  return acc / (double)k;
}

// One level: the C(n, k) subsets of size k (grid.x over their ranks, grid.y over
// sets); the level k+1 above is complete.
__global__ __launch_bounds__(256) void k_set_gen_level(const double* __restrict__ G, double* __restrict__ out,
                                                       int n, int k) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t s = blockIdx.y;
  if (i >= binom(n, k)) return;
  const uint32_t X = unrank_subset(i, n, k);
  const double* __restrict__ Gs = G + s * (size_t)n * n;
  double* __restrict__ o = out + (s << n);
  o[X] = set_gen_value<kSetMaxN>(X, n, k, [&](int e, int p) { return Gs[(size_t)e * n + p]; },
                                 [&](uint32_t Y) { return o[Y]; });
}

// Sets of at most kSetLdsMax elements: one block of 256 threads per set (grid.x) keeps
// the set's 2^n values and its n x n law in LDS, orders the subsets by size once, and
// runs every level with a barrier between levels; then writes the 2^n values.
__global__ __launch_bounds__(256) void k_set_gen_lds(const double* __restrict__ G, double* __restrict__ out, int n) {
  __shared__ double P[1 << kSetLdsMax];
  __shared__ double Gl[kSetLdsMax * kSetLdsMax];
  __shared__ uint16_t order[1 << kSetLdsMax];
  __shared__ int cnt[kSetLdsMax + 1], off[kSetLdsMax + 2];
  const size_t s = blockIdx.x;
  const uint32_t nmask = 1u << n;
  for (int i = threadIdx.x; i < n * n; i += 256) Gl[i] = G[s * (size_t)n * n + i];
  for (uint32_t X = threadIdx.x; X < nmask; X += 256) P[X] = X == nmask - 1u ? 1.0 : 0.0;
  if (threadIdx.x <= (unsigned)n) cnt[threadIdx.x] = 0;
  __syncthreads();
  for (uint32_t X = threadIdx.x; X < nmask; X += 256) atomicAdd(&cnt[__popc(X)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    off[0] = 0;
    for (int k = 0; k <= n; ++k) off[k + 1] = off[k] + cnt[k];
    for (int k = 0; k <= n; ++k) cnt[k] = 0;
  }
  __syncthreads();
  for (uint32_t X = threadIdx.x; X < nmask; X += 256) {
    const int k = __popc(X);
    order[off[k] + atomicAdd(&cnt[k], 1)] = (uint16_t)X;
  }
  __syncthreads();
  for (int k = n - 1; k >= 1; --k) {
    const int lo = off[k], num = off[k + 1] - off[k];
    for (int i = threadIdx.x; i < num; i += 256) {
      const uint32_t X = order[lo + i];
      P[X] = set_gen_value<kSetLdsMax>(X, n, k, [&](int e, int p) { return Gl[e * n + p]; },
                                       [&](uint32_t Y) { return P[Y]; });
    }
    __syncthreads();
  }
  double* __restrict__ o = out + (s << n);
  for (uint32_t X = threadIdx.x; X < nmask; X += 256) o[X] = P[X];
}

// With the caller's equilibrium weights peq[X] of the proper subsets: the set's
// P_eq(S) = sum_{X != S} peq[X] out[X] (Eq. eq_P_eq_n), one block of 256 threads per
// set, thread t summing X = t, t + 256, ... and a fixed-order tree over the threads.
__global__ __launch_bounds__(256) void k_set_peq(const double* __restrict__ peq, const double* __restrict__ out,
                                                 double* __restrict__ peq_set, int n) {
  __shared__ double red[256];
  const size_t s = blockIdx.x;
  const uint32_t full = (1u << n) - 1u;
  const double* __restrict__ p = peq + (s << n);
  const double* __restrict__ o = out + (s << n);
  double acc = 0.0;
  for (uint32_t X = threadIdx.x; X < full; X += 256) acc += p[X] * o[X];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) peq_set[s] = red[0];
}

// psub[X] = peq[X] out[X] / P_eq(S) for X != S (Eq. eq_p_S_S), psub[S] = 0: the
// probability of visiting subset X while the chain sits at S (grid.x over bitmasks,
// grid.y over sets).
__global__ void k_set_psub(const double* __restrict__ peq, const double* __restrict__ out,
                           const double* __restrict__ peq_set, double* __restrict__ psub, int n) {
  const uint32_t X = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t s = blockIdx.y;
  if (X >= (1u << n)) return;
  const size_t i = (s << n) + X;
  psub[i] = X == (1u << n) - 1u ? 0.0 : peq[i] * out[i] / peq_set[s];
}

}  // namespace mc3
