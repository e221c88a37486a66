// couplings.hpp -- the seeded SK instance generator on the device.
#pragma once
#include "common.hpp"

namespace mc3 {

constexpr uint32_t kTagCoupling = 5u;   // the coupling stream

// J64 (Np x Np, row-major) of an instance from a seed.  Pair a < b reads block b of
// the coupling stream (tag 5, chain 0, step 0, edge a), words w0..w3.  kind 0 (the +-1
// instances, energy scale 1/sqrt(N)): +1 if bit 0 of w0 is set, else -1.  kind 1
// (Gaussian couplings of variance 1/N, energy scale 1): Box-Muller,
// u1 = (u53(w0, w1) + 1) / 2^53 in (0, 1], u2 = u53(w2, w3) / 2^53 in [0, 1),
// (sqrt(-2 ln u1) cos(2 pi u2)) * inv_sqrt_n.  Symmetric, zero diagonal, zero rows and
// columns N .. Np-1.  One thread per element.
__global__ void k_gen_couplings(double* __restrict__ J64, int N, int Np, int kind, Key key, double inv_sqrt_n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)Np * Np) return;
  const int i = (int)(idx / Np), j = (int)(idx % Np);
  double v = 0.0;
  if (i < N && j < N && i != j) {
    const int a = min(i, j), b = max(i, j);
    const uint4 w = stream_block(key, kTagCoupling, 0u, 0u, (uint32_t)a, (uint32_t)b);
    if (kind == 0) {
      v = (w.x & 1u) ? 1.0 : -1.0;
    } else {
      const double u1 = ((double)u53_of(w.x, w.y) + 1.0) * 0x1.0p-53;
      const double u2 = (double)u53_of(w.z, w.w) * 0x1.0p-53;
      const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
      v = z * inv_sqrt_n;
    }
  }
  J64[idx] = v;
}

// The couplings as every scorer reads them: the strict upper triangle of a loaded J64
// (rows i < j) mirrored below the diagonal and the diagonal cleared, so that the pair
// sums (which read i < j only) and the field update (which reads whole rows and
// columns) see the same symmetric, zero-diagonal matrix whatever the caller left
// below the diagonal.  One thread per element at or below the diagonal; the upper
// triangle is only read.
__global__ void k_mirror_upper(double* __restrict__ J64, int Np) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)Np * Np) return;
  const int i = (int)(idx / Np), j = (int)(idx % Np);
  if (j > i) return;
  J64[idx] = j == i ? 0.0 : J64[(size_t)j * Np + i];
}

}  // namespace mc3
