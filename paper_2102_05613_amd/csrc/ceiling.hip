// ceiling.hip -- the attainable BF16 matrix-core rate and the clock it runs at.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "mc3_ceiling.h"

namespace {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// A 32-bit hash (an integer finaliser: xor-shifts and odd multipliers).
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

// Two bfloat16 values with random signs and mantissas and exponents 2^-6 .. 2^-3 (the
// range of a split coupling term of a Gaussian J at N = 1024) from 32 random bits.
__device__ __forceinline__ uint32_t rand_bf16x2(uint32_t r) {
  const uint32_t lo = (r & 0x807Fu) | ((0x79u + ((r >> 7) & 3u)) << 7);
  const uint32_t hi = ((r >> 16) & 0x807Fu) | ((0x79u + ((r >> 23) & 3u)) << 7);
  return lo | (hi << 16);
}

// Each wave: 8 independent chains of 32x32x16 BF16 matrix-core operations over `iters`
// rounds of 64 operations; each round cycles through 8 A operands of random data in
// the coupling terms' range and 4 B operands of random +-1 (as the scoring kernel's
// operands change from one operation to the next); lane 0 of each block stamps the
// shader clock and the constant wall clock before and after the loop.  The sums land
// in `out` so that no operation is dead.
__global__ __launch_bounds__(512, 2) void k_mfma_loop(float* __restrict__ out, unsigned long long* __restrict__ stamps,
                                                      int iters) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  union Op {
    uint32_t u[4];
    bf16x8 v;
  };
  Op a[8], b[4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int p = 0; p < 4; ++p) a[i].u[p] = rand_bf16x2(mix32(t * 64u + 4u * i + p));
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int p = 0; p < 4; ++p) b[j].u[p] = (mix32(0x9E3779B9u ^ (t * 16u + 4u * j + p)) & 0x80008000u) | 0x3F803F80u;
  f32x16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
  const unsigned long long c0 = (unsigned long long)clock64(), w0 = (unsigned long long)wall_clock64();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int rot = 0; rot < 8; ++rot)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[(i + 2 * rot) % 8].v, b[(j + rot) % 4].v, acc[i][j],
                                                             0, 0, 0);
  }
  const unsigned long long c1 = (unsigned long long)clock64(), w1 = (unsigned long long)wall_clock64();
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) s += acc[i][j][e];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (threadIdx.x == 0) {
    stamps[4 * (size_t)blockIdx.x + 0] = c0;
    stamps[4 * (size_t)blockIdx.x + 1] = w0;
    stamps[4 * (size_t)blockIdx.x + 2] = c1;
    stamps[4 * (size_t)blockIdx.x + 3] = w1;
  }
}

constexpr int kThreads = 512;

}  // namespace

extern "C" int mc3c_mfma_ceiling(int iters, int blocks, int repeats, double* tflops, double* ghz) {
  if (iters < 1 || blocks < 1 || repeats < 1 || !tflops || !ghz) return -1;
  int dev = 0, wall_khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return (int)e;
  float* out = nullptr;
  unsigned long long* stamps = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  e = hipMalloc(&out, (size_t)blocks * kThreads * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&stamps, (size_t)blocks * 4 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  double best = 0.0;
  std::vector<unsigned long long> h((size_t)blocks * 4);
  for (int rep = -1; e == hipSuccess && rep < repeats; ++rep) {
    e = hipEventRecord(t0, nullptr);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_mfma_loop, dim3(blocks), dim3(kThreads), 0, nullptr, out, stamps, iters);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(t1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e == hipSuccess && rep >= 0 && ms > 0.0f) {
      const double flops = (double)blocks * (kThreads / 64) * (double)iters * 64.0 * 32768.0;
      best = std::max(best, flops / (ms * 1e-3) / 1e12);
    }
  }
  if (e == hipSuccess) e = hipMemcpy(h.data(), stamps, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
  if (e == hipSuccess) {
    std::vector<double> f;
    for (int b = 0; b < blocks; ++b) {
      const double cyc = (double)(h[4 * b + 2] - h[4 * b + 0]);
      const double sec = (double)(h[4 * b + 3] - h[4 * b + 1]) / ((double)wall_khz * 1e3);
      if (sec > 0.0) f.push_back(cyc / sec / 1e9);
    }
    std::sort(f.begin(), f.end());
    *ghz = f.empty() ? 0.0 : f[f.size() / 2];
    *tflops = best;
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (out) (void)hipFree(out);
  if (stamps) (void)hipFree(stamps);
  return e == hipSuccess ? 0 : (int)e;
}
