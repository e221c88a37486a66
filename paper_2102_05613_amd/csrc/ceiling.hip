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

// The same kind of loop with other traffic mixed in, per round of 64 MFMAs: R 128-bit
// LDS reads (lane-contiguous fragments of a 24 KiB buffer, as the scoring kernel reads
// its A fragments; each consumed eight MFMAs after it was issued), V VALU operations of
// the B expansion's kind (shift, and, or), L 32-bit global loads from an L2-resident
// window, and NB workgroup barriers.  Operands: 4 A sets of random data in the split
// terms' range, 2 B sets of random +-1.
template <int R, int V, int L, int NB>
__global__ __launch_bounds__(512, 2) void k_mfma_mix(float* __restrict__ out, const uint32_t* __restrict__ src,
                                                     int iters) {
  static_assert(R % 8 == 0 && V % 24 == 0 && NB <= 2, "per-round counts");
  __shared__ uint4 lds[24 * 64];
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < 24 * 64; i += blockDim.x)
    lds[i] = make_uint4(mix32(i), mix32(i + 1u), mix32(i + 2u), mix32(i + 3u));
  __syncthreads();
  union Op {
    uint32_t u[4];
    bf16x8 v;
    uint4 q;
  };
  Op a[4], b[2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int p = 0; p < 4; ++p) a[i].u[p] = rand_bf16x2(mix32(t * 64u + 4u * i + p));
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int p = 0; p < 4; ++p) b[j].u[p] = (mix32(0x9E3779B9u ^ (t * 16u + 4u * j + p)) & 0x80008000u) | 0x3F803F80u;
  f32x16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
  uint32_t sink = 0u, vsink = 0u, lsink = 0u;
  int off = (int)(threadIdx.x >> 6) * 3;
  // window of 64 rows x 64 words per block slot, inside the 8 x 4096 + 64 x 64 word buffer
  const uint32_t* __restrict__ g = src + (blockIdx.x & 7u) * 4096u + lane;
  for (int it = 0; it < iters; ++it) {
    // the loads in two halves, each consumed four rounds of 8 MFMAs after its issue
    constexpr int L0 = (L + 1) / 2;
    uint32_t gl[L0 > 0 ? L0 : 1];
#pragma unroll
    for (int rot = 0; rot < 8; ++rot) {
      if (rot == 0 || rot == 4) {
#pragma unroll
        for (int q = 0; q < (rot == 0 ? L0 : L - L0); ++q) gl[q] = g[((it + q + rot) & 63) * 64];
      }
      Op rd[R / 8 > 0 ? R / 8 : 1];
#pragma unroll
      for (int q = 0; q < R / 8; ++q) rd[q].q = lds[((off + rot * (R / 8) + q) % 24) * 64 + lane];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[(i + rot) % 4].v, b[(j + rot) % 2].v, acc[i][j], 0, 0,
                                                             0);
#pragma unroll
      for (int q = 0; q < R / 8; ++q) sink ^= rd[q].u[0] ^ rd[q].u[1] ^ rd[q].u[2] ^ rd[q].u[3];
#pragma unroll
      for (int v = 0; v < V / 8; v += 3) vsink ^= (((sink + (uint32_t)(rot * 7 + v)) << (v & 15)) & 0x80008000u) |
                                                  0x3F803F80u;
      if (rot == 3 || rot == 7) {
#pragma unroll
        for (int q = 0; q < (rot == 3 ? L0 : L - L0); ++q) lsink ^= gl[q];
      }
      if (NB > 0 && (rot == 3 || (NB > 1 && rot == 7))) __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);   // each round of 8 MFMAs keeps its own traffic
    }
    off += 7;
  }
  float s = (float)((sink ^ vsink ^ lsink) & 1u);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) s += acc[i][j][e];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

constexpr int kThreads = 512;
constexpr size_t kMixWords = 8 * 4096 + 64 * 64;

template <int R, int V, int L, int NB>
hipError_t time_mix(float* out, const uint32_t* src, int iters, int repeats, hipEvent_t t0, hipEvent_t t1,
                    double* best) {
  *best = 0.0;
  for (int rep = -1; rep < repeats; ++rep) {
    hipError_t e = hipEventRecord(t0, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mfma_mix<R, V, L, NB>), dim3(256), dim3(kThreads), 0, nullptr, out, src, iters);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(t1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e != hipSuccess) return e;
    if (rep >= 0 && ms > 0.0f)
      *best = std::max(*best, 256.0 * (kThreads / 64) * (double)iters * 64.0 * 32768.0 / (ms * 1e-3) / 1e12);
  }
  return hipSuccess;
}

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

extern "C" int mc3c_mfma_mix(int mix, int iters, int repeats, double* tflops) {
  if (mix < 0 || mix > 4 || iters < 1 || repeats < 1 || !tflops) return -1;
  float* out = nullptr;
  uint32_t* src = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = hipMalloc(&out, (size_t)256 * kThreads * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&src, kMixWords * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(src, 0, kMixWords * sizeof(uint32_t));
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  double best = 0.0;
  if (e == hipSuccess) {
    switch (mix) {
      case 0: e = time_mix<0, 0, 0, 0>(out, src, iters, repeats, t0, t1, &best); break;
      case 1: e = time_mix<32, 72, 5, 1>(out, src, iters, repeats, t0, t1, &best); break;
      case 2: e = time_mix<16, 120, 11, 1>(out, src, iters, repeats, t0, t1, &best); break;
      case 3: e = time_mix<32, 0, 0, 0>(out, src, iters, repeats, t0, t1, &best); break;
      default: e = time_mix<16, 0, 0, 0>(out, src, iters, repeats, t0, t1, &best); break;
    }
  }
  if (e == hipSuccess) *tflops = best;
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (out) (void)hipFree(out);
  if (src) (void)hipFree(src);
  return e == hipSuccess ? 0 : (int)e;
}
