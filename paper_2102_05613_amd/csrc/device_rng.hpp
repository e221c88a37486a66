// device_rng.hpp -- counter-based random numbers and exp for the MCMCMC kernels.
//
// Philox4x32-10 as defined by Salmon, Moraes, Dror and Shaw ("Parallel random
// numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with
// the round permutation, and a Weyl-sequence key schedule.
//
// Stream layout: word n of stream (tag, chain, step, edge) is element n%4 of the
// block at counter (n/4, edge, step, tag<<28 | chain) under key (seed lo, seed hi).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mc3 {

enum : uint32_t { kTagInit = 1u, kTagRoot = 2u, kTagEdge = 3u, kTagSelect = 4u };

struct Key { uint32_t lo, hi; };

__device__ __forceinline__ uint4 philox10(uint4 c, Key k) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    // one 32x32 -> 64-bit product per multiplier (high and low halves together)
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k.lo, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k.hi, (uint32_t)p0);
    k.lo += 0x9E3779B9u;
    k.hi += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ uint4 stream_block(Key k, uint32_t tag, uint32_t chain, uint32_t step,
                                              uint32_t edge, uint32_t block) {
  return philox10(make_uint4(block, edge, step, (tag << 28) | (chain & 0x0FFFFFFFu)), k);
}

__device__ __forceinline__ uint32_t pick(uint4 b, uint32_t i) {
  return i == 0 ? b.x : (i == 1 ? b.y : (i == 2 ? b.z : b.w));
}

// Integer in [0, n): floor(w n / 2^32).
__device__ __forceinline__ uint32_t randint(uint32_t w, uint32_t n) {
  return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

// 53-bit uniform integer: top 27 bits of w0 then top 26 bits of w1.
__device__ __forceinline__ uint64_t u53_of(uint32_t w0, uint32_t w1) {
  return ((uint64_t)(w0 >> 5) << 26) | (uint64_t)(w1 >> 6);
}

// exp(x) for the selection weights (x <= 0 in use).  Cody-Waite reduction
// x = k ln2 + r with ln 2 split into a head of 32 significant bits (k * head exact)
// and a tail; exp(r) by its Taylor series to degree 13 (Horner); times 2^k built from
// the exponent field.  x < -708 gives 0.  Every operation is a separately rounded
// IEEE double operation (this file is compiled without FMA contraction), so the
// value is a fixed function of x.
__device__ __forceinline__ double exp_weight(double x) {
  if (x != x) return x;
  if (x < -708.0) return 0.0;
  if (x > 709.0) return __longlong_as_double(0x7FF0000000000000ll);
  const double log2e = 0x1.71547652b82fep+0;
  const double ln2_head = 0x1.62e42ff000000p-1;
  const double ln2_tail = -0x1.718432a1b0e26p-35;
  double kd = floor(__dmul_rn(x, log2e) + 0.5);
  int k = (int)kd;
  double r = __dsub_rn(__dsub_rn(x, __dmul_rn(kd, ln2_head)), __dmul_rn(kd, ln2_tail));
  // 1/n!, n = 13 down to 2, each the double nearest the exact rational
  double p = 0x1.6124613a86d09p-33;
  p = __dadd_rn(__dmul_rn(p, r), 0x1.1eed8eff8d898p-29);
  p = __dadd_rn(__dmul_rn(p, r), 0x1.ae64567f544e4p-26);
  p = __dadd_rn(__dmul_rn(p, r), 0x1.27e4fb7789f5cp-22);
  p = __dadd_rn(__dmul_rn(p, r), 0x1.71de3a556c734p-19);
  p = __dadd_rn(__dmul_rn(p, r), 0x1.a01a01a01a01ap-16);
  p = __dadd_rn(__dmul_rn(p, r), 0x1.a01a01a01a01ap-13);
  p = __dadd_rn(__dmul_rn(p, r), 0x1.6c16c16c16c17p-10);
  p = __dadd_rn(__dmul_rn(p, r), 0x1.1111111111111p-7);
  p = __dadd_rn(__dmul_rn(p, r), 0x1.5555555555555p-5);
  p = __dadd_rn(__dmul_rn(p, r), 0x1.5555555555555p-3);
  p = __dadd_rn(__dmul_rn(p, r), 0x1.0p-1);
  p = __dadd_rn(__dmul_rn(p, r), 1.0);
  p = __dadd_rn(__dmul_rn(p, r), 1.0);
  double two_k = __longlong_as_double((long long)(k + 1023) << 52);
  return __dmul_rn(p, two_k);
}

}  // namespace mc3
