/* mc3_ceiling.h -- the attainable rate of the BF16 matrix cores on this device.
 *
 * A measurement aid for the scoring kernel's roofline: the published dense BF16 peak
 * assumes the peak engine clock, which a device sustaining matrix-core work at full
 * power may not hold.  This library runs a plain loop of independent 32x32x16 BF16
 * matrix-core operations on every compute unit at the scoring kernel's occupancy
 * (one 512-thread block per compute unit, two waves per SIMD; operands of the same
 * kind, changing from one operation to the next: random data in the split coupling
 * terms' range for A, random +-1 for B) and reports its rate and the engine clock it
 * ran at.
 * It is not part of the Monte Carlo path.  Compiled for gfx950 into libmc3ceil.so.
 */
#ifndef MC3_CEILING_H
#define MC3_CEILING_H

#ifdef __cplusplus
extern "C" {
#endif

/* Run the loop once untimed, then `repeats` timed launches of `iters` rounds (each
 * round: 64 matrix-core operations per wave, 32768 flops each) over `blocks` blocks of
 * 512 threads on the current device's null stream.
 *   tflops  (out, host): the best rate of the timed launches, in TFLOP/s, timed with
 *           HIP events around each launch;
 *   ghz     (out, host): the median over blocks of (shader-clock cycles) / (constant
 *           wall-clock time) of the last launch, in GHz.
 * Allocates and frees its own device buffers.  Returns 0 on success, -1 for
 * iters < 1, blocks < 1 or repeats < 1, or a HIP error code. */
int mc3c_mfma_ceiling(int iters, int blocks, int repeats, double* tflops, double* ghz);

/* The same kind of loop (256 blocks of 512 threads, operands of the same kind) with
 * the scoring kernel's other traffic mixed in, per round of 64 matrix-core operations:
 *   mix 0: none;
 *   mix 1: the split scoring kernel's own mix, scaled from its 48 MFMAs a wave per
 *          32-k chunk: 32 LDS reads of 128 bits, 72 VALU operations, 5 global 32-bit
 *          loads, 1 workgroup barrier;
 *   mix 2: the mix of a 64-row x 128-column wave tile (half the LDS reads, twice the
 *          B expansion and word loads): 16, 120, 11, 1;
 *   mix 3: 32 LDS reads only;  mix 4: 16 LDS reads only.
 * One untimed launch, then `repeats` timed launches of `iters` rounds; tflops (out,
 * host): the best rate, timed with HIP events.  Allocates and frees its own device
 * buffers.  Returns 0, -1 for a mix outside 0..4, iters < 1 or repeats < 1, or a HIP
 * error code. */
int mc3c_mfma_mix(int mix, int iters, int repeats, double* tflops);

#ifdef __cplusplus
}
#endif

#endif /* MC3_CEILING_H */
