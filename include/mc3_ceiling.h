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

#ifdef __cplusplus
}
#endif

#endif /* MC3_CEILING_H */
