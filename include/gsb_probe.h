/* gsb_probe.h -- measurement of this device's ceilings (libgsb_probe.so).
 *
 * Not part of the GSB hot path and not linked into libgsb.so: micro-benchmarks that
 * measure what the chip itself delivers, against which the step kernels' roofline
 * fractions (stated against the published peaks) can be read.
 */
#ifndef GSB_PROBE_H
#define GSB_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Fills out[0 .. min(count, 16) - 1] with, in order:
 *   dense MFMA rate in FLOP/s (OP/s for int8) of the forms the step kernels use, from
 *   every CU running 4 waves per SIMD of 8 independent MFMA chains --
 *     [0] FP8 x FP8 16x16x128, [1] FP4 x FP8 16x16x128, [2] int8 16x16x64,
 *     [3] bf16 16x16x32, [4] binary32 16x16x4;
 *   read bandwidth in bytes/s -- [5] L2, over 2 MiB with device-scope (L1-skipping)
 *     16-byte loads, four in flight per thread, 8 workgroups of 256 threads per CU;
 *     streaming over [6] 64 MiB (MALL) and [7] 2 GiB (HBM);
 *   [8] streaming write bandwidth over 2 GiB;
 *   [9] the shader clock in Hz during a busy kernel (s_memtime against the constant-rate
 *     wall clock);
 *   the 32 x 32 MFMA shapes -- [10] FP8 x FP8 32x32x64, [11] int8 32x32x32,
 *     [12] bf16 32x32x16;
 *   matrix-core / vector-ALU sharing of a SIMD, in milliseconds, with one workgroup of
 *     8 waves per CU (each SIMD one wave of each kind): 20000 rounds of four FP4 x FP8
 *     16x16x128 MFMAs on waves 0-3 and of 20 binary32 multiplies and adds on waves 4-7 --
 *     [13] the MFMA waves alone, [14] the VALU waves alone, [15] both.
 * Allocates and frees 2 GiB of device memory on the current device; runs on the null
 * stream and synchronises the device.  out: host.
 * Returns 0, or the hipError_t of the first failing call (1 for a NULL out). */
int32_t gsb_probe_ceilings(double* out, int32_t count);

#ifdef __cplusplus
}
#endif

#endif /* GSB_PROBE_H */
