/*
 * bm_peak.h -- attainable-peak probes of libbm.so (measurement support, not part of block
 * matching).  The benchmark divides its achieved rates by these as well as by the
 * published MI355X peaks.
 *
 * Both calls run on the current device, allocate their own small device buffers, launch on
 * `stream` (a hipStream_t as void*, NULL = the null stream), wait for their own work and
 * return BM_OK, BM_EINVAL (bad argument) or BM_EDEVICE (HIP error).
 */
#ifndef BM_PEAK_H_
#define BM_PEAK_H_

#include <stdint.h>

#include "bm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Matrix-core rate of a precision form's matrix instruction: shape 0 the instruction the
 * cross-term kernels issue (BM_PREC_FP32: v_mfma_f32_16x16x4f32; BM_PREC_BF16X4 /
 * BM_PREC_FP16X3: v_mfma_f32_16x16x32_{bf16,f16}), shape 1 the 32 x 32 instruction of the
 * same precision (v_mfma_f32_32x32x2f32, v_mfma_f32_32x32x16_{bf16,f16}).  Four 4-wave
 * blocks per compute unit, each wave running `iterations` x 4 independent accumulator
 * chains back to back.  *tflops receives the dense rate in TFLOP/s (2 M N K flops per
 * instruction). */
bm_status bm_peak_mfma(int32_t precision, int32_t shape, int32_t iterations, void* stream,
                       double* tflops);

/* Device-to-device streaming copy of `bytes` (>= 1 MiB) with float4 loads and stores;
 * the best of `repeats` timed runs after one warm-up.  *gbps receives (read + written
 * bytes) / time in GB/s (1e9 bytes per second). */
bm_status bm_peak_copy(int64_t bytes, int32_t repeats, void* stream, double* gbps);

#ifdef __cplusplus
}
#endif

#endif  /* BM_PEAK_H_ */
