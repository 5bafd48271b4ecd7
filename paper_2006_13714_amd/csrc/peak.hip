// Attainable-peak probes for the roofline denominators on gfx950: a matrix-op loop per
// precision form (the same matrix instructions the cross-term kernels issue, four
// independent accumulator chains per wave, every SIMD of every compute unit busy) and a
// streaming device copy (float4 loads and stores, grid-stride).  Both are timed with HIP
// events on the caller's stream and return rates of the work they did.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

#include "../../include/bm.h"
#include "../../include/bm_peak.h"
#include "plan.h"

namespace bmk {

typedef float f4p __attribute__((ext_vector_type(4)));
typedef unsigned int u4p __attribute__((ext_vector_type(4)));
typedef __bf16 bf8p __attribute__((ext_vector_type(8)));
typedef _Float16 h8p __attribute__((ext_vector_type(8)));

constexpr int kPeakChains = 4;

typedef float f16p __attribute__((ext_vector_type(16)));

// SHAPE 0: the 16 x 16 instructions the cross-term kernels issue; SHAPE 1: the 32 x 32
// instructions of the same precision (for comparison of the two shapes' rates).
template <int PREC, int SHAPE>
__global__ void __launch_bounds__(256) mfma_loop_kernel(float* out, int iters, float seed) {
  using Acc = std::conditional_t<SHAPE == 0, f4p, f16p>;
  Acc acc[kPeakChains];
#pragma unroll
  for (int q = 0; q < kPeakChains; ++q) acc[q] = Acc{};
  const float a = seed * (float)(threadIdx.x + 1), b = seed * 0.5f;
  u4p ua, ub;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ua[i] = __float_as_uint(a) ^ (i * 0x01010101u);
    ub[i] = __float_as_uint(b) ^ (i * 0x00FF00FFu);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < kPeakChains; ++q) {
      if constexpr (SHAPE == 0) {
        if constexpr (PREC == BM_PREC_FP32)
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
        else if constexpr (PREC == BM_PREC_FP16X3)
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8p, ua),
                                                          __builtin_bit_cast(h8p, ub), acc[q], 0, 0, 0);
        else
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8p, ua),
                                                           __builtin_bit_cast(bf8p, ub), acc[q], 0, 0, 0);
      } else {
        if constexpr (PREC == BM_PREC_FP32)
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[q], 0, 0, 0);
        else if constexpr (PREC == BM_PREC_FP16X3)
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8p, ua),
                                                          __builtin_bit_cast(h8p, ub), acc[q], 0, 0, 0);
        else
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8p, ua),
                                                           __builtin_bit_cast(bf8p, ub), acc[q], 0, 0, 0);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < kPeakChains; ++q)
#pragma unroll
    for (int i = 0; i < (SHAPE == 0 ? 4 : 16); ++i) s += acc[q][i];
  if (s == 1234.5f) out[threadIdx.x] = s;  // keeps the chains live; never true in practice
}

// Grid-stride copy, four float4 loads in flight per thread before their stores.
__global__ void __launch_bounds__(256) copy_kernel(const f4p* __restrict__ src,
                                                   f4p* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const f4p v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
    dst[i] = v0;
    dst[i + stride] = v1;
    dst[i + 2 * stride] = v2;
    dst[i + 3 * stride] = v3;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace bmk

using namespace bmk;

extern "C" {

bm_status bm_peak_mfma(int32_t precision, int32_t shape, int32_t iterations, void* stream,
                       double* tflops) {
  if (!tflops || iterations < 1 || shape < 0 || shape > 1) return fail(BM_EINVAL, "bad argument");
  if (precision < BM_PREC_FP32 || precision > BM_PREC_FP16X3)
    return fail(BM_EINVAL, "unknown precision %d", precision);
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  hipStream_t s = (hipStream_t)stream;
  float* out = nullptr;
  if ((e = hipMalloc(&out, 256 * sizeof(float))) != hipSuccess) return hip_fail(e, "hipMalloc");
  // four 4-wave blocks per compute unit: four waves per SIMD
  const int blocks = 4 * n_cu;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  auto launch = [&](int iters) {
    (void)hipGetLastError();
    const dim3 g(blocks), b(256);
    if (shape == 0) {
      if (precision == BM_PREC_FP32)
        hipLaunchKernelGGL((mfma_loop_kernel<BM_PREC_FP32, 0>), g, b, 0, s, out, iters, 1e-3f);
      else if (precision == BM_PREC_FP16X3)
        hipLaunchKernelGGL((mfma_loop_kernel<BM_PREC_FP16X3, 0>), g, b, 0, s, out, iters, 1e-3f);
      else
        hipLaunchKernelGGL((mfma_loop_kernel<BM_PREC_BF16X4, 0>), g, b, 0, s, out, iters, 1e-3f);
    } else {
      if (precision == BM_PREC_FP32)
        hipLaunchKernelGGL((mfma_loop_kernel<BM_PREC_FP32, 1>), g, b, 0, s, out, iters, 1e-3f);
      else if (precision == BM_PREC_FP16X3)
        hipLaunchKernelGGL((mfma_loop_kernel<BM_PREC_FP16X3, 1>), g, b, 0, s, out, iters, 1e-3f);
      else
        hipLaunchKernelGGL((mfma_loop_kernel<BM_PREC_BF16X4, 1>), g, b, 0, s, out, iters, 1e-3f);
    }
    return hipGetLastError();
  };
  e = launch(iterations / 8 + 1);  // warm-up (clocks)
  if (e == hipSuccess) e = hipEventRecord(t0, s);
  if (e == hipSuccess) e = launch(iterations);
  if (e == hipSuccess) e = hipEventRecord(t1, s);
  if (e == hipSuccess) e = hipEventSynchronize(t1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  (void)hipFree(out);
  if (e != hipSuccess) return hip_fail(e, "matrix-op probe");
  const double mn = shape == 0 ? 16.0 * 16 : 32.0 * 32;
  const double k = precision == BM_PREC_FP32 ? (shape == 0 ? 4 : 2) : (shape == 0 ? 32 : 16);
  const double ops = (double)blocks * 4 /*waves*/ * kPeakChains * (double)iterations;
  *tflops = 2.0 * mn * k * ops / (ms * 1e-3) / 1e12;
  return BM_OK;
}

bm_status bm_peak_copy(int64_t bytes, int32_t repeats, void* stream, double* gbps) {
  if (!gbps || bytes < (1 << 20) || repeats < 1) return fail(BM_EINVAL, "bad argument");
  const int64_t n = bytes / 16;
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  hipStream_t s = (hipStream_t)stream;
  void *src = nullptr, *dst = nullptr;
  if ((e = hipMalloc(&src, n * 16)) != hipSuccess) return hip_fail(e, "hipMalloc");
  if ((e = hipMalloc(&dst, n * 16)) != hipSuccess) {
    (void)hipFree(src);
    return hip_fail(e, "hipMalloc");
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  const int blocks = 16 * n_cu;
  float best = 0.f;
  e = hipMemsetAsync(src, 0, n * 16, s);
  for (int r = 0; r <= repeats && e == hipSuccess; ++r) {  // r = 0: warm-up
    (void)hipGetLastError();
    if ((e = hipEventRecord(t0, s)) != hipSuccess) break;
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, s,
                       static_cast<const f4p*>(src), static_cast<f4p*>(dst), n);
    if ((e = hipGetLastError()) != hipSuccess) break;
    if ((e = hipEventRecord(t1, s)) != hipSuccess) break;
    if ((e = hipEventSynchronize(t1)) != hipSuccess) break;
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
    if (r > 0 && (best == 0.f || ms < best)) best = ms;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  (void)hipFree(src);
  (void)hipFree(dst);
  if (e != hipSuccess) return hip_fail(e, "copy probe");
  *gbps = 2.0 * (double)n * 16 / (best * 1e-3) / 1e9;
  return BM_OK;
}

}  // extern "C"
