// Rounding of float32 values to the bfloat16 hi + lo split shared by the split cross-term
// kernels and the norm pass.
//
// hi = RNE_bf16(x), lo = RNE_bf16(x - hi); hi + lo has at most 16 significant bits, so it is
// exact in float32.  The bfloat16 split form pairs its cross term (all four products of the
// parts) with the norms of these rounded values, so that N'_i + N'_j - 2 C'_ij is the exact
// squared distance of the rounded patches (Lemma 2 applied to the rounded image) and the
// cancellation leaves no rounding bias from the split.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmk {

// Bits of RNE_bf16(v) (v finite).
__device__ __forceinline__ uint32_t bf16_rne_bits(float v) {
  const uint32_t b = __float_as_uint(v);
  return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

// hi + lo of the bfloat16 split of v, as a float32 value.
__device__ __forceinline__ float bf16_split_value(float v) {
  const float hi = __uint_as_float(bf16_rne_bits(v) << 16);
  const float lo = __uint_as_float(bf16_rne_bits(v - hi) << 16);
  return hi + lo;
}

}  // namespace bmk
