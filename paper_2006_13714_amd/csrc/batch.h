// Device records of the uneven-batch path (one launch over many images of different
// shapes) and the helper that reads them as wave-uniform values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bm_internal.h"

namespace bmk {

// One image of a batch norm launch.  Images are laid out in launch order; image i owns
// the workgroups [tile_begin, next image's tile_begin).
struct BatchNorm {
  const float* img;
  float* out;
  const float* centers;  // per-channel centring constants or null
  float* amax;           // per-tile max |x - centre| map or null
  NormGeom g;
  int tile_begin, tiles_x;
};

// One image of a persistent cross-term launch.  Images of one launch are stored in the
// order their work is handed out; image i owns items [item_begin, next item_begin).
struct BatchXc {
  const float* img;
  const float* nrm;
  const float* centers;
  const float* amax;
  int* idx;
  float* dist;
  int cls;         // shape class: (C - 1) * 3 + (ceil(P / 2) - 2)
  int item_begin;  // first work item (reference block) of this image in its launch
  FastGeom g;
};

constexpr int kBatchClasses = 12;  // C 1..4 x ceil(P/2) 2..4

// Read a record at a wave-uniform address into scalar registers.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "record size");
  constexpr int n = sizeof(T) / 4;
  uint32_t w[n];
  __builtin_memcpy(w, p, sizeof(T));
#pragma unroll
  for (int i = 0; i < n; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  T out;
  __builtin_memcpy(&out, w, sizeof(T));
  return out;
}

}  // namespace bmk
