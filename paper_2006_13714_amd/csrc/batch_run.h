// Host entry to the uneven-batch launch sequence, shared by bm_match_batch and the server.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace bmk {

// One image of a batch: its plan, image, norm map and the norm pass's auxiliary slots
// (device memory the caller owns; see aux_at) and outputs.
struct BatchEntry {
  const bm_plan_s* plan;
  const float* img;
  float* nrm;
  NormAux aux;
  int32_t* idx;
  float* dist;
};

// Device bytes of the launch header (work counters and records) for n images.
int64_t batch_header_bytes(int n);

// Enqueue the whole batch on `s`; d_header holds batch_header_bytes(n) bytes and must not
// be reused before the launches have finished.
bm_status run_batch(const BatchEntry* e, int n, void* d_header, hipStream_t s);

}  // namespace bmk
