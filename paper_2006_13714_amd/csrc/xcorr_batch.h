// Persistent cross-term / distance / top-K launch over many images of uneven shapes.
//
// The workgroups of one launch (as many as the device keeps resident) repeatedly take the
// next work item from a device counter until the list is exhausted.  A work item is one
// 4 x 4 reference block of one image; the host orders the images by decreasing cost per
// block, so the last items handed out are the cheapest and the tail stays short.  Each item
// runs exactly the per-block computation of the single-image kernel (xcorr_fast.h) with
// its image's geometry and per-image tuned parameters (bounding-sweep row step, buffer
// capacity); the shape class (channels, patch side) selects the compiled body.
//
// A kernel's register count and workgroup shape, and with them how many workgroups a
// compute unit keeps, are shared by every body compiled into it.  The bodies are therefore
// grouped in tiers of similar shape (batch_tier): float32 tier 3 holds one channel, tier 0
// two and three channels and tier 1 four channels; the split forms' tier 0 holds one
// channel and tier 2 two to four channels (8-wave blocks).  A batch runs one persistent
// launch per tier present.
#pragma once

#include "batch.h"
#include "xcorr_fast.h"

namespace bmk {

template <int PREC, int KR, int NT, int C, int H2, bool NSTRIP>
__device__ __forceinline__ void batch_block(const BatchXc& r, int blk, unsigned char* lds) {
  if constexpr (PREC != 0 && H2 < 3) {
    // split forms need patch sides 5..8; the host never forms such items
    (void)r, (void)blk, (void)lds;
  } else {
    (void)NSTRIP;
    lane_block<CtFor<PREC, C, H2>, C, KR, NT, false>(r.img, r.nrm, r.centers, r.amax, r.idx,
                                                     r.dist, r.g, blk, lds);
  }
}

template <int PREC, int KR, int NT, int TIER, int C, int H2>
__device__ __forceinline__ void batch_tier_block(const BatchXc& r, int blk, unsigned char* lds) {
  if constexpr (batch_tier(PREC, C) == TIER)
    batch_block<PREC, KR, NT, C, H2, batch_norm_strip(PREC, TIER)>(r, blk, lds);
  else
    (void)r, (void)blk, (void)lds;
}

// waves per SIMD the compiler must leave room for: float32 tier 0 (2..3 channels) keeps
// two; the float32 1-channel tier three (its bodies need under 168 registers); the 8-wave
// tier needs two per SIMD by construction; the split forms' 1-channel tier with K <= 16
// fits three (168 registers, no spills), with larger K it keeps the compiler's choice
constexpr int batch_min_waves(int prec, int tier, int kr) {
  if (tier == 1) return 1;
  if (tier == 3) return 3;
  if (prec == 0 || tier == 2) return 2;
  return kr == 1 ? 3 : 1;
}

template <int PREC, int KR, int NT, int TIER>
__global__ void __launch_bounds__(64 * batch_max_waves(TIER))
__attribute__((amdgpu_waves_per_eu(batch_min_waves(PREC, TIER, KR))))
xcorr_topk_batch(const BatchXc* __restrict__ recs, int n_recs, int n_items,
                 unsigned* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int s_item;
  for (;;) {
    // every wave of the previous item has passed the item's internal barriers, and all
    // reach this barrier before the next item's staging overwrites LDS
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= n_items) break;
    int lo = 0, hi = n_recs - 1;  // last image whose first item is <= it
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (load_uniform(&recs[mid].item_begin) <= it) lo = mid;
      else hi = mid - 1;
    }
    const BatchXc r = load_uniform(&recs[lo]);
    const int blk = it - r.item_begin;
    switch (r.cls) {
      case 0: batch_tier_block<PREC, KR, NT, TIER, 1, 2>(r, blk, lds); break;
      case 1: batch_tier_block<PREC, KR, NT, TIER, 1, 3>(r, blk, lds); break;
      case 2: batch_tier_block<PREC, KR, NT, TIER, 1, 4>(r, blk, lds); break;
      case 3: batch_tier_block<PREC, KR, NT, TIER, 2, 2>(r, blk, lds); break;
      case 4: batch_tier_block<PREC, KR, NT, TIER, 2, 3>(r, blk, lds); break;
      case 5: batch_tier_block<PREC, KR, NT, TIER, 2, 4>(r, blk, lds); break;
      case 6: batch_tier_block<PREC, KR, NT, TIER, 3, 2>(r, blk, lds); break;
      case 7: batch_tier_block<PREC, KR, NT, TIER, 3, 3>(r, blk, lds); break;
      case 8: batch_tier_block<PREC, KR, NT, TIER, 3, 4>(r, blk, lds); break;
      case 9: batch_tier_block<PREC, KR, NT, TIER, 4, 2>(r, blk, lds); break;
      case 10: batch_tier_block<PREC, KR, NT, TIER, 4, 3>(r, blk, lds); break;
      case 11: batch_tier_block<PREC, KR, NT, TIER, 4, 4>(r, blk, lds); break;
      default: break;
    }
  }
}

typedef void (*XcBatchKernel)(const BatchXc*, int, int, unsigned*);

template <int PREC, int KR, int NT>
static XcBatchKernel batch_tier_kernel(int tier) {
  switch (tier) {
    case 0: return xcorr_topk_batch<PREC, KR, NT, 0>;
    case 1:
      if constexpr (PREC == 0) return xcorr_topk_batch<PREC, KR, NT, 1>;
      break;
    case 2:
      if constexpr (PREC != 0) return xcorr_topk_batch<PREC, KR, NT, 2>;
      break;
    case 3:
      if constexpr (PREC == 0) return xcorr_topk_batch<PREC, KR, NT, 3>;
      break;
  }
  return nullptr;
}

}  // namespace bmk
