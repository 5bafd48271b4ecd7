// Kernel entry points of the fused window-masked cross-correlation + distance assembly +
// top-K for gfx950 (C <= 4 channels, patch side 3..8, K <= 32, a candidate span of NT * 16
// columns per 4 x 4 reference block): the single-image kernel and the 3D (volume) kernel,
// both one workgroup per reference block in XCD-aware order, and the dispatch tables over
// (precision, channels, patch, K registers, span tiles).  The block itself (Lemma 2's
// distance assembly on the matrix cores, Theorem 1's selection with one reference per
// lane) is lane_block of xcorr_lane.h; the contraction policy (contract.h) selects float32
// products or the hi/lo split forms.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>
#include <stdint.h>

#include "bm_internal.h"
#include "contract.h"
#include "xcorr_common.h"
#include "xcorr_lane.h"

namespace bmk {

// Waves per SIMD the compiler keeps registers for: the 1-channel split blocks fit four
// 4-wave workgroups per compute unit in LDS, so their registers are held to 128 (they need
// about 100-120).
template <class CT, int C, int KR>
constexpr int fast_waves_per_eu() { return (CT::kSplit && C == 1) ? 4 : 1; }

// Single image: one workgroup per reference block, XCD-aware block order.
template <class CT, int C, int KR, int NT>
__global__ void __launch_bounds__(64 * fast_max_waves(CT::kSplit ? 1 : 0, C))
__attribute__((amdgpu_waves_per_eu(fast_waves_per_eu<CT, C, KR>())))
xcorr_topk_fast(const float* __restrict__ img, const float* __restrict__ nrm,
                const float* __restrict__ centers, const float* __restrict__ amax,
                int* __restrict__ out_idx, float* __restrict__ out_dist, const FastGeom g) {
  extern __shared__ __align__(16) unsigned char lds[];
  lane_block<CT, C, KR, NT, false>(img, nrm, centers, amax, out_idx, out_dist, g,
                                   xcd_remap(blockIdx.x, g.nwg_total), lds);
}

typedef void (*XcFastKernel)(const float*, const float*, const float*, const float*, int*,
                             float*, const FastGeom);

// 3D search over a volume: one workgroup per (reference depth z, 4 x 4 reference block),
// XCD-aware order over both.  Norm maps (and max maps) of every slab are stacked by depth;
// outputs are stacked by reference depth.
template <class CT, int C, int KR, int NT>
__global__ void __launch_bounds__(64 * fast_max_waves(CT::kSplit ? 1 : 0, C))
xcorr_topk_depth(const float* __restrict__ vol, const float* __restrict__ nrm,
                 const float* __restrict__ amax, int* __restrict__ out_idx,
                 float* __restrict__ out_dist, const FastGeom g, const DepthGeom dg) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int t = xcd_remap(blockIdx.x, g.nwg_total * dg.Z);
  const int z = t / g.nwg_total;
  const int blk = t - z * g.nwg_total;
  const size_t slab = (size_t)g.H * g.W, nslab = (size_t)g.Hv * g.Wv;
  const size_t outs = (size_t)g.nry * g.nrx * g.K;
  const int lo = z - dg.before;
  const DepthWin dw{vol, nrm, amax, max(0, lo), min(dg.Z - 1, lo + dg.c - 1), dg.tiles};
  lane_block<CT, C, KR, NT, true>(vol + z * slab, nrm + z * nslab, nullptr,
                                  amax ? amax + (size_t)z * dg.tiles : nullptr,
                                  out_idx + z * outs, out_dist + z * outs, g, blk, lds, &dw);
}

typedef void (*XcDepthKernel)(const float*, const float*, const float*, int*, float*,
                              const FastGeom, const DepthGeom);

// policy for (precision, C, H2): 0 float32, 1 bfloat16 split, 2 float16 split
template <int PREC, int C, int H2>
using CtFor = std::conditional_t<PREC == 0, CtF32<C, H2>, CtSplit<C, H2, PREC == 2>>;

template <int PREC, int C, int H2, int KR>
static XcDepthKernel depth_nt(int nt) {
  if constexpr (PREC != 0 && H2 < 3) {
    return nullptr;
  } else {
    switch (nt) {
      case 2: return xcorr_topk_depth<CtFor<PREC, C, H2>, C, KR, 2>;
      case 3: return xcorr_topk_depth<CtFor<PREC, C, H2>, C, KR, 3>;
    }
    return nullptr;
  }
}

template <int PREC, int C>
static XcDepthKernel depth_h2(int h2, int kr, int nt) {
  switch (h2 * 4 + kr) {
    case 2 * 4 + 1: return depth_nt<PREC, C, 2, 1>(nt);
    case 2 * 4 + 2: return depth_nt<PREC, C, 2, 2>(nt);
    case 3 * 4 + 1: return depth_nt<PREC, C, 3, 1>(nt);
    case 3 * 4 + 2: return depth_nt<PREC, C, 3, 2>(nt);
    case 4 * 4 + 1: return depth_nt<PREC, C, 4, 1>(nt);
    case 4 * 4 + 2: return depth_nt<PREC, C, 4, 2>(nt);
  }
  return nullptr;
}

template <int PREC, int C, int H2, int KR>
static XcFastKernel fast_nt(int nt) {
  if constexpr (PREC != 0 && H2 < 3) {
    return nullptr;  // split forms: patch side 5..8
  } else {
    switch (nt) {
      case 2: return xcorr_topk_fast<CtFor<PREC, C, H2>, C, KR, 2>;
      case 3: return xcorr_topk_fast<CtFor<PREC, C, H2>, C, KR, 3>;
    }
    return nullptr;
  }
}

template <int PREC, int C, int H2>
static XcFastKernel fast_kr(int kr, int nt) {
  switch (kr) {
    case 1: return fast_nt<PREC, C, H2, 1>(nt);
    case 2: return fast_nt<PREC, C, H2, 2>(nt);
  }
  return nullptr;
}

// All specialised kernels for one (precision, C): each is its own translation unit.
template <int PREC, int C>
static XcFastKernel fast_h2(int h2, int kr, int nt) {
  switch (h2) {
    case 2: return fast_kr<PREC, C, 2>(kr, nt);
    case 3: return fast_kr<PREC, C, 3>(kr, nt);
    case 4: return fast_kr<PREC, C, 4>(kr, nt);
  }
  return nullptr;
}

}  // namespace bmk
