// Definitions shared by the specialised cross-term kernels (xcorr_fast.h, xcorr_lane.h).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bm_internal.h"

namespace bmk {

// Upper bound of max |x - centre| over the strip rows [y0, y1] x columns [x0, x1] (image
// coordinates, already clipped) in `nmap` stacked per-tile maps of the norm pass (`stride`
// entries apart): the largest entry over the tiles that hold those pixels.  The lanes read
// the entries in parallel and a wave-wide max reduces them; the result is the same in
// every lane and every wave.
__device__ __forceinline__ float strip_absmax(const float* __restrict__ amax, const FastGeom& g,
                                              int y0, int y1, int x0, int x1, int lane,
                                              int nmap = 1, size_t stride = 0) {
  const int ty0 = min(y0 / kNormTY, g.nty - 1), ty1 = min(y1 / kNormTY, g.nty - 1);
  const int tx0 = min(x0 / kNormTX, g.ntx - 1), tx1 = min(x1 / kNormTX, g.ntx - 1);
  const int nx = tx1 - tx0 + 1, per = nx * (ty1 - ty0 + 1);
  float m = 0.f;
  for (int i = lane; i < per * nmap; i += 64) {
    const int k = i / per, e = i - k * per;
    const int ty = ty0 + e / nx, tx = tx0 + e - (e / nx) * nx;
    m = fmaxf(m, amax[k * stride + (size_t)ty * g.ntx + tx]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  return m;
}

// Candidate slabs of a 3D search (Sec. IV, 3D Self-Convolution): the reference's d-channel
// slab is the one passed to lane_block as `img` / `nrm`; its candidates come from the
// d-channel slabs z0..z1 of the volume (channel planes of H x W), each with its own norm map
// (Hv x Wv) and, in the float16 form, its own per-tile max map.
struct DepthWin {
  const float* vol;
  const float* nrm;
  const float* amax;
  int z0, z1;
  int tiles;  // entries of one slab's max map
};

}  // namespace bmk
