// Patch-norm box filter for gfx950.
//
// N[y][x] = sum_c sum_{l<P} sum_{m<P} (X_c[y+l][x+m] - center_c)^2, the entries of
// h_X (.) h_X (Sec. III-B, the normalisation vector h_X; used by Lemma 2).  center_c comes
// from the centring pass when centring is on (centers[c]); otherwise it is zero.
//
// One workgroup of 256 threads produces a kNormTY x kNormTX output tile (16 x 64: four
// outputs per thread, one column and four rows).  Per channel it stages the
// (TY+P-1) x (TX+P-1) input window in LDS (each thread keeps the twelve loads of each of
// up to four channels in flight together, in rows of 32 consecutive columns, no index
// divisions), adds the horizontal P-tap sums of
// squares of its columns into per-thread float64 accumulators (channels summed there),
// and after the last channel forms the vertical P-tap sums.  Sums are direct (no prefix or
// summed-area tables, whose rounding grows with the image) and carried in float64, so every
// output is the float32 rounding of the exact norm.  Each input element is read once from
// HBM (halos come from L2) and each output written once.
//
// For the bfloat16 split form the staged values are first rounded to hi + lo (split16.h),
// so the map holds the norms of the rounded image that the form's cross term multiplies.
//
// Each tile also writes max |x - center_c| over its staged window (all channels) to a
// per-tile map when asked; the float16 split form takes its per-block pre-scale from it.
//
// The batch form covers many images in one launch: workgroup b finds its image by a
// binary search over the images' first tile numbers.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "bm_internal.h"
#include "split16.h"

namespace bmk {

constexpr int kMaxP = 16;
constexpr int kStageRows = kNormTY + kMaxP - 1;  // 31
constexpr int kStageCols = kNormTX + kMaxP - 1;  // 79
constexpr int kStageRS = 80;                     // LDS row stride (floats)

static_assert(kNormTX == 64 && kNormTY == 16, "thread layout below");

struct NormLds {
  float tile[kStageRows][kStageRS];
  double hs[kStageRows][kNormTX];
  float red[4];
};

__device__ __forceinline__ void norm_tile(const float* __restrict__ img, float* __restrict__ out,
                                          const NormGeom& g, const float* __restrict__ centers,
                                          float* __restrict__ amax, int bx, int by, NormLds& sh) {
  const int t = threadIdx.x;
  const int ox0 = bx * kNormTX;
  const int oy0 = by * kNormTY;
  const int rows = kNormTY + g.P - 1;
  const int cols = kNormTX + g.P - 1;
  // staging layout: 8 rows x 32 columns of threads, 4 x 3 loads each
  const int ly = t >> 5, lx = t & 31;
  // horizontal sums: column hc, rows hr + 4 k; vertical sums: column hc, rows 4 vr .. + 3
  const int hc = t & 63, hr = t >> 6;
  double hacc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) hacc[k] = 0.0;
  float vmax = 0.f;

  // The loads of up to kNormPre channels are in flight together from the start (channel
  // c + kNormPre's are issued as channel c's registers free up), so one load latency is
  // exposed per kNormPre channels instead of one per channel.
  constexpr int kNormPre = 4;
  float v[kNormPre][4][3];
  auto load = [&](int c, float (&dst)[4][3]) __attribute__((always_inline)) {
    const float* plane = img + (size_t)c * g.H * g.W;
    const float cc = centers ? centers[c] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int y = oy0 + ly + 8 * i, x = ox0 + lx + 32 * j;
        const bool ok = (ly + 8 * i < rows) & (lx + 32 * j < cols) & (y < g.H) & (x < g.W);
        dst[i][j] = ok ? plane[(size_t)y * g.W + x] - cc : 0.f;
      }
  };
#pragma unroll
  for (int u = 0; u < kNormPre; ++u)
    if (u < g.C) load(u, v[u]);
  for (int c0 = 0; c0 < g.C; c0 += kNormPre) {
#pragma unroll
    for (int u = 0; u < kNormPre; ++u) {
      const int c = c0 + u;
      if (c >= g.C) break;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          float x = v[u][i][j];
          if (g.round_bf16) x = bf16_split_value(x);
          vmax = fmaxf(vmax, fabsf(x));
          if ((ly + 8 * i < kStageRows) & (lx + 32 * j < kStageRS))
            sh.tile[ly + 8 * i][lx + 32 * j] = x;
        }
      __syncthreads();
      if (c + kNormPre < g.C) load(c + kNormPre, v[u]);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int r = hr + 4 * k;
        if (r < rows) {
          double s = 0.0;
          for (int m = 0; m < g.P; ++m) {
            const double x = (double)sh.tile[r][hc + m];
            s = fma(x, x, s);
          }
          hacc[k] += s;
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (hr + 4 * k < rows) sh.hs[hr + 4 * k][hc] = hacc[k];
  __syncthreads();
  {
    const int ox = ox0 + hc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int orow = 4 * hr + q;
      double s = 0.0;
      for (int l = 0; l < g.P; ++l) s += sh.hs[orow + l][hc];
      const int oy = oy0 + orow;
      if (oy < g.Hv && ox < g.Wv) out[(size_t)oy * g.Wv + ox] = (float)s;
    }
  }
  if (amax) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o));
    if ((t & 63) == 0) sh.red[t >> 6] = vmax;
    __syncthreads();
    if (t == 0) {
      const int ntx = (g.Wv + kNormTX - 1) / kNormTX;
      amax[by * ntx + bx] = fmaxf(fmaxf(sh.red[0], sh.red[1]), fmaxf(sh.red[2], sh.red[3]));
    }
  }
}

// four workgroups (16 waves) per compute unit: registers held to 128
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
norm_box_kernel(const float* __restrict__ img, float* __restrict__ out, NormGeom g,
                const float* __restrict__ centers, float* __restrict__ amax) {
  __shared__ NormLds sh;
  norm_tile(img, out, g, centers, amax, blockIdx.x, blockIdx.y, sh);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
norm_box_batch_kernel(const BatchNorm* __restrict__ items, int n, unsigned* __restrict__ counters,
                      int n_counters) {
  __shared__ NormLds sh;
  // the persistent cross-term launches that follow on the stream start from zero
  if (blockIdx.x == 0 && (int)threadIdx.x < n_counters) counters[threadIdx.x] = 0u;
  const int b = blockIdx.x;
  int lo = 0, hi = n - 1;  // last image whose first tile is <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (load_uniform(&items[mid].tile_begin) <= b) lo = mid;
    else hi = mid - 1;
  }
  const BatchNorm it = load_uniform(&items[lo]);
  const int t = b - it.tile_begin;
  const int ty = t / it.tiles_x;
  norm_tile(it.img, it.out, it.g, it.centers, it.amax, t - ty * it.tiles_x, ty, sh);
}

void norm_tiles(const NormGeom& g, int* tiles_x, int* tiles_y) {
  *tiles_x = (g.Wv + kNormTX - 1) / kNormTX;
  *tiles_y = (g.Hv + kNormTY - 1) / kNormTY;
}

hipError_t launch_norm(const float* img, float* out, const NormGeom& g, const float* centers,
                       float* amax, hipStream_t stream) {
  int tx, ty;
  norm_tiles(g, &tx, &ty);
  (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
  hipLaunchKernelGGL(norm_box_kernel, dim3(tx, ty), dim3(256), 0, stream, img, out, g, centers,
                     amax);
  return hipGetLastError();
}

hipError_t launch_norm_batch(const BatchNorm* d_items, int n, int total_tiles,
                             unsigned* d_counters, int n_counters, hipStream_t stream) {
  if (n < 1 || total_tiles < 1 || n_counters > 256) return hipErrorInvalidValue;
  (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
  hipLaunchKernelGGL(norm_box_batch_kernel, dim3(total_tiles), dim3(256), 0, stream, d_items, n,
                     d_counters, n_counters);
  return hipGetLastError();
}

}  // namespace bmk
