// Patch-norm box filter for gfx950.
//
// N[y][x] = sum_c sum_{l<P} sum_{m<P} (X_c[y+l][x+m] - center_c)^2, the entries of
// h_X (.) h_X (Sec. III-B, the normalisation vector h_X; used by Lemma 2).  center_c comes
// from the centring pass when centring is on (centers[c]); otherwise it is zero.
//
// One workgroup of 256 threads produces a kNormTY x kNormTX output tile (one output per
// thread; 8 x 32, so a 512 x 512 image gives 1024 workgroups and every compute unit has
// several to overlap their load / sum / store phases).  It stages the (TY+P-1) x (TX+P-1)
// input window of one channel in LDS with coalesced row loads, forms the horizontal P-tap
// sums of squares, then the vertical P-tap sums, and accumulates over channels.  Sums are
// direct (no prefix or summed-area tables, whose rounding grows with the image) and
// carried in float64, so every output is the float32 rounding of the exact norm.  Each
// input element is read once from HBM (halos come from L2) and each output written once.
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

static_assert(kNormTX * kNormTY == 256, "one output per thread");

struct NormLds {
  float tile[kNormTY + kMaxP - 1][kNormTX + kMaxP];
  double hs[kNormTY + kMaxP - 1][kNormTX];
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
  const int orow = t / kNormTX, ocol = t - (t / kNormTX) * kNormTX;  // this thread's output
  double acc = 0.0;
  float vmax = 0.f;

  for (int c = 0; c < g.C; ++c) {
    const float* plane = img + (size_t)c * g.H * g.W;
    const float cc = centers ? centers[c] : 0.f;
    for (int i = t; i < rows * cols; i += 256) {
      const int rr = i / cols, xx = i - (i / cols) * cols;
      const int y = oy0 + rr, x = ox0 + xx;
      float v = 0.f;
      if (y < g.H && x < g.W) v = plane[(size_t)y * g.W + x] - cc;
      if (g.round_bf16) v = bf16_split_value(v);
      sh.tile[rr][xx] = v;
      vmax = fmaxf(vmax, fabsf(v));
    }
    __syncthreads();
    for (int i = t; i < rows * kNormTX; i += 256) {
      const int rr = i / kNormTX, cx = i - (i / kNormTX) * kNormTX;
      double s = 0.0;
      for (int m = 0; m < g.P; ++m) {
        const double v = (double)sh.tile[rr][cx + m];
        s += v * v;
      }
      sh.hs[rr][cx] = s;
    }
    __syncthreads();
    double s = 0.0;
    for (int l = 0; l < g.P; ++l) s += sh.hs[orow + l][ocol];
    acc += s;
    __syncthreads();
  }
  {
    const int oy = oy0 + orow, ox = ox0 + ocol;
    if (oy < g.Hv && ox < g.Wv) out[(size_t)oy * g.Wv + ox] = (float)acc;
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

__global__ void __launch_bounds__(256)
norm_box_kernel(const float* __restrict__ img, float* __restrict__ out, NormGeom g,
                const float* __restrict__ centers, float* __restrict__ amax) {
  __shared__ NormLds sh;
  norm_tile(img, out, g, centers, amax, blockIdx.x, blockIdx.y, sh);
}

__global__ void __launch_bounds__(256)
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
