// Group gather and aggregation for gfx950 (Sec. IV, image reconstruction): after block
// matching, the group of reference i is Y_i = [X_{S_i(1)}, ..., X_{S_i(K)}]; a restorer
// processes each group and deposits every patch back at its location, dividing each pixel
// by the number of deposited patches covering it.
//
// Both are HBM-bound element-wise passes over the n_ref K C P^2 group values.
//  * gather: a workgroup takes a run of (reference, k) items; each lane keeps one fixed
//    element offset of an item (no per-element division), writes are coalesced.  An index
//    that is -1 or names no valid patch position gives a zero patch.
//  * aggregate: sums are 64-bit integers of fixed-point values, so they are exact up to one
//    rounding per contribution and independent of the order additions land in (bitwise
//    deterministic).  The fixed-point exponent E comes from a device-side max |value| pass:
//    |v| < 2^e, E = 62 - e - ceil(log2(n_ref K + 1)), so no sum of at most n_ref K
//    contributions can overflow.  Deposits are accumulated per tile of tb x tb references
//    (one workgroup per tile and channel) in LDS, over the region their search windows
//    cover, and the region is added to the image accumulators once; a deposit outside the
//    region (an index that is not a window member) goes to the image accumulators directly.
//    Coverage counts need no per-element work: the count of pixel p is the number of
//    deposited patches whose P x P footprint holds p, i.e. the P x P box sum of the
//    histogram of patch positions, which takes one 32-bit atomic per (reference, k) item.
//    The final pass box-filters the histogram in LDS, divides in float64 and rounds once
//    to float32.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bm_internal.h"

namespace bmk {

constexpr int kGroupThreads = 256;
constexpr int kTileLdsBytes = 64 * 1024;  // LDS of one aggregation tile's accumulators

__device__ __forceinline__ bool valid_position(int j, const GroupGeom& g, int* qy, int* qx) {
  if (j < 0) return false;
  const int y = j / g.W, x = j - y * g.W;
  if (y >= g.Hv || x >= g.Wv) return false;
  *qy = y;
  *qx = x;
  return true;
}

// Lane layout over items of `per` elements: with per <= 64 a wave covers 64 / per items at
// once and lane l keeps element l % per of item l / per; otherwise one item, lanes striding
// its elements by 64.
struct ItemLanes {
  int ipw;   // items per wave step
  int sub;   // this lane's item within the step
  int e0;    // this lane's first element
  int step;  // element stride within an item
  bool on;   // lane holds an element
};

__device__ __forceinline__ ItemLanes item_lanes(int per, int lane) {
  ItemLanes L;
  if (per <= 64) {
    L.ipw = 64 / per;
    L.sub = lane / per;
    L.e0 = lane - L.sub * per;
    L.step = per;
    L.on = L.sub < L.ipw;
  } else {
    L.ipw = 1;
    L.sub = 0;
    L.e0 = lane;
    L.step = 64;
    L.on = true;
  }
  return L;
}

// items [blockIdx.x * ib, ...) of the n_ref * K (reference, k) items; each lane takes kU
// items per pass so their index and pixel loads are in flight together
constexpr int kU = 4;

__global__ void __launch_bounds__(kGroupThreads)
gather_kernel(const float* __restrict__ img, const int32_t* __restrict__ idx,
              float* __restrict__ groups, GroupGeom g, int ib) {
  const int PP = g.P * g.P, CPP = g.C * PP;
  const long long i0 = (long long)blockIdx.x * ib;
  const long long items = g.n_ref * g.K;
  const int n_items = (int)min((long long)ib, items - i0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const ItemLanes L = item_lanes(CPP, lane);
  if (!L.on) return;
  const int stride = (kGroupThreads / 64) * L.ipw;
  // loads are unconditional (clamped to valid addresses) and masked afterwards, so the kU
  // items' loads issue back to back
  for (int it0 = wave * L.ipw + L.sub; it0 < n_items; it0 += kU * stride) {
    int j[kU], base[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) j[u] = idx[i0 + min(it0 + u * stride, n_items - 1)];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      int qy = 0, qx = 0;
      base[u] = (it0 + u * stride < n_items && valid_position(j[u], g, &qy, &qx))
                    ? qy * g.W + qx : -1;
    }
    for (int e = L.e0; e < CPP; e += L.step) {
      const int c = e / PP;
      const int rem = e - c * PP;
      const int l = rem / g.P;
      const int off = (c * g.H + l) * g.W + (rem - l * g.P);
      float v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) v[u] = img[(size_t)max(base[u], 0) + off];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int it = it0 + u * stride;
        if (it < n_items) groups[(i0 + it) * CPP + e] = base[u] >= 0 ? v[u] : 0.f;
      }
    }
  }
}

// accumulators [C*H*W] int64, position histogram [H*W] int32 (index qy * W + qx), max-|v|
// slot (uint bits of a float)
__global__ void __launch_bounds__(kGroupThreads)
agg_zero_kernel(unsigned long long* __restrict__ acc, int* __restrict__ cnt,
                unsigned* __restrict__ slot, long long n_acc, long long n_cnt) {
  for (long long e = (long long)blockIdx.x * kGroupThreads + threadIdx.x; e < n_acc;
       e += (long long)gridDim.x * kGroupThreads) {
    acc[e] = 0ull;
    if (e < n_cnt) cnt[e] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *slot = 0u;
}

// max |v| over `total` values; VEC: 16-byte loads of the 4-aligned bulk, then the tail
template <bool VEC>
__global__ void __launch_bounds__(kGroupThreads)
agg_absmax_kernel(const float* __restrict__ groups, long long total, unsigned* __restrict__ slot) {
  __shared__ float red[kGroupThreads / 64];
  float m = 0.f;
  const long long tid = (long long)blockIdx.x * kGroupThreads + threadIdx.x;
  const long long nth = (long long)gridDim.x * kGroupThreads;
  long long done = 0;
  if constexpr (VEC) {
    // four independent 16-byte loads per pass (indices clamped: a repeated element does not
    // change a maximum)
    const float4* g4 = reinterpret_cast<const float4*>(groups);
    const long long n4 = total >> 2;
    for (long long e = tid; e < n4; e += 4 * nth) {
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = g4[min(e + u * nth, n4 - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        m = fmaxf(m, fmaxf(fmaxf(fabsf(v[u].x), fabsf(v[u].y)), fmaxf(fabsf(v[u].z), fabsf(v[u].w))));
    }
    done = n4 << 2;
  }
  for (long long e = done + tid; e < total; e += nth) m = fmaxf(m, fabsf(groups[e]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kGroupThreads / 64; ++w) m = fmaxf(m, red[w]);
    atomicMax(slot, __float_as_uint(m));  // non-negative floats order like their bits
  }
}

__device__ __forceinline__ int fixed_exponent(unsigned slot_bits, int cnt_bits) {
  const float m = __uint_as_float(slot_bits);
  const int e = m > 0.f ? ilogbf(m) + 1 : 0;  // m < 2^e
  return max(-200, min(200, 62 - e - cnt_bits));
}

// round(v 2^E) as a two's-complement 64-bit integer.  |v 2^E| < 2^62 by the choice of E, so
// x = v 2^E is exact in float (a power-of-two scaling; |x| < 0.5 may flush to 0 and rounds
// to 0 either way) and r = rint(x) is an integer float.  The magnitude a = |r| splits into
// exact halves hi = floor(a 2^-32) and lo = a - hi 2^32 (a has at most 24 significant bits,
// so lo is a multiple of a's ulp below 2^32); the sign is applied in integers.
__device__ __forceinline__ unsigned long long to_fixed(float v, int E) {
  const float r = rintf(ldexpf(v, E));
  const float a = fabsf(r);
  const float hi = floorf(a * 0x1p-32f);
  const float lo = fmaf(hi, -0x1p32f, a);
  const unsigned long long mag =
      ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo;
  return r < 0.f ? 0ull - mag : mag;
}

// One workgroup of NTH threads per (tile of tb x tb references, channel c = blockIdx.y).
template <int NTH>
__global__ void __launch_bounds__(NTH)
agg_tile_kernel(const float* __restrict__ groups, const int32_t* __restrict__ idx,
                unsigned long long* __restrict__ acc, int* __restrict__ cnt,
                const unsigned* __restrict__ slot, GroupGeom g) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int n_px = g.th * g.tw;
  unsigned long long* accl = reinterpret_cast<unsigned long long*>(lds);
  const int c = blockIdx.y;
  const bool counts = c == 0;  // channel 0 workgroups add the position histogram
  const int ty = blockIdx.x / g.ntx, tx = blockIdx.x - (blockIdx.x / g.ntx) * g.ntx;
  const int ry0 = ty * g.tb, rx0 = tx * g.tb;
  const int nty_r = min(g.tb, g.nry - ry0), ntx_r = min(g.tb, g.nrx - rx0);
  const int Y0 = ry0 * g.s - g.r, X0 = rx0 * g.s - g.r;  // region origin (may be negative)

  for (int i = threadIdx.x; i < n_px; i += NTH) accl[i] = 0ull;
  __syncthreads();

  const int E = fixed_exponent(*slot, g.cnt_bits);
  const int PP = g.P * g.P;
  const int n_items = nty_r * ntx_r * g.K;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const ItemLanes L = item_lanes(PP, lane);
  if (L.on) {
    const int stride = (NTH / 64) * L.ipw;
    // loads unconditional (an item past the tile's end reads item 0 of the tile) and masked
    // afterwards, so the kU items' loads issue back to back
    for (int it0 = wave * L.ipw + L.sub; it0 < n_items; it0 += kU * stride) {
      long long item[kU];
      int j[kU], qyv[kU], qxv[kU];
      bool ok[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int it = it0 + u * stride < n_items ? it0 + u * stride : 0;
        const int ri = it / g.K;
        const int k = it - ri * g.K;
        const int a = ri / ntx_r;
        const int b = ri - a * ntx_r;
        item[u] = ((long long)(ry0 + a) * g.nrx + rx0 + b) * g.K + k;
        j[u] = idx[item[u]];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        qyv[u] = qxv[u] = 0;
        ok[u] = it0 + u * stride < n_items && valid_position(j[u], g, &qyv[u], &qxv[u]);
        if (counts && ok[u] && L.e0 == 0) atomicAdd(&cnt[qyv[u] * g.W + qxv[u]], 1);
      }
      // a patch wholly inside the region (every window member) takes region offset
      // rbase + l tw + m; others check each element
      int rbase[kU];
      bool inside[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int py = qyv[u] - Y0, px = qxv[u] - X0;
        inside[u] = ok[u] && (unsigned)py <= (unsigned)(g.th - g.P) &&
                    (unsigned)px <= (unsigned)(g.tw - g.P);
        rbase[u] = py * g.tw + px;
      }
      for (int e = L.e0; e < PP; e += L.step) {
        const int l = e / g.P;
        const int m = e - l * g.P;
        const int loff = l * g.tw + m;
        float v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] = groups[(item[u] * g.C + c) * PP + e];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          if (inside[u]) {
            atomicAdd(&accl[rbase[u] + loff], to_fixed(v[u], E));
          } else if (ok[u]) {
            const int qy = qyv[u], qx = qxv[u];
            const unsigned long long q = to_fixed(v[u], E);
            const int py = qy + l - Y0, px = qx + m - X0;
            if ((unsigned)py < (unsigned)g.th && (unsigned)px < (unsigned)g.tw)
              atomicAdd(&accl[py * g.tw + px], q);
            else
              atomicAdd(&acc[(size_t)c * g.H * g.W + (size_t)(qy + l) * g.W + qx + m], q);
          }
        }
      }
    }
  }
  __syncthreads();

  // add the region to the image accumulators (pixels outside the image hold no deposits)
  for (int i = threadIdx.x; i < n_px; i += NTH) {
    const int py = i / g.tw, px = i - (i / g.tw) * g.tw;
    const int y = Y0 + py, x = X0 + px;
    if ((unsigned)y >= (unsigned)g.H || (unsigned)x >= (unsigned)g.W) continue;
    const unsigned long long v = accl[i];
    if (v) atomicAdd(&acc[(size_t)c * g.H * g.W + (size_t)y * g.W + x], v);
  }
}

// Untiled deposits (a tile region that does not fit LDS): image accumulators directly.
__global__ void __launch_bounds__(kGroupThreads)
agg_deposit_kernel(const float* __restrict__ groups, const int32_t* __restrict__ idx,
                   unsigned long long* __restrict__ acc, int* __restrict__ cnt,
                   const unsigned* __restrict__ slot, GroupGeom g, int ib) {
  const int E = fixed_exponent(*slot, g.cnt_bits);
  const int PP = g.P * g.P, CPP = g.C * PP;
  const long long i0 = (long long)blockIdx.x * ib;
  const int n_items = (int)min((long long)ib, g.n_ref * g.K - i0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const ItemLanes L = item_lanes(CPP, lane);
  if (!L.on) return;
  for (int it = wave * L.ipw + L.sub; it < n_items; it += (kGroupThreads / 64) * L.ipw) {
    int qy, qx;
    if (!valid_position(idx[i0 + it], g, &qy, &qx)) continue;
    if (L.e0 == 0) atomicAdd(&cnt[qy * g.W + qx], 1);
    const float* src = groups + (i0 + it) * CPP;
    for (int e = L.e0; e < CPP; e += L.step) {
      const int c = e / PP;
      const int rem = e - c * PP;
      const int l = rem / g.P;
      const int m = rem - l * g.P;
      const size_t pix = (size_t)(qy + l) * g.W + qx + m;
      atomicAdd(&acc[(size_t)c * g.H * g.W + pix], to_fixed(src[e], E));
    }
  }
}

// Output tile of the normalisation: kNY x kNX pixels; the coverage count of pixel (y, x)
// is the sum of the position histogram over rows y-P+1..y and columns x-P+1..x, formed
// from an LDS copy of the histogram tile (column sums, then row sums).
constexpr int kNX = 64, kNY = 16, kPMax = 16;

__global__ void __launch_bounds__(kGroupThreads)
agg_normalise_kernel(const unsigned long long* __restrict__ acc, const int* __restrict__ hist,
                     const unsigned* __restrict__ slot, float* __restrict__ out, GroupGeom g) {
  __shared__ int hs[(kNY + kPMax - 1) * (kNX + kPMax - 1)];
  __shared__ int vs[kNY * (kNX + kPMax - 1)];
  const int P = g.P;
  const int HR = kNY + P - 1, HC = kNX + P - 1;
  const int x0 = blockIdx.x * kNX, y0 = blockIdx.y * kNY;
  for (int i = threadIdx.x; i < HR * HC; i += kGroupThreads) {
    const int r = i / HC, cc = i - (i / HC) * HC;
    const int y = y0 - P + 1 + r, x = x0 - P + 1 + cc;
    hs[i] = ((unsigned)y < (unsigned)g.H && (unsigned)x < (unsigned)g.W) ? hist[y * g.W + x] : 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kNY * HC; i += kGroupThreads) {
    const int r = i / HC, cc = i - (i / HC) * HC;
    int sum = 0;
    for (int l = 0; l < P; ++l) sum += hs[(r + l) * HC + cc];
    vs[i] = sum;
  }
  __syncthreads();
  const int E = fixed_exponent(*slot, g.cnt_bits);
  for (int i = threadIdx.x; i < kNY * kNX; i += kGroupThreads) {
    const int r = i / kNX, xx = i - (i / kNX) * kNX;
    const int y = y0 + r, x = x0 + xx;
    if (y >= g.H || x >= g.W) continue;
    int n = 0;
    for (int m = 0; m < P; ++m) n += vs[r * HC + xx + m];
    for (int c = 0; c < g.C; ++c) {
      const size_t e = ((size_t)c * g.H + y) * g.W + x;
      const double v = ldexp((double)(long long)acc[e], -E);
      out[e] = n > 0 ? (float)(v / n) : 0.f;
    }
  }
}

static int grid_for(long long total) {
  long long b = (total + kGroupThreads - 1) / kGroupThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

// items per workgroup of the item-run kernels: about 2048 elements each
static int items_per_block(int per) { return per >= 2048 ? 1 : 2048 / per; }

hipError_t launch_gather(const float* img, const int32_t* idx, float* groups, const GroupGeom& g,
                         hipStream_t s) {
  const long long items = g.n_ref * g.K;
  if (items == 0) return hipSuccess;
  const int ib = items_per_block(g.C * g.P * g.P);
  const long long blocks = (items + ib - 1) / ib;
  if (blocks >= (1ll << 31)) return hipErrorInvalidValue;
  (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)blocks), dim3(kGroupThreads), 0, s, img, idx,
                     groups, g, ib);
  return hipGetLastError();
}

// Tiling of the aggregation for a plan: the largest tb in {4, 2, 1} whose window region
// (th = (tb - 1) s + 2 r + P rows, likewise columns) fits kTileLdsBytes; tb = 0 if none does.
// (8 x 8 tiles on 1024-thread workgroups halve the region additions but measured slower:
// 146 vs 133 us on the 512 x 512 workload.)
void aggregate_tiling(GroupGeom& g) {
  g.tb = g.th = g.tw = g.ntx = g.nty = 0;
  for (int tb : {4, 2, 1}) {
    const long long th = (long long)(tb - 1) * g.s + g.wspan + g.P;
    if (th * th * 8 <= kTileLdsBytes) {
      g.tb = tb;
      g.th = g.tw = (int)th;
      g.ntx = (g.nrx + tb - 1) / tb;
      g.nty = (g.nry + tb - 1) / tb;
      return;
    }
  }
}

// workspace: [acc: C*H*W int64][cnt: H*W int32][slot] (256-byte aligned parts)
long long aggregate_workspace_bytes(const GroupGeom& g) {
  auto a256 = [](long long x) { return (x + 255) & ~255ll; };
  return a256(8ll * g.C * g.H * g.W) + a256(4ll * g.H * g.W) + 256;
}

hipError_t launch_aggregate(const float* groups, const int32_t* idx, float* out, void* ws,
                            const GroupGeom& g, hipStream_t s) {
  auto a256 = [](long long x) { return (x + 255) & ~255ll; };
  char* base = static_cast<char*>(ws);
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(base);
  int* cnt = reinterpret_cast<int*>(base + a256(8ll * g.C * g.H * g.W));
  unsigned* slot = reinterpret_cast<unsigned*>(base + a256(8ll * g.C * g.H * g.W) +
                                               a256(4ll * g.H * g.W));
  const long long n_acc = (long long)g.C * g.H * g.W;
  const long long total = g.n_ref * g.K * (long long)g.C * g.P * g.P;
  (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
  hipLaunchKernelGGL(agg_zero_kernel, dim3(grid_for(n_acc)), dim3(kGroupThreads), 0, s, acc, cnt,
                     slot, n_acc, (long long)g.H * g.W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (total > 0) {
    const int gmax = grid_for(total / 4 + 1) < 2048 ? grid_for(total / 4 + 1) : 2048;
    (void)hipGetLastError();
    if ((reinterpret_cast<uintptr_t>(groups) & 15) == 0)
      hipLaunchKernelGGL(agg_absmax_kernel<true>, dim3(gmax), dim3(kGroupThreads), 0, s, groups,
                         total, slot);
    else
      hipLaunchKernelGGL(agg_absmax_kernel<false>, dim3(gmax), dim3(kGroupThreads), 0, s, groups,
                         total, slot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (g.tb > 0) {
      const long long tiles = (long long)g.ntx * g.nty;
      const int lds = g.th * g.tw * 8;
      (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
      hipLaunchKernelGGL(agg_tile_kernel<kGroupThreads>, dim3((unsigned)tiles, (unsigned)g.C),
                         dim3(kGroupThreads), lds, s, groups, idx, acc, cnt, slot, g);
    } else {
      const int ib = items_per_block(g.C * g.P * g.P);
      const long long blocks = (g.n_ref * g.K + ib - 1) / ib;
      if (blocks >= (1ll << 31)) return hipErrorInvalidValue;
      (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
      hipLaunchKernelGGL(agg_deposit_kernel, dim3((unsigned)blocks), dim3(kGroupThreads), 0, s,
                         groups, idx, acc, cnt, slot, g, ib);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
  hipLaunchKernelGGL(agg_normalise_kernel, dim3((g.W + kNX - 1) / kNX, (g.H + kNY - 1) / kNY),
                     dim3(kGroupThreads), 0, s, acc, cnt, slot, out, g);
  return hipGetLastError();
}

}  // namespace bmk
