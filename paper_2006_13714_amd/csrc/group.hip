// Group gather and aggregation for gfx950 (Sec. IV, image reconstruction): after block
// matching, the group of reference i is Y_i = [X_{S_i(1)}, ..., X_{S_i(K)}]; a restorer
// processes each group and deposits every patch back at its location, dividing each pixel
// by the number of deposited patches covering it.
//
// Both are HBM-bound element-wise passes.
//  * gather: one thread per group element (reference, k, channel, row, column), coalesced
//    writes; an index that is -1 or does not name a valid patch position gives a zero patch.
//  * aggregate: deposits with 64-bit integer atomics on fixed-point values, so the sums are
//    exact up to one rounding per contribution and independent of the order the atomics
//    land in (bitwise deterministic).  The fixed-point exponent E comes from a device-side
//    max |value| pass: |v| < 2^e, E = 62 - e - ceil(log2(n_ref K + 1)), so no sum of at most
//    n_ref K contributions can overflow.  Coverage counts use 32-bit atomics; a final pass
//    divides in float64 and rounds once to float32.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bm_internal.h"

namespace bmk {

constexpr int kGroupThreads = 256;

__device__ __forceinline__ bool valid_position(long long j, const GroupGeom& g, int* qy, int* qx) {
  if (j < 0) return false;
  const long long y = j / g.W, x = j - (j / g.W) * g.W;
  if (y >= g.Hv || x >= g.Wv) return false;
  *qy = (int)y;
  *qx = (int)x;
  return true;
}

__global__ void __launch_bounds__(kGroupThreads)
gather_kernel(const float* __restrict__ img, const int32_t* __restrict__ idx,
              float* __restrict__ groups, GroupGeom g) {
  const long long per = (long long)g.C * g.P * g.P;
  const long long total = g.n_ref * g.K * per;
  for (long long e = (long long)blockIdx.x * kGroupThreads + threadIdx.x; e < total;
       e += (long long)gridDim.x * kGroupThreads) {
    const long long ik = e / per;
    const int rem = (int)(e - ik * per);
    const int c = rem / (g.P * g.P);
    const int l = (rem / g.P) % g.P;
    const int m = rem % g.P;
    int qy, qx;
    float v = 0.f;
    if (valid_position(idx[ik], g, &qy, &qx)) v = img[((size_t)c * g.H + qy + l) * g.W + qx + m];
    groups[e] = v;
  }
}

// accumulators [C*H*W] int64, counts [H*W] int32, max-|v| slot (uint bits of a float)
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

__global__ void __launch_bounds__(kGroupThreads)
agg_absmax_kernel(const float* __restrict__ groups, long long total, unsigned* __restrict__ slot) {
  __shared__ float red[kGroupThreads / 64];
  float m = 0.f;
  for (long long e = (long long)blockIdx.x * kGroupThreads + threadIdx.x; e < total;
       e += (long long)gridDim.x * kGroupThreads)
    m = fmaxf(m, fabsf(groups[e]));
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

__global__ void __launch_bounds__(kGroupThreads)
agg_deposit_kernel(const float* __restrict__ groups, const int32_t* __restrict__ idx,
                   unsigned long long* __restrict__ acc, int* __restrict__ cnt,
                   const unsigned* __restrict__ slot, GroupGeom g) {
  const int E = fixed_exponent(*slot, g.cnt_bits);
  const long long per = (long long)g.C * g.P * g.P;
  const long long total = g.n_ref * g.K * per;
  for (long long e = (long long)blockIdx.x * kGroupThreads + threadIdx.x; e < total;
       e += (long long)gridDim.x * kGroupThreads) {
    const long long ik = e / per;
    int qy, qx;
    if (!valid_position(idx[ik], g, &qy, &qx)) continue;
    const int rem = (int)(e - ik * per);
    const int c = rem / (g.P * g.P);
    const int l = (rem / g.P) % g.P;
    const int m = rem % g.P;
    const long long q = llrint(ldexp((double)groups[e], E));
    const size_t pix = (size_t)(qy + l) * g.W + qx + m;
    atomicAdd(&acc[(size_t)c * g.H * g.W + pix], (unsigned long long)q);
    if (c == 0) atomicAdd(&cnt[pix], 1);
  }
}

__global__ void __launch_bounds__(kGroupThreads)
agg_normalise_kernel(const unsigned long long* __restrict__ acc, const int* __restrict__ cnt,
                     const unsigned* __restrict__ slot, float* __restrict__ out, GroupGeom g) {
  const int E = fixed_exponent(*slot, g.cnt_bits);
  const long long hw = (long long)g.H * g.W;
  const long long total = (long long)g.C * hw;
  for (long long e = (long long)blockIdx.x * kGroupThreads + threadIdx.x; e < total;
       e += (long long)gridDim.x * kGroupThreads) {
    const int n = cnt[e % hw];
    const double v = ldexp((double)(long long)acc[e], -E);
    out[e] = n > 0 ? (float)(v / n) : 0.f;
  }
}

static int grid_for(long long total) {
  long long b = (total + kGroupThreads - 1) / kGroupThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

hipError_t launch_gather(const float* img, const int32_t* idx, float* groups, const GroupGeom& g,
                         hipStream_t s) {
  const long long total = g.n_ref * g.K * (long long)g.C * g.P * g.P;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(grid_for(total)), dim3(kGroupThreads), 0, s, img, idx,
                     groups, g);
  return hipGetLastError();
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
  hipLaunchKernelGGL(agg_zero_kernel, dim3(grid_for(n_acc)), dim3(kGroupThreads), 0, s, acc, cnt,
                     slot, n_acc, (long long)g.H * g.W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (total > 0) {
    hipLaunchKernelGGL(agg_absmax_kernel, dim3(grid_for(total) < 4096 ? grid_for(total) : 4096),
                       dim3(kGroupThreads), 0, s, groups, total, slot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(agg_deposit_kernel, dim3(grid_for(total)), dim3(kGroupThreads), 0, s,
                       groups, idx, acc, cnt, slot, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(agg_normalise_kernel, dim3(grid_for(n_acc)), dim3(kGroupThreads), 0, s, acc,
                     cnt, slot, out, g);
  return hipGetLastError();
}

}  // namespace bmk
