// Statistics pre-pass for centring and the float16 pre-scale.
//
// The squared distance is invariant to subtracting a constant per channel, so the
// library may compute every step on x - c_ch (c_ch: a subsampled per-channel mean) to
// shrink the operands of the cancellation N_i + N_j - 2 C_ij.  The float16 split form also
// needs max |x| to pick a power-of-two pre-scale that keeps its hi/lo parts in range.
//
// Output (float[9] in the workspace): [0] max |x| over the image (as an ordered bit
// pattern; non-negative floats compare like integers), [1 + c] centre of channel c (0 when
// centring is off).  The maximum uses atomicMax (order-independent); the centres are
// summed by one workgroup over a fixed subsample in a fixed order, so both are
// deterministic.
#include <hip/hip_runtime.h>

namespace bmk {

constexpr int kStatsThreads = 256;
constexpr int kCenterSamples = 8192;  // per channel

__global__ void __launch_bounds__(kStatsThreads)
stats_kernel(const float* __restrict__ img, int C, int HW, int do_center,
             float* __restrict__ stats) {
  __shared__ float smax[kStatsThreads];
  __shared__ double ssum[kStatsThreads];
  const int tid = threadIdx.x;
  const long long n = (long long)C * HW;
  float m = 0.f;
  for (long long i = (long long)blockIdx.x * kStatsThreads + tid; i < n;
       i += (long long)gridDim.x * kStatsThreads)
    m = fmaxf(m, fabsf(img[i]));
  smax[tid] = m;
  __syncthreads();
  for (int w = kStatsThreads / 2; w > 0; w >>= 1) {
    if (tid < w) smax[tid] = fmaxf(smax[tid], smax[tid + w]);
    __syncthreads();
  }
  if (tid == 0) atomicMax(reinterpret_cast<unsigned int*>(stats), __float_as_uint(smax[0]));

  if (blockIdx.x != 0) return;
  const int step = HW > kCenterSamples ? HW / kCenterSamples : 1;
  const int ns = (HW + step - 1) / step;
  for (int c = 0; c < C; ++c) {
    double acc = 0.0;
    if (do_center)
      for (int k = tid; k < ns; k += kStatsThreads) acc += (double)img[(long long)c * HW + (long long)k * step];
    ssum[tid] = acc;
    __syncthreads();
    for (int w = kStatsThreads / 2; w > 0; w >>= 1) {
      if (tid < w) ssum[tid] += ssum[tid + w];
      __syncthreads();
    }
    if (tid == 0) stats[1 + c] = do_center ? (float)(ssum[0] / ns) : 0.f;
    __syncthreads();
  }
}

hipError_t launch_stats(const float* img, int C, int H, int W, bool center, float* stats,
                        hipStream_t stream) {
  hipError_t e = hipMemsetAsync(stats, 0, 9 * sizeof(float), stream);
  if (e != hipSuccess) return e;
  const long long n = (long long)C * H * W;
  int blocks = (int)((n + kStatsThreads * 16 - 1) / (kStatsThreads * 16));
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  hipLaunchKernelGGL(stats_kernel, dim3(blocks), dim3(kStatsThreads), 0, stream, img, C, H * W,
                     center ? 1 : 0, stats);
  return hipGetLastError();
}

}  // namespace bmk
