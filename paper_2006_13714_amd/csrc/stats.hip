// Centring pre-pass (optional, BM_FLAG_CENTER).
//
// The squared distance is invariant to subtracting a constant per channel, so the library
// may compute every step on x - c_ch to shrink the operands of the cancellation
// N_i + N_j - 2 C_ij (Lemma 2, Sec. III-B).  c_ch is the mean of a fixed subsample of
// channel ch (every step-th element, at most kCenterSamples), summed by one workgroup in a
// fixed order in float64, so it is deterministic.
//
// Output: centers[c], c < C (float[8] slot in the workspace).
#include <hip/hip_runtime.h>

namespace bmk {

constexpr int kStatsThreads = 256;
constexpr int kCenterSamples = 8192;  // per channel

__device__ __forceinline__ void channel_means(const float* __restrict__ img, int C, int HW,
                                              float* __restrict__ centers, double* ssum) {
  const int tid = threadIdx.x;
  const int step = HW > kCenterSamples ? HW / kCenterSamples : 1;
  const int ns = (HW + step - 1) / step;
  for (int c = 0; c < C; ++c) {
    double acc = 0.0;
    for (int k = tid; k < ns; k += kStatsThreads)
      acc += (double)img[(long long)c * HW + (long long)k * step];
    ssum[tid] = acc;
    __syncthreads();
    for (int w = kStatsThreads / 2; w > 0; w >>= 1) {
      if (tid < w) ssum[tid] += ssum[tid + w];
      __syncthreads();
    }
    if (tid == 0) centers[c] = (float)(ssum[0] / ns);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kStatsThreads)
center_kernel(const float* __restrict__ img, int C, int HW, float* __restrict__ centers) {
  __shared__ double ssum[kStatsThreads];
  channel_means(img, C, HW, centers, ssum);
}

hipError_t launch_centers(const float* img, int C, int H, int W, float* centers,
                          hipStream_t stream) {
  (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
  hipLaunchKernelGGL(center_kernel, dim3(1), dim3(kStatsThreads), 0, stream, img, C, H * W,
                     centers);
  return hipGetLastError();
}

}  // namespace bmk
