// Non-local means kernels (nlm.h): float32 contraction, C 1..4, patch 3..8, 2..3 tile columns.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "nlm.h"

namespace bmk {

static NlmKernel nlm_kernel(int c, int h2, int nt) {
  switch (c) {
    case 1: return nlm_h2<1>(h2, nt);
    case 2: return nlm_h2<2>(h2, nt);
    case 3: return nlm_h2<3>(h2, nt);
    case 4: return nlm_h2<4>(h2, nt);
  }
  return nullptr;
}

// LDS of one NLM workgroup: the float32 strip and norm strip as in the BM kernel, one 16 x 16
// weight tile per wave, and (reusing the same bytes after the sweep) the per-wave patch sums
// and Theta of the 16 references.
int nlm_lds_bytes(const XcGeom& g) {
  const int npb = g.C * (g.Pe / 2);
  const int a = g.lds_buf_off + g.WS * 16 * 16 * 4;
  const int red = g.WS * 16 * npb * 16 * 4 + g.WS * 16 * 4;
  return a > red ? a : red;
}

hipError_t launch_nlm(const float* img, const float* nrm, float* patch, float* theta,
                      const XcGeom& g, float b, hipStream_t stream) {
  NlmKernel k = nlm_kernel(g.C, g.Pe / 2, g.NT);
  if (!k || g.WS < 1 || g.WS > 4) return hipErrorInvalidValue;
  const int lds = nlm_lds_bytes(g);
  {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> set;  // per (kernel, device)
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    int& cur = set[std::make_pair(reinterpret_cast<const void*>(k), dev)];
    if (lds > cur) {
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
      if (e != hipSuccess) return e;
      cur = lds;
    }
  }
  const float kexp = -1.4426950408889634f / (b * b);  // exp(-d / b^2) = exp2(d * kexp)
  (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
  hipLaunchKernelGGL(k, dim3(g.nwg_total), dim3(64 * g.WS), lds, stream, img, nrm, patch, theta,
                     fast_geom(g), kexp);
  return hipGetLastError();
}

}  // namespace bmk
