// Dispatch for the specialised cross-term / top-K kernels (xcorr_fast.h).
#include <hip/hip_runtime.h>

#include "bm_internal.h"

namespace bmk {

typedef void (*XcKernel)(const float*, const float*, int*, float*, const XcGeom);
XcKernel fast_kernel_c1(int h2, int kr, int nt);
XcKernel fast_kernel_c2(int h2, int kr, int nt);
XcKernel fast_kernel_c3(int h2, int kr, int nt);
XcKernel fast_kernel_c4(int h2, int kr, int nt);

static XcKernel fast_kernel(int c, int h2, int kr, int nt) {
  switch (c) {
    case 1: return fast_kernel_c1(h2, kr, nt);
    case 2: return fast_kernel_c2(h2, kr, nt);
    case 3: return fast_kernel_c3(h2, kr, nt);
    case 4: return fast_kernel_c4(h2, kr, nt);
  }
  return nullptr;
}

hipError_t prepare_xcorr_fast(int c, int h2, int kr, int nt, int lds_bytes) {
  XcKernel k = fast_kernel(c, h2, kr, nt);
  if (!k) return hipErrorInvalidValue;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

hipError_t launch_xcorr_fast(int c, int h2, int kr, int nt, const float* img, const float* nrm,
                             int* idx, float* dist, const XcGeom& g, hipStream_t stream) {
  XcKernel k = fast_kernel(c, h2, kr, nt);
  if (!k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(g.nwg_total), dim3(64 * g.WS), g.lds_bytes, stream, img, nrm, idx,
                     dist, g);
  return hipGetLastError();
}

}  // namespace bmk
