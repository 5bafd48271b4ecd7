// Dispatch for the specialised cross-term / top-K kernels (xcorr_fast.h).
#include <hip/hip_runtime.h>

#include "bm_internal.h"

namespace bmk {

typedef void (*XcFastKernel)(const float*, const float*, const float*, const float*, int*,
                             float*, const FastGeom);
typedef void (*XcDepthKernel)(const float*, const float*, const float*, int*, float*,
                              const FastGeom, const DepthGeom);
#define BMK_DECL(P)                                            \
  XcFastKernel fast_kernel_p##P##_c1(int h2, int kr, int nt);    \
  XcFastKernel fast_kernel_p##P##_c2(int h2, int kr, int nt);    \
  XcFastKernel fast_kernel_p##P##_c3(int h2, int kr, int nt);    \
  XcFastKernel fast_kernel_p##P##_c4(int h2, int kr, int nt);    \
  XcDepthKernel depth_kernel_p##P##_c1(int h2, int kr, int nt);  \
  XcDepthKernel depth_kernel_p##P##_c2(int h2, int kr, int nt);  \
  XcDepthKernel depth_kernel_p##P##_c3(int h2, int kr, int nt);  \
  XcDepthKernel depth_kernel_p##P##_c4(int h2, int kr, int nt);
BMK_DECL(0)
BMK_DECL(1)
BMK_DECL(2)
#undef BMK_DECL

static XcFastKernel fast_kernel(int prec, int c, int h2, int kr, int nt) {
  typedef XcFastKernel (*Pick)(int, int, int);
  static const Pick table[3][4] = {
      {fast_kernel_p0_c1, fast_kernel_p0_c2, fast_kernel_p0_c3, fast_kernel_p0_c4},
      {fast_kernel_p1_c1, fast_kernel_p1_c2, fast_kernel_p1_c3, fast_kernel_p1_c4},
      {fast_kernel_p2_c1, fast_kernel_p2_c2, fast_kernel_p2_c3, fast_kernel_p2_c4}};
  if (prec < 0 || prec > 2 || c < 1 || c > 4) return nullptr;
  return table[prec][c - 1](h2, kr, nt);
}

hipError_t prepare_xcorr_fast(int prec, int c, int h2, int kr, int nt, int lds_bytes) {
  XcFastKernel k = fast_kernel(prec, c, h2, kr, nt);
  if (!k) return hipErrorInvalidValue;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

hipError_t launch_xcorr_fast(int prec, int c, int h2, int kr, int nt, const float* img,
                             const float* nrm, const float* centers, const float* amax,
                             int* idx, float* dist, const XcGeom& g, hipStream_t stream) {
  XcFastKernel k = fast_kernel(prec, c, h2, kr, nt);
  if (!k) return hipErrorInvalidValue;
  (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
  hipLaunchKernelGGL(k, dim3(g.nwg_total), dim3(64 * g.WS), g.lds_bytes, stream, img, nrm,
                     centers, amax, idx, dist, fast_geom(g));
  return hipGetLastError();
}

// 3D search kernels (one workgroup per reference depth and 4 x 4 reference block)
static XcDepthKernel depth_kernel(int prec, int c, int h2, int kr, int nt) {
  typedef XcDepthKernel (*Pick)(int, int, int);
  static const Pick table[3][4] = {
      {depth_kernel_p0_c1, depth_kernel_p0_c2, depth_kernel_p0_c3, depth_kernel_p0_c4},
      {depth_kernel_p1_c1, depth_kernel_p1_c2, depth_kernel_p1_c3, depth_kernel_p1_c4},
      {depth_kernel_p2_c1, depth_kernel_p2_c2, depth_kernel_p2_c3, depth_kernel_p2_c4}};
  if (prec < 0 || prec > 2 || c < 1 || c > 4) return nullptr;
  return table[prec][c - 1](h2, kr, nt);
}

hipError_t prepare_xcorr_depth(int prec, int c, int h2, int kr, int nt, int lds_bytes) {
  XcDepthKernel k = depth_kernel(prec, c, h2, kr, nt);
  if (!k) return hipErrorInvalidValue;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

hipError_t launch_xcorr_depth(int prec, int c, int h2, int kr, int nt, const float* vol,
                              const float* nrm, const float* amax, int* idx, float* dist,
                              const XcGeom& g, const DepthGeom& dg, hipStream_t stream) {
  XcDepthKernel k = depth_kernel(prec, c, h2, kr, nt);
  if (!k) return hipErrorInvalidValue;
  const long long blocks = (long long)g.nwg_total * dg.Z;
  if (blocks < 1 || blocks >= (1ll << 31)) return hipErrorInvalidValue;
  (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * g.WS), g.lds_bytes, stream, vol, nrm,
                     amax, idx, dist, fast_geom(g), dg);
  return hipGetLastError();
}

}  // namespace bmk
