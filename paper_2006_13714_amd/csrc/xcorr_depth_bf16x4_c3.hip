// 3D search kernels (cross-term / top-K over a depth window of slabs): precision form
// bf16x4, 3-plane patches.
#include "xcorr_fast.h"

namespace bmk {

XcDepthKernel depth_kernel_p1_c3(int h2, int kr, int nt) { return depth_h2<1, 3>(h2, kr, nt); }

}  // namespace bmk
