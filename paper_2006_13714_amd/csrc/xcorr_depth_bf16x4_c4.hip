// 3D search kernels (cross-term / top-K over a depth window of slabs): precision form
// bf16x4, 4-plane patches.
#include "xcorr_fast.h"

namespace bmk {

XcDepthKernel depth_kernel_p1_c4(int h2, int kr, int nt) { return depth_h2<1, 4>(h2, kr, nt); }

}  // namespace bmk
