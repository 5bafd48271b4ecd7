// Specialised cross-term / top-K kernels: precision form f16x3, 2 channels.
#include "xcorr_fast.h"

namespace bmk {

XcFastKernel fast_kernel_p2_c2(int h2, int kr, int nt) { return fast_h2<2, 2>(h2, kr, nt); }

}  // namespace bmk
