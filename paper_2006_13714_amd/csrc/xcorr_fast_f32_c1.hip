// Specialised cross-term / top-K kernels: precision form f32, 1 channel.
#include "xcorr_fast.h"

namespace bmk {

XcFastKernel fast_kernel_p0_c1(int h2, int kr, int nt) { return fast_h2<0, 1>(h2, kr, nt); }

}  // namespace bmk
