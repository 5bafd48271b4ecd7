// Specialised cross-term / top-K kernels: precision form bf16x4, 2 channels.
#include "xcorr_fast.h"

namespace bmk {

XcFastKernel fast_kernel_p1_c2(int h2, int kr, int nt) { return fast_h2<1, 2>(h2, kr, nt); }

}  // namespace bmk
