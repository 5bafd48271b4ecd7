// Specialised cross-term / top-K kernels: precision form bf16x4, 3 channels.
#include "xcorr_fast.h"

namespace bmk {

XcFastKernel fast_kernel_p1_c3(int h2, int kr, int nt) { return fast_h2<1, 3>(h2, kr, nt); }

}  // namespace bmk
