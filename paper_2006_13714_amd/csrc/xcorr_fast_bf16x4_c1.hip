// Specialised cross-term / top-K kernels: precision form bf16x4, 1 channel.
#include "xcorr_fast.h"

namespace bmk {

XcFastKernel fast_kernel_p1_c1(int h2, int kr, int nt) { return fast_h2<1, 1>(h2, kr, nt); }

}  // namespace bmk
