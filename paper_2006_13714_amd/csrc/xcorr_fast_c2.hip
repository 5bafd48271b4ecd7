// Specialised cross-term / top-K kernels for 2 channels (see xcorr_fast.h).
#include "xcorr_fast.h"

namespace bmk {

XcKernel fast_kernel_c2(int h2, int kr, int nt) { return fast_h2<2>(h2, kr, nt); }

}  // namespace bmk
