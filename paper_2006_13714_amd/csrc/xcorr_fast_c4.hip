// Specialised cross-term / top-K kernels for 4 channels (see xcorr_fast.h).
#include "xcorr_fast.h"

namespace bmk {

XcKernel fast_kernel_c4(int h2, int kr, int nt) { return fast_h2<4>(h2, kr, nt); }

}  // namespace bmk
