// Specialised cross-term / top-K kernels for 1 channel (see xcorr_fast.h).
#include "xcorr_fast.h"

namespace bmk {

XcKernel fast_kernel_c1(int h2, int kr, int nt) { return fast_h2<1>(h2, kr, nt); }

}  // namespace bmk
