// Persistent uneven-batch kernels: precision form f32, K <= 32, 3 tile columns.
#include "xcorr_batch.h"

namespace bmk {

XcBatchKernel batch_kernel_p0_k2_t3(int tier) { return batch_tier_kernel<0, 2, 3>(tier); }

}  // namespace bmk
