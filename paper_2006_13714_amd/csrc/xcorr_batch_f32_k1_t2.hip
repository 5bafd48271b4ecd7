// Persistent uneven-batch kernels: precision form f32, K <= 16, 2 tile columns.
#include "xcorr_batch.h"

namespace bmk {

XcBatchKernel batch_kernel_p0_k1_t2(int tier) { return batch_tier_kernel<0, 1, 2>(tier); }

}  // namespace bmk
