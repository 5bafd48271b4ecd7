// Persistent uneven-batch kernels: precision form bf16x4, K <= 32, 3 tile columns.
#include "xcorr_batch.h"

namespace bmk {

XcBatchKernel batch_kernel_p1_k2_t3(int tier) { return batch_tier_kernel<1, 2, 3>(tier); }

}  // namespace bmk
