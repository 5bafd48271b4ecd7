// Persistent uneven-batch kernels: precision form bf16x4, K <= 16, 2 tile columns.
#include "xcorr_batch.h"

namespace bmk {

XcBatchKernel batch_kernel_p1_k1_t2(int tier) { return batch_tier_kernel<1, 1, 2>(tier); }

}  // namespace bmk
