// Persistent uneven-batch kernels: precision form f16x3, K <= 32, 3 tile columns.
#include "xcorr_batch.h"

namespace bmk {

XcBatchKernel batch_kernel_p2_k2_t3(int tier) { return batch_tier_kernel<2, 2, 3>(tier); }

}  // namespace bmk
