// Persistent uneven-batch kernels: precision form f16x3, K <= 16, 2 tile columns.
#include "xcorr_batch.h"

namespace bmk {

XcBatchKernel batch_kernel_p2_k1_t2(int tier) { return batch_tier_kernel<2, 1, 2>(tier); }

}  // namespace bmk
