// Serving entry points (filled in by their own source).
#include "plan.h"

using namespace bmk;

extern "C" {

bm_status bm_server_create(const bm_server_cfg*, bm_server_t*) {
  return fail(BM_ENOTSUP, "server not built");
}
bm_status bm_submit(bm_server_t, const bm_desc*, const float*, uint64_t*) {
  return fail(BM_ENOTSUP, "server not built");
}
bm_status bm_poll(bm_server_t, uint64_t, int32_t*, float*, bm_request_stats*) {
  return fail(BM_ENOTSUP, "server not built");
}
bm_status bm_cancel(bm_server_t, uint64_t) { return fail(BM_ENOTSUP, "server not built"); }
bm_status bm_server_destroy(bm_server_t) { return fail(BM_ENOTSUP, "server not built"); }

}  // extern "C"
