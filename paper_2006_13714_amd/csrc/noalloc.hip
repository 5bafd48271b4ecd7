// bm_match without any allocation: the workspace (norm map, centring slot, per-tile max
// map) lives in a fixed device array instead of plan- or caller-owned memory.
//
// `scratch` is a file-scope device array of kScratchBytes.  Host code never passes its
// name to a kernel or a copy (in host code the name is only a stand-in, not a device
// address): the first call on a device, with that device current, looks up the array's
// device address with hipGetSymbolAddress and keeps it per device; every later call uses
// that address.  Each device the library runs on holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bm.h"
#include "plan.h"

namespace bmk {

constexpr int64_t kScratchBytes = BM_NOALLOC_MAX_WORKSPACE;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of this device's copy of `scratch` (looked up once per device).
static bm_status scratch_for(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(BM_ENOTSUP, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BM_OK;
}

}  // namespace bmk

using namespace bmk;

extern "C" {

bm_status bm_match_noalloc(bm_plan_t plan, const float* d_img, int32_t* d_idx, float* d_dist,
                           void* stream) {
  if (!plan) return fail(BM_EINVAL, "plan is NULL");
  if (!d_img || !d_idx || !d_dist) return fail(BM_EINVAL, "NULL device pointer");
  const int64_t need = plan_workspace_bytes(*plan);
  if (need > kScratchBytes)
    return fail(BM_EINVAL, "workspace of %lld bytes exceeds the %lld-byte fixed scratch of "
                           "bm_match_noalloc", (long long)need, (long long)kScratchBytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != plan->device)
    return fail(BM_EINVAL, "plan made on device %d, current is %d", plan->device, dev);
  void* ws = nullptr;
  bm_status st = scratch_for(dev, &ws);
  if (st != BM_OK) return st;
  // every byte of the workspace that the kernels read is written earlier in the same
  // call (norm map, centring constants, max map), so nothing needs clearing
  return run_match(*plan, d_img, d_idx, d_dist, ws, (hipStream_t)stream);
}

}  // extern "C"
