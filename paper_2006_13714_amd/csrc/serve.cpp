// Serving entry points: the scheduler core (serve_core.h) driven by a HIP executor.
//
// Device memory: one arena of hbm_budget_bytes, allocated when the server starts and
// sub-allocated per request (image, norm map, centring slot, outputs) and per step (batch
// header), so admission never calls the device allocator.  Host memory: one pinned arena
// holding each queued request's image, into which its results are copied back.
// A step copies its requests' images in on the input stream, runs the uneven-batch launch
// (one norm launch and the persistent cross-term launches) on one of two compute streams
// taken in turn, and copies the results out on the output stream, the three joined by
// events.  Copies of one step therefore overlap the kernels of its neighbours, and the
// kernels of consecutive steps overlap each other's tails.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <new>
#include <string>

#include "batch_run.h"
#include "plan.h"
#include "serve_core.h"

namespace bmk {

namespace {

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// request memory: [image][plan workspace layout: norm map, auxiliary slots][idx][dist]
struct DevLayout {
  int64_t img, nrm, aux, idx, dist, total;
};

DevLayout dev_layout(const bm_desc& d) {
  DevLayout L;
  const int64_t hv = d.height - d.patch + 1, wv = d.width - d.patch + 1;
  const int64_t out = desc_n_ref(d) * d.k * 4;
  L.img = 0;
  L.nrm = L.img + align256((int64_t)d.channels * d.height * d.width * 4);
  L.aux = L.nrm + align256(hv * wv * 4);
  L.idx = L.nrm + desc_workspace_bytes(d);
  L.dist = L.idx + align256(out);
  L.total = L.dist + align256(out);
  return L;
}

struct StepState {
  hipEvent_t in = nullptr, comp = nullptr, done = nullptr;
  bool recorded = false;
  bm_status status = BM_OK;
  ~StepState() {
    for (hipEvent_t e : {in, comp, done})
      if (e) (void)hipEventDestroy(e);
  }
};

class HipExecutor : public Executor {
 public:
  ~HipExecutor() override {
    for (hipStream_t s : {in_, comp_[0], comp_[1], out_})
      if (s) (void)hipStreamDestroy(s);
    if (dev_) (void)hipFree(dev_);
    if (host_) (void)hipHostFree(host_);
  }

  bm_status init(int device, int64_t dev_bytes, int64_t host_bytes) {
    device_ = device;
    hipError_t e = hipDeviceGetAttribute(&max_lds_, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    if ((e = hipMalloc(&dev_, dev_bytes)) != hipSuccess) {
      (void)hipGetLastError();
      dev_ = nullptr;
      return fail(BM_ENOMEM, "server device arena hipMalloc(%lld)", (long long)dev_bytes);
    }
    if ((e = hipHostMalloc(&host_, host_bytes, hipHostMallocDefault)) != hipSuccess) {
      (void)hipGetLastError();
      host_ = nullptr;
      return fail(BM_ENOMEM, "server host arena hipHostMalloc(%lld)", (long long)host_bytes);
    }
    for (hipStream_t* s : {&in_, &comp_[0], &comp_[1], &out_})
      if ((e = hipStreamCreateWithFlags(s, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreateWithFlags");
    return BM_OK;
  }

  bm_status thread_init() override {
    hipError_t e = hipSetDevice(device_);
    return e == hipSuccess ? BM_OK : hip_fail(e, "hipSetDevice");
  }

  int64_t request_bytes(const bm_desc& d) override { return dev_layout(d).total; }
  int64_t step_header_bytes(int n) override { return batch_header_bytes(n); }
  void* host_base() override { return host_; }

  bm_status prepare(Request* r) override {
    auto p = std::make_shared<bm_plan_s>();
    p->desc = r->desc;
    p->device = device_;
    bm_status st = choose_config(r->desc, max_lds_, p.get());
    if (st != BM_OK) return st;
    r->exec = p;
    return BM_OK;
  }

  bm_status begin_step(Step* s) override {
    auto ss = std::make_shared<StepState>();
    s->exec = ss;
    hipError_t e;
    for (hipEvent_t* ev : {&ss->in, &ss->comp, &ss->done})
      if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess) {
        *ev = nullptr;
        return hip_fail(e, "hipEventCreate");
      }
    hipStream_t comp = comp_[next_++ % 2];
    char* dbase = static_cast<char*>(dev_);
    char* hbase = static_cast<char*>(host_);
    std::vector<BatchEntry> ent(s->reqs.size());
    for (size_t i = 0; i < s->reqs.size(); ++i) {
      Request* r = s->reqs[i];
      const DevLayout L = dev_layout(r->desc);
      char* d = dbase + r->dev_off;
      e = hipMemcpyAsync(d + L.img, hbase + r->host_off, r->img_bytes, hipMemcpyHostToDevice, in_);
      if (e != hipSuccess) return hip_fail(e, "request image copy");
      const bm_plan_s* plan = static_cast<const bm_plan_s*>(r->exec.get());
      ent[i] = BatchEntry{plan, reinterpret_cast<const float*>(d + L.img),
                          reinterpret_cast<float*>(d + L.nrm), aux_at(*plan, d + L.aux),
                          reinterpret_cast<int32_t*>(d + L.idx), reinterpret_cast<float*>(d + L.dist)};
    }
    if ((e = hipEventRecord(ss->in, in_)) != hipSuccess ||
        (e = hipStreamWaitEvent(comp, ss->in, 0)) != hipSuccess)
      return hip_fail(e, "input event");
    bm_status st = run_batch(ent.data(), (int)ent.size(), dbase + s->hdr_off, comp);
    if (st != BM_OK) return st;
    if ((e = hipEventRecord(ss->comp, comp)) != hipSuccess ||
        (e = hipStreamWaitEvent(out_, ss->comp, 0)) != hipSuccess)
      return hip_fail(e, "compute event");
    for (size_t i = 0; i < s->reqs.size(); ++i) {
      Request* r = s->reqs[i];
      const DevLayout L = dev_layout(r->desc);
      const int64_t n = r->n_ref * r->desc.k * 4;
      char* d = dbase + r->dev_off;
      char* h = hbase + r->host_off;
      if ((e = hipMemcpyAsync(h, d + L.idx, n, hipMemcpyDeviceToHost, out_)) != hipSuccess ||
          (e = hipMemcpyAsync(h + n, d + L.dist, n, hipMemcpyDeviceToHost, out_)) != hipSuccess)
        return hip_fail(e, "result copy");
    }
    if ((e = hipEventRecord(ss->done, out_)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    ss->recorded = true;
    return BM_OK;
  }

  bool step_done(Step* s) override {
    auto* ss = static_cast<StepState*>(s->exec.get());
    if (!ss->recorded) return true;
    const hipError_t q = hipEventQuery(ss->done);
    if (q == hipErrorNotReady) return false;
    if (q != hipSuccess) ss->status = hip_fail(q, "step completion");
    return true;
  }

  void wait_step(Step* s) override {
    auto* ss = static_cast<StepState*>(s->exec.get());
    if (ss && ss->recorded) {
      (void)hipEventSynchronize(ss->done);
      return;
    }
    // a step that failed while being enqueued: wait for whatever it did enqueue
    for (hipStream_t st : {in_, comp_[0], comp_[1], out_}) (void)hipStreamSynchronize(st);
  }

  std::string last_message() override { return last_error(); }

  bm_status step_status(Step* s) override {
    auto* ss = static_cast<StepState*>(s->exec.get());
    return ss ? ss->status : BM_OK;
  }

 private:
  int device_ = 0, max_lds_ = 0;
  void* dev_ = nullptr;
  void* host_ = nullptr;
  hipStream_t in_ = nullptr, out_ = nullptr;
  hipStream_t comp_[2] = {nullptr, nullptr};
  unsigned next_ = 0;
};

}  // namespace
}  // namespace bmk

struct bm_server_s {
  std::unique_ptr<bmk::HipExecutor> ex;
  std::unique_ptr<bmk::Scheduler> sch;
};

using namespace bmk;

extern "C" {

bm_status bm_server_create(const bm_server_cfg* cfg, bm_server_t* out) {
  if (!cfg || !out) return fail(BM_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->hbm_budget_bytes < (1 << 20) || cfg->max_inflight < 1 || cfg->max_queue < 1 ||
      cfg->max_step < 0 || cfg->max_step > 64)
    return fail(BM_EINVAL, "server configuration out of range");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::unique_ptr<bm_server_s> s(new (std::nothrow) bm_server_s);
  if (!s) return fail(BM_ENOMEM, "host allocation failed");
  s->ex.reset(new HipExecutor);
  // host staging: room for the queue's images (at least 256 MiB, at most 8 GiB)
  const int64_t host_bytes =
      std::min<int64_t>(std::max<int64_t>(cfg->hbm_budget_bytes, 256ll << 20), 8ll << 30);
  bm_status st = s->ex->init(dev, cfg->hbm_budget_bytes, host_bytes);
  if (st != BM_OK) return st;
  s->sch.reset(new Scheduler(s->ex.get(), *cfg, cfg->hbm_budget_bytes, host_bytes));
  st = s->sch->start();
  if (st != BM_OK) return st;
  *out = s.release();
  return BM_OK;
}

bm_status bm_submit(bm_server_t srv, const bm_desc* desc, const float* host_img, uint64_t* ticket) {
  if (!srv || !desc || !host_img || !ticket) return fail(BM_EINVAL, "NULL argument");
  bm_status st = validate_desc(desc);
  if (st != BM_OK) return st;
  if (desc->window_depth > 0) return fail(BM_ENOTSUP, "the server takes 2D requests");
  if (desc->precision != BM_PREC_FP32 && !fast_eligible(*desc))
    return fail(BM_ENOTSUP, "split precision needs C <= 4, patch 5..8, K <= 32 and "
                            "17 <= 3*stride + window <= 48");
  const char* why = "";
  st = srv->sch->submit(*desc, host_img, ticket, &why);
  if (st != BM_OK) return fail(st, "%s", why);
  return BM_OK;
}

bm_status bm_poll(bm_server_t srv, uint64_t ticket, int32_t* host_idx, float* host_dist,
                  bm_request_stats* stats) {
  if (!srv) return fail(BM_EINVAL, "NULL server");
  std::string why;
  bm_status st = srv->sch->poll(ticket, host_idx, host_dist, stats, &why);
  if (st == BM_ENOTFOUND) return fail(st, "unknown or retired ticket %llu", (unsigned long long)ticket);
  if (st != BM_OK && st != BM_EAGAIN)
    return fail(st, "request %llu did not complete%s%s", (unsigned long long)ticket,
                why.empty() ? "" : ": ", why.c_str());
  return st;
}

bm_status bm_cancel(bm_server_t srv, uint64_t ticket) {
  if (!srv) return fail(BM_EINVAL, "NULL server");
  bm_status st = srv->sch->cancel(ticket);
  if (st != BM_OK) return fail(st, "unknown or retired ticket %llu", (unsigned long long)ticket);
  return BM_OK;
}

bm_status bm_server_destroy(bm_server_t srv) {
  if (!srv) return fail(BM_EINVAL, "NULL server");
  srv->sch->shutdown();
  srv->sch.reset();
  srv->ex.reset();
  delete srv;
  return BM_OK;
}

}  // extern "C"
