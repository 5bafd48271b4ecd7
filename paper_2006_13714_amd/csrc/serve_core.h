// Serving scheduler core: request queue, admission by device-memory footprint, continuous
// batching of admitted requests into launch steps, completion, poll and cancel.
//
// Device work goes through an Executor (serve.cpp: HIP streams, the uneven-batch launch and
// the result copies), so this file has no HIP dependency and its logic can be exercised on
// the host with a stand-in executor.
//
// One scheduler thread repeats:
//   1. retire finished steps: their requests become Done (results in host memory) and
//      their device memory returns to the budget;
//   2. admit queued requests in arrival order while their footprint fits in the device
//      arena and fewer than max_inflight are admitted;
//   3. launch the newly admitted requests as one step (copies in, one batch launch,
//      copies out), without waiting for earlier steps: steps overlap on the device.
// A step takes at most kMaxStep requests (and at most half of max_inflight), so that
// under load several steps are in flight: slots freed by one step are refilled while the
// others still run, and one step's copies overlap another's kernels.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/bm.h"

namespace bmk {

// First-fit sub-allocator of the byte range [0, size) in `align`-byte units; neighbouring
// free ranges are merged on release.
class RangeAlloc {
 public:
  explicit RangeAlloc(int64_t size = 0, int64_t align = 256) { reset(size, align); }
  void reset(int64_t size, int64_t align = 256) {
    align_ = align;
    size_ = size / align * align;
    free_.clear();
    used_.clear();
    in_use_ = 0;
    if (size_ > 0) free_[0] = size_;
  }
  bool alloc(int64_t bytes, int64_t* off) {
    const int64_t need = std::max<int64_t>(align_, (bytes + align_ - 1) / align_ * align_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const int64_t o = it->first, len = it->second;
      free_.erase(it);
      if (len > need) free_[o + need] = len - need;
      used_[o] = need;
      in_use_ += need;
      *off = o;
      return true;
    }
    return false;
  }
  void release(int64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    int64_t o = off, len = u->second;
    used_.erase(u);
    in_use_ -= len;
    auto nx = free_.lower_bound(o);
    if (nx != free_.end() && nx->first == o + len) {
      len += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == o) {
        o = pv->first;
        len += pv->second;
        free_.erase(pv);
      }
    }
    free_[o] = len;
  }
  int64_t used() const { return in_use_; }
  int64_t size() const { return size_; }
  int64_t largest_free() const {
    int64_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<int64_t, int64_t> free_, used_;
  int64_t size_ = 0, align_ = 256, in_use_ = 0;
};

enum class ReqState { Queued, Admitted, Done, Failed, Cancelled };

struct Request {
  uint64_t ticket = 0;
  bm_desc desc{};
  int64_t n_ref = 0;
  int64_t img_bytes = 0, out_bytes = 0;  // host: image in, idx + dist out
  int64_t dev_bytes = 0;                 // device footprint (image, norms, outputs)
  int64_t host_off = -1, dev_off = -1;
  ReqState state = ReqState::Queued;
  bool cancel_requested = false;
  bm_status status = BM_OK;
  std::string message;         // why it failed (the executor's message at the time)
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::shared_ptr<void> exec;  // executor's per-request state (plan)
};

struct Step {
  std::vector<Request*> reqs;
  int64_t hdr_off = -1;
  std::shared_ptr<void> exec;  // executor's per-step state (stream, event)
};

class Executor {
 public:
  virtual ~Executor() {}
  virtual bm_status thread_init() { return BM_OK; }      // on the scheduler thread
  virtual int64_t request_bytes(const bm_desc& d) = 0;     // device bytes of one request
  virtual int64_t step_header_bytes(int n) = 0;            // device bytes of a step's header
  virtual void* host_base() = 0;                           // host arena
  virtual bm_status prepare(Request* r) = 0;               // per-request plan (on admission)
  virtual bm_status begin_step(Step* s) = 0;                // enqueue copies and launches
  virtual bool step_done(Step* s) = 0;                      // non-blocking completion test
  virtual void wait_step(Step* s) = 0;                      // blocking
  virtual bm_status step_status(Step*) { return BM_OK; }    // after completion
  virtual std::string last_message() { return ""; }         // text of the last failure
};

inline double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

inline int64_t desc_n_ref(const bm_desc& d) {
  return (int64_t)((d.height - d.patch) / d.stride + 1) * ((d.width - d.patch) / d.stride + 1);
}

class Scheduler {
 public:
  static constexpr int64_t kMaxStep = 8;

  Scheduler(Executor* ex, const bm_server_cfg& cfg, int64_t dev_arena, int64_t host_arena)
      : ex_(ex), cfg_(cfg) {
    dev_.reset(dev_arena);
    host_.reset(host_arena);
  }
  ~Scheduler() { shutdown(); }

  bm_status start() {
    std::unique_lock<std::mutex> lk(mu_);
    thread_ = std::thread([this] { loop(); });
    cv_.wait(lk, [this] { return started_; });
    return init_status_;
  }

  // Validation of the descriptor is the caller's; this checks capacity and queues.  The
  // image is copied into the reserved host block outside the lock.
  bm_status submit(const bm_desc& d, const float* img, uint64_t* ticket, const char** why) {
    auto r = std::make_unique<Request>();
    r->desc = d;
    r->n_ref = desc_n_ref(d);
    r->img_bytes = (int64_t)d.channels * d.height * d.width * 4;
    r->out_bytes = r->n_ref * d.k * 8;
    r->dev_bytes = ex_->request_bytes(d);
    {
      std::unique_lock<std::mutex> lk(mu_);
      if (stop_) return *why = "server is shutting down", BM_EINVAL;
      if (r->dev_bytes + ex_->step_header_bytes(1) > dev_.size())
        return *why = "request alone exceeds the device budget", BM_EBUSY;
      if ((int64_t)(queue_.size() + copying_) >= cfg_.max_queue) return *why = "queue full", BM_EBUSY;
      if (!host_.alloc(std::max(r->img_bytes, r->out_bytes), &r->host_off))
        return *why = "host staging memory full", BM_EBUSY;
      ++copying_;
    }
    std::memcpy(static_cast<char*>(ex_->host_base()) + r->host_off, img, r->img_bytes);
    std::unique_lock<std::mutex> lk(mu_);
    --copying_;
    r->ticket = next_ticket_++;
    r->t_submit = now_s();
    *ticket = r->ticket;
    queue_.push_back(r.get());
    reqs_[r->ticket] = std::move(r);
    cv_.notify_all();
    return BM_OK;
  }

  // A finished request is retired under the lock and its results copied outside it.
  bm_status poll(uint64_t t, int32_t* idx, float* dist, bm_request_stats* st,
                 std::string* message = nullptr) {
    std::unique_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(mu_);
      auto it = reqs_.find(t);
      if (it == reqs_.end()) return BM_ENOTFOUND;
      if (it->second->state == ReqState::Queued || it->second->state == ReqState::Admitted)
        return BM_EAGAIN;
      r = std::move(it->second);
      reqs_.erase(it);
    }
    bm_status s = BM_OK;
    if (r->state == ReqState::Done) {
      const char* base = static_cast<const char*>(ex_->host_base()) + r->host_off;
      const int64_t n = r->n_ref * r->desc.k;
      if (idx) std::memcpy(idx, base, n * 4);
      if (dist) std::memcpy(dist, base + n * 4, n * 4);
      if (st) {
        st->queue_s = r->t_admit - r->t_submit;
        st->device_s = r->t_done - r->t_admit;
        st->total_s = r->t_done - r->t_submit;
        st->n_ref = r->n_ref;
      }
    } else {
      s = r->state == ReqState::Cancelled ? BM_ECANCELED : r->status;
      if (message) *message = r->message;
    }
    if (r->host_off >= 0) {
      std::unique_lock<std::mutex> lk(mu_);
      host_.release(r->host_off);
    }
    return s;
  }

  bm_status cancel(uint64_t t) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(t);
    if (it == reqs_.end()) return BM_ENOTFOUND;
    Request* r = it->second.get();
    if (r->state == ReqState::Queued) {
      queue_.erase(std::find(queue_.begin(), queue_.end(), r));
      r->state = ReqState::Cancelled;
      host_.release(r->host_off);
      r->host_off = -1;
    } else if (r->state == ReqState::Admitted) {
      r->cancel_requested = true;  // the step finishes; its results are dropped
    }
    return BM_OK;
  }

  void shutdown() {
    {
      std::unique_lock<std::mutex> lk(mu_);
      if (!thread_.joinable()) return;
      stop_ = true;
      cv_.notify_all();
    }
    thread_.join();
  }

  // for tests and reporting
  int64_t device_in_use() {
    std::unique_lock<std::mutex> lk(mu_);
    return dev_.used();
  }
  int64_t steps_launched() const { return steps_launched_.load(); }
  int64_t max_step_size() const { return max_step_.load(); }
  int64_t max_overlap() const { return max_overlap_.load(); }

 private:
  void loop() {
    bm_status is = ex_->thread_init();
    {
      std::unique_lock<std::mutex> lk(mu_);
      init_status_ = is;
      started_ = true;
      cv_.notify_all();
      if (is != BM_OK) stop_ = true;
    }
    std::vector<std::unique_ptr<Step>> inflight;
    for (;;) {
      // 1. retire finished steps
      for (size_t i = 0; i < inflight.size();) {
        if (!ex_->step_done(inflight[i].get())) {
          ++i;
          continue;
        }
        finish(inflight[i].get());
        inflight.erase(inflight.begin() + i);
      }
      std::unique_ptr<Step> step(new Step);
      {
        std::unique_lock<std::mutex> lk(mu_);
        if (stop_) {
          if (inflight.empty()) break;
        } else {
          admit(step.get());
        }
        if (step->reqs.empty()) {
          if (inflight.empty()) {
            if (stop_) break;
            if (!queue_.empty()) {
              // nothing resident and the head still does not fit: it never will
              Request* r = queue_.front();
              queue_.pop_front();
              fail_request(r, BM_ENOMEM);
              continue;
            }
            cv_.wait(lk, [this] { return stop_ || !queue_.empty(); });
            continue;
          }
          // device work in flight: check again shortly (or at once on new arrivals); the
          // system clock keeps this on pthread_cond_timedwait
          cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::microseconds(100));
          continue;
        }
      }
      // 3. launch the step outside the lock
      bm_status s = ex_->begin_step(step.get());
      if (s != BM_OK) {
        ex_->wait_step(step.get());
        std::unique_lock<std::mutex> lk(mu_);
        for (Request* r : step->reqs) fail_request(r, s);
        dev_.release(step->hdr_off);
        continue;
      }
      steps_launched_++;
      max_step_ = std::max<int64_t>(max_step_.load(), (int64_t)step->reqs.size());
      inflight.push_back(std::move(step));
      max_overlap_ = std::max<int64_t>(max_overlap_.load(), (int64_t)inflight.size());
    }
    std::unique_lock<std::mutex> lk(mu_);
    for (Request* r : queue_) r->state = ReqState::Cancelled;
    queue_.clear();
  }

  // 2. admission (lock held): arrival order, stop at the first request that does not fit.
  //    The step header is reserved first, sized for the most requests this step can take.
  void admit(Step* step) {
    const int64_t max_step = cfg_.max_step > 0 ? cfg_.max_step : kMaxStep;
    const int64_t step_cap = std::max<int64_t>(1, std::min<int64_t>(max_step, cfg_.max_inflight / 2));
    const int64_t room = std::min<int64_t>(std::min<int64_t>((int64_t)queue_.size(), step_cap),
                                           cfg_.max_inflight - admitted_);
    if (room <= 0) return;
    if (!admit_some(step, room) && room > 1) {
      // the header for `room` requests may be what leaves the head out: a step of one
      // needs the smallest header
      admit_some(step, 1);
    }
  }

  // Reserve a header for up to `room` requests, then admit in arrival order while they
  // fit; false (nothing reserved) if not even the head fits.
  bool admit_some(Step* step, int64_t room) {
    if (!dev_.alloc(ex_->step_header_bytes((int)room), &step->hdr_off)) return false;
    std::vector<Request*> take;
    while (!queue_.empty() && (int64_t)take.size() < room) {
      Request* r = queue_.front();
      int64_t off;
      if (!dev_.alloc(r->dev_bytes, &off)) break;
      r->dev_off = off;
      bm_status ps = ex_->prepare(r);
      queue_.pop_front();
      if (ps != BM_OK) {
        fail_request(r, ps);
        continue;
      }
      r->state = ReqState::Admitted;
      r->t_admit = now_s();
      ++admitted_;
      take.push_back(r);
    }
    if (take.empty()) {
      dev_.release(step->hdr_off);
      step->hdr_off = -1;
      return false;
    }
    step->reqs = std::move(take);
    return true;
  }

  void fail_request(Request* r, bm_status s) {
    if (r->dev_off >= 0) dev_.release(r->dev_off);
    r->dev_off = -1;
    r->exec.reset();
    if (r->state == ReqState::Admitted) --admitted_;
    r->state = r->cancel_requested ? ReqState::Cancelled : ReqState::Failed;
    r->status = s;
    r->message = ex_->last_message();
    r->t_done = now_s();
  }

  void finish(Step* step) {
    const double t = now_s();
    const bm_status st = ex_->step_status(step);
    std::unique_lock<std::mutex> lk(mu_);
    if (st != BM_OK) {
      for (Request* r : step->reqs) fail_request(r, st);
      dev_.release(step->hdr_off);
      cv_.notify_all();
      return;
    }
    for (Request* r : step->reqs) {
      dev_.release(r->dev_off);
      r->dev_off = -1;
      r->exec.reset();
      r->t_done = t;
      --admitted_;
      if (r->cancel_requested) {
        r->state = ReqState::Cancelled;
        host_.release(r->host_off);
        r->host_off = -1;
      } else {
        r->state = ReqState::Done;
      }
    }
    dev_.release(step->hdr_off);
    cv_.notify_all();
  }

  Executor* ex_;
  bm_server_cfg cfg_;
  RangeAlloc dev_, host_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Request*> queue_;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs_;
  uint64_t next_ticket_ = 1;
  int64_t admitted_ = 0;
  int64_t copying_ = 0;  // submissions copying their image (counted against max_queue)
  bool stop_ = false, started_ = false;
  bm_status init_status_ = BM_OK;
  std::thread thread_;
  std::atomic<int64_t> steps_launched_{0}, max_step_{0}, max_overlap_{0};
};

}  // namespace bmk
