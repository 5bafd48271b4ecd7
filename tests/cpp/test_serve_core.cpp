// Host test of the serving scheduler core with a stand-in executor (no device): admission by
// footprint, continuous batching, overlap of steps, cancel / poll states, failures, shutdown
// and the range allocator.  Prints "ALL OK" on success; any failed check aborts with a
// message.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <vector>

#include "serve_core.h"

using namespace bmk;

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

// Completes a step `secs_per_ref * refs` after it starts; results are a function of the
// request's ticket and position so that mixing up buffers is detected.
class MockExecutor : public Executor {
 public:
  explicit MockExecutor(int64_t host_bytes, double secs_per_ref = 2e-8)
      : host_(host_bytes), spr_(secs_per_ref) {}
  int64_t request_bytes(const bm_desc& d) override {
    return (int64_t)d.channels * d.height * d.width * 4 + desc_n_ref(d) * d.k * 8;
  }
  int64_t step_header_bytes(int n) override { return 256 + 64 * n; }
  void* host_base() override { return host_.data(); }
  bm_status prepare(Request* r) override {
    if (r->desc.flags == 0xBAD) return BM_ENOTSUP;
    return BM_OK;
  }
  struct St {
    double t_end;
  };
  bm_status begin_step(Step* s) override {
    double refs = 0;
    for (Request* r : s->reqs) {
      refs += r->n_ref;
      const float* img = reinterpret_cast<const float*>(host_.data() + r->host_off);
      const float first = img[0];  // image must still be intact when the step starts
      const int64_t n = r->n_ref * r->desc.k;
      int32_t* idx = reinterpret_cast<int32_t*>(host_.data() + r->host_off);
      float* dist = reinterpret_cast<float*>(host_.data() + r->host_off + n * 4);
      for (int64_t i = 0; i < n; ++i) {
        idx[i] = (int32_t)((r->ticket * 1000003ull + i) & 0x7fffffff);
        dist[i] = first + (float)i;
      }
      max_step_ = std::max<int64_t>(max_step_, (int64_t)s->reqs.size());
    }
    if (fail_next_) {
      fail_next_ = false;
      return BM_EDEVICE;
    }
    auto st = std::make_shared<St>();
    st->t_end = now_s() + spr_ * refs;
    s->exec = st;
    return BM_OK;
  }
  bool step_done(Step* s) override {
    auto* st = static_cast<St*>(s->exec.get());
    return !st || now_s() >= st->t_end;
  }
  void wait_step(Step* s) override {
    while (!step_done(s)) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  std::string last_message() override { return "mock launch failure"; }
  std::atomic<bool> fail_next_{false};
  int64_t max_step_ = 0;

 private:
  std::vector<char> host_;
  double spr_;
};

static bm_desc desc(int H, int W, int C = 1, int K = 16) {
  bm_desc d{};
  d.height = H;
  d.width = W;
  d.channels = C;
  d.patch = 8;
  d.stride = 3;
  d.window = 39;
  d.k = K;
  return d;
}

static std::vector<float> image(const bm_desc& d, float v) {
  return std::vector<float>((size_t)d.channels * d.height * d.width, v);
}

static bm_status wait_poll(Scheduler& s, uint64_t t, std::vector<int32_t>* idx,
                           std::vector<float>* dist, bm_request_stats* st) {
  for (int i = 0; i < 200000; ++i) {
    bm_status r = s.poll(t, idx ? idx->data() : nullptr, dist ? dist->data() : nullptr, st);
    if (r != BM_EAGAIN) return r;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  return BM_EAGAIN;
}

static void check_result(const Request& meta, uint64_t t, float first, const std::vector<int32_t>& idx,
                         const std::vector<float>& dist) {
  const int64_t n = meta.n_ref * meta.desc.k;
  for (int64_t i = 0; i < n; i += 97) {
    CHECK(idx[i] == (int32_t)((t * 1000003ull + i) & 0x7fffffff));
    CHECK(dist[i] == first + (float)i);
  }
}

static void test_alloc() {
  RangeAlloc a(4096, 256);
  int64_t o1, o2, o3, o4;
  CHECK(a.alloc(300, &o1) && o1 == 0);
  CHECK(a.alloc(256, &o2) && o2 == 512);
  CHECK(a.alloc(1024, &o3) && o3 == 768);
  CHECK(a.used() == 512 + 256 + 1024);
  a.release(o2);
  CHECK(a.alloc(200, &o4) && o4 == 512);  // first fit reuses the hole
  a.release(o4);
  a.release(o1);
  a.release(o3);
  CHECK(a.used() == 0 && a.largest_free() == 4096);  // fully coalesced
  CHECK(!a.alloc(4097, &o1));
  CHECK(a.alloc(4096, &o1) && o1 == 0);
}

static void test_basic_and_results() {
  MockExecutor ex(64 << 20);
  bm_server_cfg cfg{256 << 20, 64, 1024};
  Scheduler s(&ex, cfg, cfg.hbm_budget_bytes, 64 << 20);
  CHECK(s.start() == BM_OK);
  std::vector<uint64_t> t;
  std::vector<bm_desc> ds;
  for (int i = 0; i < 20; ++i) {
    bm_desc d = desc(64 + 8 * i, 80 + 4 * i, 1 + i % 4);
    auto img = image(d, (float)i);
    uint64_t tk;
    const char* why;
    CHECK(s.submit(d, img.data(), &tk, &why) == BM_OK);
    t.push_back(tk);
    ds.push_back(d);
  }
  std::set<uint64_t> uniq(t.begin(), t.end());
  CHECK(uniq.size() == t.size());
  for (int i = 0; i < 20; ++i) {
    Request meta;
    meta.desc = ds[i];
    meta.n_ref = desc_n_ref(ds[i]);
    std::vector<int32_t> idx(meta.n_ref * ds[i].k);
    std::vector<float> dist(idx.size());
    bm_request_stats st;
    CHECK(wait_poll(s, t[i], &idx, &dist, &st) == BM_OK);
    check_result(meta, t[i], (float)i, idx, dist);
    CHECK(st.n_ref == meta.n_ref);
    CHECK(st.queue_s >= 0 && st.device_s >= 0);
    CHECK(std::abs(st.total_s - (st.queue_s + st.device_s)) < 1e-9);
    CHECK(s.poll(t[i], nullptr, nullptr, nullptr) == BM_ENOTFOUND);  // retired
  }
  CHECK(s.device_in_use() == 0);
  s.shutdown();
}

static void test_admission_by_footprint() {
  // each request needs ~1.2 MB; the budget holds two plus headers
  MockExecutor ex(64 << 20, 1e-6);
  bm_desc d = desc(256, 256);
  const int64_t need = ex.request_bytes(d);
  bm_server_cfg cfg{2 * need + 4096, 64, 1024};
  Scheduler s(&ex, cfg, cfg.hbm_budget_bytes, 64 << 20);
  CHECK(s.start() == BM_OK);
  std::vector<uint64_t> t;
  for (int i = 0; i < 8; ++i) {
    auto img = image(d, (float)i);
    uint64_t tk;
    const char* why;
    CHECK(s.submit(d, img.data(), &tk, &why) == BM_OK);
    t.push_back(tk);
  }
  int64_t peak = 0;
  for (int i = 0; i < 8; ++i) {
    bm_status r;
    while ((r = s.poll(t[i], nullptr, nullptr, nullptr)) == BM_EAGAIN) {
      peak = std::max(peak, s.device_in_use());
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    CHECK(r == BM_OK);
  }
  CHECK(peak <= cfg.hbm_budget_bytes);
  CHECK(ex.max_step_ <= 2);
  CHECK(s.max_step_size() <= Scheduler::kMaxStep);
  // a request larger than the whole budget is refused at once
  bm_desc big = desc(2048, 2048, 4);
  auto img = image(big, 1.f);
  uint64_t tk;
  const char* why = "";
  CHECK(s.submit(big, img.data(), &tk, &why) == BM_EBUSY);
  s.shutdown();
}

static void test_header_does_not_block_head() {
  // The budget holds one request plus the header of a one-request step, but not the header
  // sized for the six queued requests: every request must still run (one step each).
  MockExecutor ex(64 << 20, 1e-7);
  bm_desc d = desc(200, 200);
  const int64_t need = (ex.request_bytes(d) + 255) / 256 * 256;
  const int64_t h1 = (ex.step_header_bytes(1) + 255) / 256 * 256;
  CHECK((ex.step_header_bytes(6) + 255) / 256 * 256 > h1);
  bm_server_cfg cfg{need + h1, 64, 1024};
  Scheduler s(&ex, cfg, cfg.hbm_budget_bytes, 64 << 20);
  CHECK(s.start() == BM_OK);
  std::vector<uint64_t> t;
  std::vector<float> first;
  for (int i = 0; i < 6; ++i) {
    auto img = image(d, 3.f + i);
    uint64_t tk;
    const char* why = "";
    CHECK(s.submit(d, img.data(), &tk, &why) == BM_OK);
    t.push_back(tk);
    first.push_back(3.f + i);
  }
  Request meta;
  meta.desc = d;
  meta.n_ref = desc_n_ref(d);
  for (int i = 0; i < 6; ++i) {
    std::vector<int32_t> idx(meta.n_ref * d.k);
    std::vector<float> dist(meta.n_ref * d.k);
    CHECK(wait_poll(s, t[i], &idx, &dist, nullptr) == BM_OK);
    check_result(meta, t[i], first[i], idx, dist);
  }
  CHECK(ex.max_step_ == 1);
  s.shutdown();
}

static void test_failure_message() {
  // a failed step reports the executor's message with the status
  MockExecutor ex(16 << 20, 1e-7);
  bm_server_cfg cfg{64 << 20, 64, 1024};
  Scheduler s(&ex, cfg, cfg.hbm_budget_bytes, 16 << 20);
  CHECK(s.start() == BM_OK);
  bm_desc d = desc(64, 64);
  auto img = image(d, 1.f);
  ex.fail_next_ = true;
  uint64_t tk;
  const char* why = "";
  CHECK(s.submit(d, img.data(), &tk, &why) == BM_OK);
  bm_status r;
  std::string msg;
  for (int i = 0; i < 200000; ++i) {
    if ((r = s.poll(tk, nullptr, nullptr, nullptr, &msg)) != BM_EAGAIN) break;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  CHECK(r == BM_EDEVICE);
  CHECK(msg == "mock launch failure");
  s.shutdown();
}

static void test_continuous_batching_overlap() {
  // slow steps: requests that arrive while the first step runs are launched as further
  // steps before it completes
  MockExecutor ex(256 << 20, 2e-6);
  bm_server_cfg cfg{512 << 20, 64, 1024};
  Scheduler s(&ex, cfg, cfg.hbm_budget_bytes, 256 << 20);
  CHECK(s.start() == BM_OK);
  std::vector<uint64_t> t;
  for (int i = 0; i < 6; ++i) {
    bm_desc d = desc(512, 512);
    auto img = image(d, (float)i);
    uint64_t tk;
    const char* why;
    CHECK(s.submit(d, img.data(), &tk, &why) == BM_OK);
    t.push_back(tk);
    std::this_thread::sleep_for(std::chrono::milliseconds(5));
  }
  for (uint64_t tk : t) CHECK(wait_poll(s, tk, nullptr, nullptr, nullptr) == BM_OK);
  CHECK(s.steps_launched() >= 2);
  CHECK(s.max_overlap() >= 2);
  s.shutdown();
}

static void test_max_step() {
  // a step takes at most max_step requests even when many wait
  MockExecutor ex(256 << 20, 1e-7);
  bm_server_cfg cfg{512 << 20, 64, 1024, 3};
  Scheduler s(&ex, cfg, cfg.hbm_budget_bytes, 256 << 20);
  CHECK(s.start() == BM_OK);
  std::vector<uint64_t> t;
  for (int i = 0; i < 12; ++i) {
    bm_desc d = desc(128, 128);
    auto img = image(d, (float)i);
    uint64_t tk;
    const char* why;
    CHECK(s.submit(d, img.data(), &tk, &why) == BM_OK);
    t.push_back(tk);
  }
  for (uint64_t tk : t) CHECK(wait_poll(s, tk, nullptr, nullptr, nullptr) == BM_OK);
  CHECK(ex.max_step_ <= 3);
  CHECK(s.max_step_size() <= 3);
  CHECK(s.steps_launched() >= 4);
  s.shutdown();
}

static void test_max_inflight_one() {
  MockExecutor ex(64 << 20, 1e-7);
  bm_server_cfg cfg{256 << 20, 1, 1024};
  Scheduler s(&ex, cfg, cfg.hbm_budget_bytes, 64 << 20);
  CHECK(s.start() == BM_OK);
  std::vector<uint64_t> t;
  for (int i = 0; i < 5; ++i) {
    bm_desc d = desc(128, 128);
    auto img = image(d, 0.f);
    uint64_t tk;
    const char* why;
    CHECK(s.submit(d, img.data(), &tk, &why) == BM_OK);
    t.push_back(tk);
  }
  for (uint64_t tk : t) CHECK(wait_poll(s, tk, nullptr, nullptr, nullptr) == BM_OK);
  CHECK(ex.max_step_ == 1 && s.max_overlap() == 1 && s.steps_launched() == 5);
  s.shutdown();
}

static void test_cancel_fail_and_limits() {
  MockExecutor ex(64 << 20, 5e-6);
  bm_server_cfg cfg{256 << 20, 1, 3};
  Scheduler s(&ex, cfg, cfg.hbm_budget_bytes, 64 << 20);
  CHECK(s.start() == BM_OK);
  bm_desc d = desc(256, 256);
  auto img = image(d, 1.f);
  uint64_t a, b, c, e;
  const char* why;
  CHECK(s.submit(d, img.data(), &a, &why) == BM_OK);
  std::this_thread::sleep_for(std::chrono::milliseconds(2));  // a is admitted (slow step)
  CHECK(s.submit(d, img.data(), &b, &why) == BM_OK);
  CHECK(s.submit(d, img.data(), &c, &why) == BM_OK);
  CHECK(s.cancel(b) == BM_OK);  // still queued behind a (max_inflight 1)
  CHECK(s.cancel(a) == BM_OK);  // admitted: finishes, results dropped
  CHECK(s.cancel(999999) == BM_ENOTFOUND);
  CHECK(wait_poll(s, a, nullptr, nullptr, nullptr) == BM_ECANCELED);
  CHECK(wait_poll(s, b, nullptr, nullptr, nullptr) == BM_ECANCELED);
  CHECK(wait_poll(s, c, nullptr, nullptr, nullptr) == BM_OK);
  CHECK(s.poll(a, nullptr, nullptr, nullptr) == BM_ENOTFOUND);
  // queue limit: three queued requests fill it while one is admitted
  uint64_t q[4];
  CHECK(s.submit(d, img.data(), &q[0], &why) == BM_OK);
  std::this_thread::sleep_for(std::chrono::milliseconds(1));
  int busy = 0;
  for (int i = 1; i < 4; ++i) busy += s.submit(d, img.data(), &q[i], &why) == BM_EBUSY;
  CHECK(busy >= 0);
  // a request whose plan cannot be made fails with that status
  bm_desc bad = d;
  bad.flags = 0xBAD;
  int tries = 0;
  while (s.submit(bad, img.data(), &e, &why) == BM_EBUSY && tries++ < 10000)
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  CHECK(wait_poll(s, e, nullptr, nullptr, nullptr) == BM_ENOTSUP);
  // a device failure while launching fails the step's requests
  ex.fail_next_ = true;
  uint64_t f;
  tries = 0;
  while (s.submit(d, img.data(), &f, &why) == BM_EBUSY && tries++ < 10000)
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  CHECK(wait_poll(s, f, nullptr, nullptr, nullptr) == BM_EDEVICE);
  s.shutdown();
  CHECK(s.device_in_use() == 0);
}

static void test_concurrent_clients() {
  MockExecutor ex(256 << 20, 1e-8);
  bm_server_cfg cfg{256 << 20, 16, 4096};
  Scheduler s(&ex, cfg, cfg.hbm_budget_bytes, 256 << 20);
  CHECK(s.start() == BM_OK);
  std::atomic<int> ok{0};
  std::vector<std::thread> th;
  for (int c = 0; c < 4; ++c)
    th.emplace_back([&, c] {
      for (int i = 0; i < 25; ++i) {
        bm_desc d = desc(64 + c * 16 + i, 96 + i, 1 + (i + c) % 3);
        auto img = image(d, (float)(c * 100 + i));
        uint64_t tk;
        const char* why;
        if (s.submit(d, img.data(), &tk, &why) != BM_OK) continue;
        Request meta;
        meta.desc = d;
        meta.n_ref = desc_n_ref(d);
        std::vector<int32_t> idx(meta.n_ref * d.k);
        std::vector<float> dist(idx.size());
        if (wait_poll(s, tk, &idx, &dist, nullptr) == BM_OK) {
          check_result(meta, tk, (float)(c * 100 + i), idx, dist);
          ok++;
        }
      }
    });
  for (auto& x : th) x.join();
  CHECK(ok == 100);
  s.shutdown();
}

static void test_shutdown_with_work() {
  MockExecutor ex(64 << 20, 1e-6);
  bm_server_cfg cfg{256 << 20, 2, 1024};
  Scheduler s(&ex, cfg, cfg.hbm_budget_bytes, 64 << 20);
  CHECK(s.start() == BM_OK);
  for (int i = 0; i < 10; ++i) {
    bm_desc d = desc(256, 256);
    auto img = image(d, 0.f);
    uint64_t tk;
    const char* why;
    CHECK(s.submit(d, img.data(), &tk, &why) == BM_OK);
  }
  s.shutdown();  // drains admitted steps, drops the queue
  CHECK(s.device_in_use() == 0);
}

int main() {
  test_alloc();
  test_basic_and_results();
  test_admission_by_footprint();
  test_header_does_not_block_head();
  test_max_step();
  test_failure_message();
  test_continuous_batching_overlap();
  test_max_inflight_one();
  test_cancel_fail_and_limits();
  test_concurrent_clients();
  test_shutdown_with_work();
  std::printf("ALL OK\n");
  return 0;
}
