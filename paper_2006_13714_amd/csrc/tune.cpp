// Autotuner: picks the kernel configuration (waves per reference block or wave grid,
// bounding-sweep row step, candidate-buffer capacity) per shape class by timing every
// candidate on the device, and remembers the winner.
//
// Shape class: channels, patch, stride, window, K-register count, precision, and coarse
// reference-grid size buckets (the grid size changes the workgroup count and so the load
// balance, not the per-workgroup code).  Winners live in a process-wide table that bm_plan
// consults; with BM_TUNE_CACHE set they are also appended to that text file and loaded from
// it on first use, one line per class: "<key> | <configuration string>".  A table of the
// same format measured on MI355X (tuned_gfx950.txt, beside the library) is loaded first.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "plan.h"

namespace bmk {

static std::mutex g_tune_mu;
static std::map<std::string, std::string> g_tuned;
static bool g_loaded = false;

static int bucket(int n) { return n < 64 ? 0 : (n < 256 ? 1 : 2); }

static std::string class_key(const bm_desc& d) {
  char buf[160];
  const int nry = (d.height - d.patch) / d.stride + 1;
  const int nrx = (d.width - d.patch) / d.stride + 1;
  const int kr = d.k <= 16 ? 1 : (d.k <= 32 ? 2 : 4);
  snprintf(buf, sizeof(buf), "c%d p%d s%d w%d kr%d prec%d hb%d wb%d", d.channels, d.patch,
           d.stride, d.window, kr, d.precision, bucket(nry), bucket(nrx));
  return buf;
}

static void load_table_file(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    char* bar = strchr(line, '|');
    if (!bar) continue;
    std::string key(line, bar - line);
    while (!key.empty() && key.back() == ' ') key.pop_back();
    std::string cfg(bar + 1);
    while (!cfg.empty() && (cfg.back() == '\n' || cfg.back() == ' ')) cfg.pop_back();
    while (!cfg.empty() && cfg.front() == ' ') cfg.erase(cfg.begin());
    TileCfg c;
    if (parse_cfg(cfg.c_str(), &c)) g_tuned[key] = cfg;
  }
  fclose(f);
}

// The table measured on MI355X that ships beside the library (tuned_gfx950.txt), used when
// the current device is a gfx950; BM_TUNE_CACHE entries, read after it, take precedence.
static void load_cache_locked() {
  if (g_loaded) return;
  g_loaded = true;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
      strncmp(prop.gcnArchName, "gfx950", 6) == 0) {
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&load_table_file), &info) && info.dli_fname) {
      std::string dir(info.dli_fname);
      const size_t slash = dir.rfind('/');
      dir = slash == std::string::npos ? std::string(".") : dir.substr(0, slash);
      load_table_file((dir + "/tuned_gfx950.txt").c_str());
    }
  } else {
    (void)hipGetLastError();
  }
  const char* path = getenv("BM_TUNE_CACHE");
  if (path) load_table_file(path);
}

bool tuned_lookup(const bm_desc& d, TileCfg* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_cache_locked();
  auto it = g_tuned.find(class_key(d));
  return it != g_tuned.end() && parse_cfg(it->second.c_str(), out);
}

static void remember(const bm_desc& d, const std::string& cfg) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_cache_locked();
  const std::string key = class_key(d);
  g_tuned[key] = cfg;
  const char* path = getenv("BM_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s | %s\n", key.c_str(), cfg.c_str());
  fclose(f);
}

// Deterministic structured test image for tuning when the caller gives none: a few
// piecewise-constant cells plus hashed noise, so the selection work resembles real inputs.
__global__ void tune_image_kernel(float* img, int C, int H, int W) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C * H * W) return;
  const int x = i % W;
  const int y = (i / W) % H;
  const int c = i / (W * H);
  unsigned h = (unsigned)i * 2654435761u ^ 0x9e3779b9u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  const float noise = (float)(h & 0xffff) / 65536.f - 0.5f;
  const float cell = (float)((((x >> 5) * 7 + (y >> 5) * 13 + c * 3) % 11)) / 10.f;
  img[i] = cell + 0.4f * noise;
}

static std::vector<TileCfg> candidates(const bm_desc& d) {
  std::vector<TileCfg> v;
  if (fast_eligible(d)) {
    for (int ws : {1, 2, 4, 8})
      for (int p1 : {1, 2, 3, 4})
        for (int cap : {32, 48, 64}) {
          if (ws > fast_max_waves(d.precision, d.channels)) continue;
          TileCfg c;
          c.fast = true;
          c.wy = ws;
          c.p1 = p1;
          c.cap = cap;
          v.push_back(c);
        }
  }
  static const int shapes[][2] = {{1, 1}, {1, 2}, {2, 1}, {2, 2}};
  for (const auto& sh : shapes)
    for (int cap : {32, 64}) {
      TileCfg c;
      c.wy = sh[0];
      c.wx = sh[1];
      c.cap = cap;
      v.push_back(c);
    }
  return v;
}

}  // namespace bmk

using namespace bmk;

extern "C" {

bm_status bm_autotune(const bm_desc* desc, const float* d_img, int32_t reps, char* out_cfg,
                      int32_t out_len) {
  bm_status st = validate_desc(desc);
  if (st != BM_OK) return st;
  if (reps < 1 || reps > 1000) return fail(BM_EINVAL, "reps must be in [1, 1000]");
  // a 3D descriptor tunes the 2D problem of one slab (its first d planes), which is the
  // configuration its plans look up
  const bm_desc d = slab_desc(*desc);
  int dev = 0, max_lds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");

  const int64_t n_ref = (int64_t)((d.height - d.patch) / d.stride + 1) *
                        ((d.width - d.patch) / d.stride + 1);
  const int64_t img_elems = (int64_t)d.channels * d.height * d.width;
  float* own_img = nullptr;
  float* nrm = nullptr;  // a plan workspace: norm map, then the auxiliary slots
  int32_t* idx = nullptr;
  float* dist = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::string best_cfg;
  float best_ms = 1e30f;
  auto cleanup = [&]() {
    if (own_img) (void)hipFree(own_img);
    if (nrm) (void)hipFree(nrm);
    if (idx) (void)hipFree(idx);
    if (dist) (void)hipFree(dist);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
  };
  if (hipMalloc(&nrm, desc_workspace_bytes(d)) != hipSuccess ||
      hipMalloc(&idx, n_ref * d.k * 4) != hipSuccess ||
      hipMalloc(&dist, n_ref * d.k * 4) != hipSuccess) {
    cleanup();
    (void)hipGetLastError();
    return fail(BM_ENOMEM, "autotune buffers");
  }
  if (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(BM_EDEVICE, "autotune stream/events");
  }
  const float* img = d_img;
  if (!img) {
    if (hipMalloc(&own_img, img_elems * 4) != hipSuccess) {
      cleanup();
      (void)hipGetLastError();
      return fail(BM_ENOMEM, "autotune image");
    }
    (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
    hipLaunchKernelGGL(tune_image_kernel, dim3((unsigned)((img_elems + 255) / 256)), dim3(256), 0,
                       s, own_img, d.channels, d.height, d.width);
    img = own_img;
  }
  // Time every candidate once; then the fastest few again, interleaved, twice more each
  // (a single pass is within the run-to-run noise of the close candidates), and keep
  // each one's minimum.
  struct Timed {
    TileCfg c;
    bm_plan_s p;
    NormAux aux;
    float ms;
  };
  std::vector<Timed> timed;
  auto time_plan = [&](const bm_plan_s& p, const NormAux& aux, float* ms) {
    bool ok = true;
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < reps && ok; ++i) ok = run_cross_topk(p, img, nrm, aux, idx, dist, s) == BM_OK;
    (void)hipEventRecord(e1, s);
    if (!ok || hipEventSynchronize(e1) != hipSuccess) return false;
    (void)hipEventElapsedTime(ms, e0, e1);
    *ms /= reps;
    return true;
  };
  for (const TileCfg& c : candidates(d)) {
    Timed t;
    t.c = c;
    t.p.desc = d;
    t.p.device = dev;
    if (apply_config(d, c, max_lds, &t.p) != BM_OK) continue;
    t.aux = plan_aux(t.p, nrm);
    if (run_norms(t.p, img, nrm, t.aux, s) != BM_OK) continue;
    if (run_cross_topk(t.p, img, nrm, t.aux, idx, dist, s) != BM_OK) continue;
    if (!time_plan(t.p, t.aux, &t.ms)) continue;
    timed.push_back(t);
  }
  std::sort(timed.begin(), timed.end(), [](const Timed& a, const Timed& b) { return a.ms < b.ms; });
  const size_t top = std::min<size_t>(timed.size(), 4);
  for (int pass = 0; pass < 2; ++pass)
    for (size_t i = 0; i < top; ++i) {
      float ms = 0.f;
      if (run_norms(timed[i].p, img, nrm, timed[i].aux, s) == BM_OK &&
          time_plan(timed[i].p, timed[i].aux, &ms))
        timed[i].ms = std::min(timed[i].ms, ms);
    }
  for (size_t i = 0; i < top; ++i) {
    if (timed[i].ms < best_ms) {
      best_ms = timed[i].ms;
      char buf[96];
      format_cfg(timed[i].c, buf, sizeof(buf));
      best_cfg = buf;
    }
  }
  e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "autotune");
  if (best_cfg.empty()) return fail(BM_ENOTSUP, "no configuration runs this shape");
  remember(d, best_cfg);
  if (out_cfg && out_len > 0) snprintf(out_cfg, out_len, "%s", best_cfg.c_str());
  return BM_OK;
}

bm_status bm_plan_config(bm_plan_t plan, char* out_cfg, int32_t out_len, int32_t* source) {
  if (!plan) return fail(BM_EINVAL, "plan is NULL");
  if (out_cfg && out_len > 0) format_cfg(plan->cfg, out_cfg, out_len);
  if (source) *source = plan->cfg_source;
  return BM_OK;
}

}  // extern "C"
