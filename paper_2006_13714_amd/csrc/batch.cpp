// Uneven batch: many images of different shapes, plans and precisions in as few launches as
// the kernels allow — one batch norm launch, then one persistent cross-term launch per
// (precision, K class, tile columns, channel tier) group of the specialised kernel, plus a
// regular launch per image whose shape only the generic kernel covers or whose reference
// blocks alone fill the device several times over (the persistent launch pays off for the
// images whose single launches would leave most of the device idle).
//
// Host side: form the groups, order each group's images by decreasing cost per reference
// block (largest contraction first, so the items handed out last are the cheapest), lay out
// the device records, copy them through a pinned staging buffer and launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "batch.h"
#include "batch_run.h"
#include "plan.h"

namespace bmk {

typedef void (*XcBatchKernel)(const BatchXc*, int, int, unsigned*);
#define BMK_DECL(P, K, T) XcBatchKernel batch_kernel_p##P##_k##K##_t##T(int tier);
BMK_DECL(0, 1, 2) BMK_DECL(0, 1, 3) BMK_DECL(0, 2, 2) BMK_DECL(0, 2, 3)
BMK_DECL(1, 1, 2) BMK_DECL(1, 1, 3) BMK_DECL(1, 2, 2) BMK_DECL(1, 2, 3)
BMK_DECL(2, 1, 2) BMK_DECL(2, 1, 3) BMK_DECL(2, 2, 2) BMK_DECL(2, 2, 3)
#undef BMK_DECL

hipError_t launch_norm_batch(const BatchNorm* d_items, int n, int total_tiles,
                             unsigned* d_counters, int n_counters, hipStream_t stream);
hipError_t launch_centers(const float* img, int C, int H, int W, float* centers,
                          hipStream_t stream);
void norm_tiles(const NormGeom& g, int* tiles_x, int* tiles_y);

static XcBatchKernel batch_kernel(int prec, int kr, int nt, int tier) {
  typedef XcBatchKernel (*Pick)(int);
  static const Pick table[3][2][2] = {
      {{batch_kernel_p0_k1_t2, batch_kernel_p0_k1_t3}, {batch_kernel_p0_k2_t2, batch_kernel_p0_k2_t3}},
      {{batch_kernel_p1_k1_t2, batch_kernel_p1_k1_t3}, {batch_kernel_p1_k2_t2, batch_kernel_p1_k2_t3}},
      {{batch_kernel_p2_k1_t2, batch_kernel_p2_k1_t3}, {batch_kernel_p2_k2_t2, batch_kernel_p2_k2_t3}}};
  if (prec < 0 || prec > 2 || kr < 1 || kr > 2 || nt < 2 || nt > 3 || tier < 0 || tier > 3)
    return nullptr;
  return table[prec][kr - 1][nt - 2](tier);
}

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

constexpr int kMaxCounters = 64;

int64_t batch_header_bytes(int n) {
  return 256 + align256((int64_t)n * sizeof(BatchXc)) + align256((int64_t)n * sizeof(BatchNorm));
}

// ---- pinned staging buffers for the record copies: a buffer is reused once the copy that
//      last read it has completed (its event), so calls stay asynchronous
namespace {
struct Staging {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  int device = -1;
  bool busy = false;
};
std::mutex g_stage_mu;
std::vector<Staging*> g_stage;

Staging* take_staging(size_t bytes, int device) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  for (Staging* s : g_stage)
    if (!s->busy && s->device == device && s->bytes >= bytes && hipEventQuery(s->done) == hipSuccess) {
      s->busy = true;
      return s;
    }
  size_t cap = 64 << 10;
  while (cap < bytes) cap <<= 1;
  Staging* s = new Staging;
  if (hipHostMalloc(&s->host, cap, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete s;
    return nullptr;
  }
  if (hipEventCreateWithFlags(&s->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(s->host);
    delete s;
    return nullptr;
  }
  s->bytes = cap;
  s->device = device;
  s->busy = true;
  g_stage.push_back(s);
  return s;
}

void release_staging(Staging* s, hipStream_t st, bool recorded_copy) {
  if (recorded_copy) (void)hipEventRecord(s->done, st);
  std::lock_guard<std::mutex> lk(g_stage_mu);
  s->busy = false;
}

struct Group {
  int prec, kr, nt, tier;
  std::vector<int> members;  // entry indices, in hand-out order
  int ws = 4, cap = 32, lds = 0, items = 0, rec_off = 0;
};
}  // namespace

// Workgroups of `k` one compute unit keeps at this size and LDS; raises the kernel's
// dynamic-LDS limit first.  Both are remembered per (kernel, device, size, LDS), so
// repeated batches (the serving loop) make no driver calls for them.
static hipError_t resident_blocks(const void* k, int dev, int threads, int lds, int* per_cu) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, int, int>, int> known;
  static std::map<std::pair<const void*, int>, int> lds_set;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(k, dev, threads, lds);
  auto it = known.find(key);
  if (it != known.end()) {
    *per_cu = it->second;
    return hipSuccess;
  }
  int& cur = lds_set[std::make_pair(k, dev)];
  if (lds > cur) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    cur = lds;
  }
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, threads, lds);
  if (e != hipSuccess) return e;
  known[key] = *per_cu;
  return hipSuccess;
}

static int shape_class(const bm_desc& d) { return (d.channels - 1) * 3 + ((d.patch + 1) / 2 - 2); }

// contraction work per reference block, up to a common factor
static int64_t block_cost(const bm_plan_s& p) {
  const int h2 = (p.desc.patch + 1) / 2;
  return (int64_t)p.desc.channels * h2 * h2;
}

bm_status run_batch(const BatchEntry* e, int n, void* d_header, hipStream_t s) {
  if (n == 0) return BM_OK;
  if (!e || n < 0 || !d_header) return fail(BM_EINVAL, "invalid batch arguments");
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_fail(he, "hipGetDevice");
  int max_lds = 0, n_cu = 0;
  if ((he = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) !=
          hipSuccess ||
      (he = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hip_fail(he, "hipDeviceGetAttribute");
  for (int b = 0; b < n; ++b) {
    const BatchEntry& x = e[b];
    if (!x.plan || !x.img || !x.nrm || !x.idx || !x.dist)
      return fail(BM_EINVAL, "batch entry %d: NULL plan or pointer", b);
    if (x.plan->device != dev)
      return fail(BM_EINVAL, "batch entry %d: plan made on device %d, current is %d", b,
                  x.plan->device, dev);
    if (plan_needs_centers(*x.plan) && !x.aux.centers)
      return fail(BM_EINVAL, "batch entry %d: centring plan without a centres slot", b);
    if (x.plan->desc.precision == BM_PREC_FP16X3 && !x.aux.amax)
      return fail(BM_EINVAL, "batch entry %d: float16 plan without a max map slot", b);
  }

  // ---- groups of the persistent kernel; the rest run their own launches one by one: the
  //      generic kernel's images, and images whose reference blocks alone fill the device
  //      several times over (kSingleBlocksPerCu per compute unit), which then run the
  //      single-image kernel with their own tuned configuration instead of the group's
  std::map<std::tuple<int, int, int, int>, Group> groups;
  std::vector<int> generic;
  constexpr int kSingleBlocksPerCu = 4;
  for (int b = 0; b < n; ++b) {
    const bm_plan_s& p = *e[b].plan;
    if (!p.geom.fast || p.geom.nwg_total >= kSingleBlocksPerCu * n_cu) {
      generic.push_back(b);
      continue;
    }
    const int tier = batch_tier(p.desc.precision, p.desc.channels);
    auto key = std::make_tuple(p.desc.precision, p.kr, p.geom.NT, tier);
    Group& g = groups[key];
    g.prec = p.desc.precision;
    g.kr = p.kr;
    g.nt = p.geom.NT;
    g.tier = tier;
    g.members.push_back(b);
  }
  if ((int)groups.size() > kMaxCounters) return fail(BM_EINVAL, "too many kernel groups");

  // ---- records
  const int64_t xc_off = 256;
  const int64_t norm_off = xc_off + align256((int64_t)n * sizeof(BatchXc));
  const size_t rec_bytes = (size_t)(batch_header_bytes(n) - xc_off);
  Staging* stg = take_staging(rec_bytes, dev);
  if (!stg) return fail(BM_ENOMEM, "pinned staging allocation failed");
  unsigned char* host = static_cast<unsigned char*>(stg->host);
  memset(host, 0, rec_bytes);
  BatchXc* hx = reinterpret_cast<BatchXc*>(host);
  BatchNorm* hn = reinterpret_cast<BatchNorm*>(host + (norm_off - xc_off));

  int rec = 0;
  for (auto& kv : groups) {
    Group& g = kv.second;
    std::stable_sort(g.members.begin(), g.members.end(), [&](int a, int b) {
      return block_cost(*e[a].plan) > block_cost(*e[b].plan);
    });
    // block size and candidate-buffer size: the members' tuned (waves, capacity) pair that
    // carries the most work (references x pixels x window positions), with the waves capped
    // at what the group's kernel takes and lowered until every member's LDS layout fits.
    // One pair serves the whole group: the launch takes the largest member's LDS, so a
    // single member's larger block or buffer would lower the occupancy of all of them.
    std::map<std::pair<int, int>, double> votes;
    for (int b : g.members) {
      const bm_desc& d = e[b].plan->desc;
      const double nref = (double)((d.height - d.patch) / d.stride + 1) *
                          ((d.width - d.patch) / d.stride + 1);
      votes[{e[b].plan->cfg.wy, e[b].plan->cfg.cap}] +=
          nref * d.channels * d.patch * d.patch * (double)d.window * d.window;
    }
    std::pair<int, int> best{4, 32};
    double best_w = -1.0;
    for (const auto& v : votes)
      if (v.second > best_w) {
        best = v.first;
        best_w = v.second;
      }
    g.cap = best.second;
    g.ws = std::max(1, std::min(best.first, batch_max_waves(g.tier)));
    for (; g.ws > 1; g.ws >>= 1) {
      bool fits = true;
      for (int b : g.members) {
        XcGeom t;
        fill_geom(e[b].plan->desc, g.ws, 1, g.cap, true, t, batch_norm_strip(g.prec, g.tier));
        fits &= t.lds_bytes <= max_lds;
      }
      if (fits) break;
    }
    g.rec_off = rec;
    for (int b : g.members) {
      const bm_plan_s& p = *e[b].plan;
      XcGeom xg;
      fill_geom(p.desc, g.ws, 1, g.cap, true, xg, batch_norm_strip(g.prec, g.tier));
      xg.p1_step = p.cfg.p1;
      if (xg.lds_bytes > max_lds) {
        release_staging(stg, s, false);
        return fail(BM_ENOTSUP, "batch entry %d: %d bytes of LDS", b, xg.lds_bytes);
      }
      g.lds = std::max(g.lds, xg.lds_bytes);
      BatchXc& r = hx[rec++];
      r.img = e[b].img;
      r.nrm = e[b].nrm;
      r.centers = e[b].aux.centers;
      r.amax = e[b].aux.amax;
      r.idx = e[b].idx;
      r.dist = e[b].dist;
      r.cls = shape_class(p.desc);
      r.item_begin = g.items;
      r.g = fast_geom(xg);
      g.items += xg.nwg_total;
    }
  }
  int tiles = 0;
  for (int b = 0; b < n; ++b) {
    const bm_plan_s& p = *e[b].plan;
    BatchNorm& r = hn[b];
    r.img = e[b].img;
    r.out = e[b].nrm;
    r.centers = e[b].aux.centers;
    r.amax = e[b].aux.amax;
    r.g = NormGeom{p.geom.H, p.geom.W, p.geom.C, p.geom.P, p.geom.Hv, p.geom.Wv,
                   p.desc.precision == BM_PREC_BF16X4 ? 1 : 0};
    int tx, ty;
    norm_tiles(r.g, &tx, &ty);
    r.tile_begin = tiles;
    r.tiles_x = tx;
    tiles += tx * ty;
  }

  unsigned char* dh = static_cast<unsigned char*>(d_header);
  he = hipMemcpyAsync(dh + xc_off, host, rec_bytes, hipMemcpyHostToDevice, s);
  release_staging(stg, s, he == hipSuccess);
  if (he != hipSuccess) return hip_fail(he, "record copy");

  // ---- launches: centring constants, all norms, persistent groups, generic images
  for (int b = 0; b < n; ++b) {
    const bm_plan_s& p = *e[b].plan;
    if (!e[b].aux.centers) continue;
    he = launch_centers(e[b].img, p.geom.C, p.geom.H, p.geom.W, e[b].aux.centers, s);
    if (he != hipSuccess) return hip_fail(he, "centring launch");
  }
  unsigned* counters = reinterpret_cast<unsigned*>(dh);
  he = launch_norm_batch(reinterpret_cast<const BatchNorm*>(dh + norm_off), n, tiles, counters,
                         (int)groups.size(), s);
  if (he != hipSuccess) return hip_fail(he, "batch norm launch");

  int q = 0;
  for (auto& kv : groups) {
    Group& g = kv.second;
    XcBatchKernel k = batch_kernel(g.prec, g.kr, g.nt, g.tier);
    if (!k) return fail(BM_ENOTSUP, "no persistent kernel for this group");
    int per_cu = 0;
    he = resident_blocks(reinterpret_cast<const void*>(k), dev, 64 * g.ws, g.lds, &per_cu);
    if (he != hipSuccess) return hip_fail(he, "persistent kernel set-up");
    if (per_cu < 1) return fail(BM_ENOTSUP, "persistent kernel does not fit a compute unit");
    const int grid = std::min(g.items, per_cu * n_cu);
    (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * g.ws), g.lds, s,
                       reinterpret_cast<const BatchXc*>(dh + xc_off) + g.rec_off,
                       (int)g.members.size(), g.items, counters + q);
    he = hipGetLastError();
    if (he != hipSuccess) return hip_fail(he, "persistent launch");
    ++q;
  }
  for (int b : generic) {
    bm_status st = run_cross_topk(*e[b].plan, e[b].img, e[b].nrm, e[b].aux, e[b].idx,
                                  e[b].dist, s);
    if (st != BM_OK) return st;
  }
  return BM_OK;
}

// bm_match_batch workspace: [header: counters + records] then per image a plan workspace
// layout [norm map][auxiliary slots]
static int64_t batch_ws_layout(int n, const bm_plan_t* plans, std::vector<int64_t>* offs) {
  int64_t off = batch_header_bytes(n);
  for (int b = 0; b < n; ++b) {
    if (offs) offs->push_back(off);
    off += desc_workspace_bytes(plans[b]->desc);
  }
  return off;
}

}  // namespace bmk

using namespace bmk;

extern "C" {

bm_status bm_batch_workspace(int32_t n, const bm_plan_t* plans, int64_t* bytes) {
  if (!bytes) return fail(BM_EINVAL, "bytes is NULL");
  if (n < 0 || (n > 0 && !plans)) return fail(BM_EINVAL, "invalid batch");
  for (int b = 0; b < n; ++b) {
    if (!plans[b]) return fail(BM_EINVAL, "plan %d is NULL", b);
    if (plan_is_3d(*plans[b])) return fail(BM_ENOTSUP, "plan %d is a 3D plan", b);
  }
  *bytes = n == 0 ? 0 : batch_ws_layout(n, plans, nullptr);
  return BM_OK;
}

bm_status bm_match_batch(int32_t n, const bm_plan_t* plans, const float* const* d_imgs,
                         int32_t* const* d_idx, float* const* d_dist, void* d_workspace,
                         void* stream) {
  if (n < 0) return fail(BM_EINVAL, "n < 0");
  if (n == 0) return BM_OK;
  if (!plans || !d_imgs || !d_idx || !d_dist) return fail(BM_EINVAL, "NULL array");
  for (int b = 0; b < n; ++b) {
    if (!plans[b]) return fail(BM_EINVAL, "plan %d is NULL", b);
    if (plan_is_3d(*plans[b])) return fail(BM_ENOTSUP, "plan %d is a 3D plan", b);
  }
  std::vector<int64_t> offs;
  const int64_t bytes = batch_ws_layout(n, plans, &offs);
  hipStream_t s = (hipStream_t)stream;
  void* ws = d_workspace;
  bool own = false;
  if (!ws) {
    hipError_t e = hipMalloc(&ws, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(BM_ENOMEM, "batch workspace hipMalloc(%lld)", (long long)bytes);
    }
    own = true;
  }
  std::vector<BatchEntry> ent(n);
  unsigned char* base = static_cast<unsigned char*>(ws);
  for (int b = 0; b < n; ++b) {
    ent[b].plan = plans[b];
    ent[b].img = d_imgs[b];
    ent[b].nrm = reinterpret_cast<float*>(base + offs[b]);
    ent[b].aux = plan_aux(*plans[b], base + offs[b]);
    ent[b].idx = d_idx[b];
    ent[b].dist = d_dist[b];
  }
  bm_status st = run_batch(ent.data(), n, ws, s);
  if (own) {
    hipError_t e = hipStreamSynchronize(s);
    (void)hipFree(ws);
    if (st == BM_OK && e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
  }
  return st;
}

}  // extern "C"
