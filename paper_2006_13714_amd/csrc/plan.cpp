// Plan configuration and the single-image launch sequence.
#include <hip/hip_runtime.h>

#include <cstring>

#include "plan.h"

namespace bmk {

hipError_t launch_norm(const float* img, float* out, const NormGeom& g, const float* center,
                       hipStream_t stream);
hipError_t launch_xcorr_f32(int ks_bucket, int kr, const float* img, const float* nrm, int* idx,
                            float* dist, const XcGeom& g, hipStream_t stream);
int f32_step_bucket(int ks);

static int kr_for(int k) { return k <= 16 ? 1 : (k <= 32 ? 2 : 4); }

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

int64_t plan_workspace_bytes(const bm_plan_s& p) {
  const XcGeom& g = p.geom;
  return align256((int64_t)g.Hv * g.Wv * 4);
}

bm_status apply_config(const bm_desc& d, const TileCfg& c, int max_lds, bm_plan_s* p) {
  XcGeom g;
  fill_geom(d, c.wy, c.wx, c.cap, g);
  if (g.lds_bytes > max_lds)
    return fail(BM_ENOTSUP, "tile needs %d bytes of LDS (limit %d)", g.lds_bytes, max_lds);
  const int bucket = f32_step_bucket(g.KS);
  if (bucket < 0) return fail(BM_ENOTSUP, "no kernel for %d contraction steps", g.KS);
  p->geom = g;
  p->ks_bucket = bucket;
  p->kr = kr_for(d.k);
  return BM_OK;
}

// Built-in rule: the largest wave grid whose LDS fits and that still gives every CU at least
// two workgroups; otherwise the configuration with the most workgroups that fits.
bm_status choose_config(const bm_desc& d, int max_lds, bm_plan_s* p) {
  static const TileCfg order[] = {{2, 2, 64}, {1, 2, 64}, {2, 1, 64}, {1, 1, 64}, {1, 1, 32}};
  const int min_wg = 512;
  bm_status best = BM_ENOTSUP;
  TileCfg chosen{0, 0, 0};
  int chosen_wg = -1;
  for (const TileCfg& c : order) {
    XcGeom g;
    fill_geom(d, c.wy, c.wx, c.cap, g);
    if (g.lds_bytes > max_lds) continue;
    if (g.nwg_total >= min_wg) {
      chosen = c;
      chosen_wg = g.nwg_total;
      break;
    }
    if (g.nwg_total > chosen_wg) {
      chosen = c;
      chosen_wg = g.nwg_total;
    }
  }
  if (chosen_wg < 0) return fail(BM_ENOTSUP, "window/patch/channels too large for LDS");
  best = apply_config(d, chosen, max_lds, p);
  return best;
}

bm_status run_match(const bm_plan_s& p, const float* d_img, int32_t* d_idx, float* d_dist,
                    void* ws, hipStream_t s) {
  if (!ws) return fail(BM_EINVAL, "no workspace");
  const XcGeom& g = p.geom;
  float* nrm = static_cast<float*>(ws);
  NormGeom ng{g.H, g.W, g.C, g.P, g.Hv, g.Wv};
  hipError_t e = launch_norm(d_img, nrm, ng, g.center, s);
  if (e != hipSuccess) return hip_fail(e, "norm launch");
  e = launch_xcorr_f32(p.ks_bucket, p.kr, d_img, nrm, d_idx, d_dist, g, s);
  if (e != hipSuccess) return hip_fail(e, "cross-term launch");
  return BM_OK;
}

}  // namespace bmk
