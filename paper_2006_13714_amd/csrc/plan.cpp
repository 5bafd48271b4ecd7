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
hipError_t prepare_xcorr_f32(int ks_bucket, int kr, int lds_bytes);
hipError_t prepare_xcorr_fast(int c, int h2, int kr, int nt, int lds_bytes);
hipError_t launch_xcorr_fast(int c, int h2, int kr, int nt, const float* img, const float* nrm,
                             int* idx, float* dist, const XcGeom& g, hipStream_t stream);

static int kr_for(int k) { return k <= 16 ? 1 : (k <= 32 ? 2 : 4); }

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

int64_t plan_workspace_bytes(const bm_plan_s& p) {
  const XcGeom& g = p.geom;
  return align256((int64_t)g.Hv * g.Wv * 4);
}

static bool fast_eligible(const bm_desc& d) {
  const int h2 = (d.patch + 1) / 2;
  const int nt = (3 * d.stride + 2 * (d.window / 2) + 1 + kTileN - 1) / kTileN;
  return d.channels <= 4 && h2 >= 2 && h2 <= 4 && d.k <= 32 && nt >= 2 && nt <= 3;
}

bm_status apply_config(const bm_desc& d, const TileCfg& c, int max_lds, bm_plan_s* p) {
  XcGeom g;
  fill_geom(d, c.wy, c.wx, c.cap, c.fast, g);
  if (g.lds_bytes > max_lds)
    return fail(BM_ENOTSUP, "tile needs %d bytes of LDS (limit %d)", g.lds_bytes, max_lds);
  if (c.fast && (!fast_eligible(d) || g.SW > kFastRS))
    return fail(BM_ENOTSUP, "shape outside the specialised kernel");
  p->geom = g;
  p->kr = kr_for(d.k);
  hipError_t e;
  if (c.fast) {
    p->ks_bucket = 0;
    e = prepare_xcorr_fast(d.channels, (d.patch + 1) / 2, p->kr, g.NT, g.lds_bytes);
  } else {
    const int bucket = f32_step_bucket(g.KS);
    if (bucket < 0) return fail(BM_ENOTSUP, "no kernel for %d contraction steps", g.KS);
    p->ks_bucket = bucket;
    e = prepare_xcorr_f32(bucket, p->kr, g.lds_bytes);
  }
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  return BM_OK;
}

// Built-in rule: prefer the specialised kernel; take the largest wave grid whose LDS fits
// and that still gives every CU at least two workgroups, else the configuration with the
// most workgroups that fits.
bm_status choose_config(const bm_desc& d, int max_lds, bm_plan_s* p) {
  // specialised kernel: waves per reference block, largest first that fits the LDS
  if (fast_eligible(d)) {
    for (int ws : {4, 2, 1}) {
      XcGeom g;
      fill_geom(d, ws, 1, 32, true, g);
      if (g.lds_bytes <= max_lds && g.SW <= kFastRS)
        return apply_config(d, TileCfg{ws, 1, 32, true}, max_lds, p);
    }
  }
  // generic kernel: the largest wave grid whose LDS fits and that still gives every CU at
  // least two workgroups, else the configuration with the most workgroups that fits
  static const TileCfg shapes[] = {{2, 2, 64, false}, {1, 2, 64, false}, {2, 1, 64, false},
                                   {1, 1, 64, false}, {1, 1, 32, false}};
  const int min_wg = 512;
  TileCfg chosen{0, 0, 0, false};
  int chosen_wg = -1;
  for (const TileCfg& c : shapes) {
    XcGeom g;
    fill_geom(d, c.wy, c.wx, c.cap, false, g);
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
  return apply_config(d, chosen, max_lds, p);
}

bm_status run_norms(const bm_plan_s& p, const float* d_img, float* d_norm, hipStream_t s) {
  const XcGeom& g = p.geom;
  NormGeom ng{g.H, g.W, g.C, g.P, g.Hv, g.Wv};
  hipError_t e = launch_norm(d_img, d_norm, ng, g.center, s);
  if (e != hipSuccess) return hip_fail(e, "norm launch");
  return BM_OK;
}

bm_status run_cross_topk(const bm_plan_s& p, const float* d_img, const float* d_norm,
                         int32_t* d_idx, float* d_dist, hipStream_t s) {
  const bm_desc& d = p.desc;
  hipError_t e = p.geom.fast ? launch_xcorr_fast(d.channels, (d.patch + 1) / 2, p.kr, p.geom.NT,
                                                 d_img, d_norm, d_idx, d_dist, p.geom, s)
                             : launch_xcorr_f32(p.ks_bucket, p.kr, d_img, d_norm, d_idx, d_dist,
                                                p.geom, s);
  if (e != hipSuccess) return hip_fail(e, "cross-term launch");
  return BM_OK;
}

bm_status run_match(const bm_plan_s& p, const float* d_img, int32_t* d_idx, float* d_dist,
                    void* ws, hipStream_t s) {
  if (!ws) return fail(BM_EINVAL, "no workspace");
  float* nrm = static_cast<float*>(ws);
  bm_status st = run_norms(p, d_img, nrm, s);
  if (st != BM_OK) return st;
  return run_cross_topk(p, d_img, nrm, d_idx, d_dist, s);
}

}  // namespace bmk
