// Plan configuration (built-in rule, autotuner table, explicit override) and the
// single-image launch sequence.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "plan.h"

namespace bmk {

hipError_t launch_norm(const float* img, float* out, const NormGeom& g, const float* centers,
                       float* amax, hipStream_t stream);
hipError_t launch_centers(const float* img, int C, int H, int W, float* centers,
                          hipStream_t stream);
hipError_t launch_xcorr_f32(int ks_bucket, int kr, const float* img, const float* nrm,
                            const float* centers, int* idx, float* dist, const XcGeom& g,
                            hipStream_t stream);
int f32_step_bucket(int ks);
hipError_t prepare_xcorr_f32(int ks_bucket, int kr, int lds_bytes);
hipError_t prepare_xcorr_fast(int prec, int c, int h2, int kr, int nt, int lds_bytes);
hipError_t prepare_xcorr_depth(int prec, int c, int h2, int kr, int nt, int lds_bytes);
hipError_t launch_xcorr_depth(int prec, int c, int h2, int kr, int nt, const float* vol,
                              const float* nrm, const float* amax, int* idx, float* dist,
                              const XcGeom& g, const DepthGeom& dg, hipStream_t stream);
hipError_t launch_xcorr_fast(int prec, int c, int h2, int kr, int nt, const float* img,
                             const float* nrm, const float* centers, const float* amax,
                             int* idx, float* dist, const XcGeom& g, hipStream_t stream);

static int kr_for(int k) { return k <= 16 ? 1 : (k <= 32 ? 2 : 4); }

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

bool parse_cfg(const char* text, TileCfg* out) {
  if (!text) return false;
  TileCfg c;
  char kind[16] = {0};
  int n = 0;
  if (sscanf(text, "%15s%n", kind, &n) != 1) return false;
  if (!strcmp(kind, "fast")) c.fast = true;
  else if (!strcmp(kind, "generic")) c.fast = false;
  else return false;
  const char* p = text + n;
  char key[16];
  int val, m;
  while (sscanf(p, " %15[a-z0-9]=%d%n", key, &val, &m) == 2) {
    if (!strcmp(key, "ws") || !strcmp(key, "wy")) c.wy = val;
    else if (!strcmp(key, "wx")) c.wx = val;
    else if (!strcmp(key, "cap")) c.cap = val;
    else if (!strcmp(key, "p1")) c.p1 = val;
    else return false;
    p += m;
  }
  while (*p == ' ') ++p;
  if (*p) return false;
  if (c.wy < 1 || c.wx < 1 || c.wy * c.wx > (c.fast ? 8 : 4) || c.cap < 32 || c.cap > 256 ||
      (c.cap & 15) || c.p1 < 1 || c.p1 > 8)
    return false;
  if (c.fast && c.wx != 1) return false;
  *out = c;
  return true;
}

void format_cfg(const TileCfg& c, char* out, int len) {
  if (c.fast) snprintf(out, len, "fast ws=%d p1=%d cap=%d", c.wy, c.p1, c.cap);
  else snprintf(out, len, "generic wy=%d wx=%d cap=%d", c.wy, c.wx, c.cap);
}

// workspace: [norm map (Hv*Wv floats)] [centring constants: 8 floats] [per-tile max map of
// the norm pass] (256-byte aligned parts)
int64_t norm_tile_count(const bm_desc& d) {
  const int64_t hv = d.height - d.patch + 1, wv = d.width - d.patch + 1;
  return ((wv + kNormTX - 1) / kNormTX) * ((hv + kNormTY - 1) / kNormTY);
}

int64_t desc_workspace_bytes(const bm_desc& d) {
  const int64_t hv = d.height - d.patch + 1, wv = d.width - d.patch + 1;
  return align256(hv * wv * 4) + 256 + align256(norm_tile_count(d) * 4);
}

bm_desc slab_desc(const bm_desc& d) {
  bm_desc t = d;
  if (d.window_depth > 0) t.channels = d.patch_depth;
  t.patch_depth = 0;
  t.window_depth = 0;
  return t;
}

// 3D plans stack Z norm maps, and Z per-tile max maps in the auxiliary region
int64_t plan_workspace_bytes(const bm_plan_s& p) {
  if (!plan_is_3d(p)) return desc_workspace_bytes(p.desc);
  const int64_t hv = p.geom.Hv, wv = p.geom.Wv;
  return align256(p.Z * hv * wv * 4) + 256 + align256(p.Z * norm_tile_count(p.desc) * 4);
}

bool plan_needs_centers(const bm_plan_s& p) { return (p.desc.flags & BM_FLAG_CENTER) != 0; }

NormAux aux_at(const bm_plan_s& p, void* slot) {
  NormAux a{nullptr, nullptr};
  if (!slot) return a;
  char* base = static_cast<char*>(slot);
  if (plan_needs_centers(p)) a.centers = reinterpret_cast<float*>(base);
  if (p.desc.precision == BM_PREC_FP16X3) a.amax = reinterpret_cast<float*>(base + 256);
  return a;
}

NormAux plan_aux(const bm_plan_s& p, void* ws) {
  if (!ws) return NormAux{nullptr, nullptr};
  return aux_at(p, static_cast<char*>(ws) + align256((int64_t)p.Z * p.geom.Hv * p.geom.Wv * 4));
}

bool fast_eligible(const bm_desc& d) {
  const int h2 = (d.patch + 1) / 2;
  const int nt = (3 * d.stride + d.window + kTileN - 1) / kTileN;
  const int h2_min = d.precision == BM_PREC_FP32 ? 2 : 3;
  return d.channels <= 4 && h2 >= h2_min && h2 <= 4 && d.k <= 32 && nt >= 2 && nt <= 3;
}

bm_status apply_config(const bm_desc& d, const TileCfg& c, int max_lds, bm_plan_s* p) {
  XcGeom g;
  fill_geom(d, c.wy, c.wx, c.cap, c.fast, g);
  if (c.fast) g.p1_step = c.p1;
  if (g.lds_bytes > max_lds)
    return fail(BM_ENOTSUP, "tile needs %d bytes of LDS (limit %d)", g.lds_bytes, max_lds);
  if (c.fast && (!fast_eligible(d) || g.SW > g.RS))
    return fail(BM_ENOTSUP, "shape outside the specialised kernel");
  if (c.fast && c.wy > fast_max_waves(d.precision, d.channels))
    return fail(BM_ENOTSUP, "%d waves per block exceed this kernel's limit", c.wy);
  if (!c.fast && d.precision != BM_PREC_FP32)
    return fail(BM_ENOTSUP, "split precision needs C <= 4, patch 5..8, K <= 32 and "
                            "17 <= 3*stride + window <= 48");
  if (!c.fast && (d.flags & BM_FLAG_NCC))
    return fail(BM_ENOTSUP, "NCC needs C <= 4, patch 3..8, K <= 32 and 17 <= 3*stride + window <= 48");
  p->geom = g;
  p->cfg = c;
  p->kr = kr_for(d.k);
  hipError_t e;
  if (c.fast) {
    p->ks_bucket = 0;
    e = prepare_xcorr_fast(d.precision, d.channels, (d.patch + 1) / 2, p->kr, g.NT, g.lds_bytes);
  } else {
    const int bucket = f32_step_bucket(g.KS);
    if (bucket < 0) return fail(BM_ENOTSUP, "no kernel for %d contraction steps", g.KS);
    p->ks_bucket = bucket;
    e = prepare_xcorr_f32(bucket, p->kr, g.lds_bytes);
  }
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  return BM_OK;
}

// Built-in rule.  Specialised kernel: the most waves per reference block (up to the
// kernel's limit) whose LDS fits.
// Generic kernel: the largest wave grid whose LDS fits and that still gives every CU at
// least two workgroups, else the configuration with the most workgroups that fits.
static bm_status builtin_config(const bm_desc& d, int max_lds, bm_plan_s* p) {
  if (fast_eligible(d)) {
    // 8-wave blocks take a 48-entry candidate buffer where it fits (fewer flushes)
    for (int ws : {8, 4, 2, 1}) {
      if (ws > fast_default_waves(d.precision, d.channels)) continue;
      for (int cap : {48, 32}) {
        if (cap == 48 && ws != 8) continue;
        XcGeom g;
        fill_geom(d, ws, 1, cap, true, g);
        if (g.lds_bytes <= max_lds && g.SW <= g.RS) {
          TileCfg c;
          c.fast = true;
          c.wy = ws;
          c.cap = cap;
          c.p1 = 2;
          return apply_config(d, c, max_lds, p);
        }
      }
    }
  }
  if (d.precision != BM_PREC_FP32)
    return fail(BM_ENOTSUP, "split precision needs C <= 4, patch 5..8, K <= 32 and "
                            "17 <= 3*stride + window <= 48 (and the LDS to stage it)");
  if (d.flags & BM_FLAG_NCC)
    return fail(BM_ENOTSUP, "NCC needs C <= 4, patch 3..8, K <= 32 and 17 <= 3*stride + window <= 48");
  static const int shapes[][3] = {{2, 2, 64}, {1, 2, 64}, {2, 1, 64}, {1, 1, 64}, {1, 1, 32}};
  const int min_wg = 512;
  TileCfg chosen;
  int chosen_wg = -1;
  for (const auto& sh : shapes) {
    XcGeom g;
    fill_geom(d, sh[0], sh[1], sh[2], false, g);
    if (g.lds_bytes > max_lds) continue;
    TileCfg c;
    c.wy = sh[0];
    c.wx = sh[1];
    c.cap = sh[2];
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

bool tuned_lookup(const bm_desc& d, TileCfg* out);  // autotuner table (tune.cpp)

bm_status choose_config(const bm_desc& d, int max_lds, bm_plan_s* p) {
  // explicit override (tuning experiments): honoured only if it applies to this shape
  const char* env = getenv("BM_CFG");
  TileCfg c;
  if (env && parse_cfg(env, &c) && apply_config(d, c, max_lds, p) == BM_OK) {
    p->cfg_source = 2;
    return BM_OK;
  }
  if (tuned_lookup(d, &c) && apply_config(d, c, max_lds, p) == BM_OK) {
    p->cfg_source = 1;
    return BM_OK;
  }
  p->cfg_source = 0;
  return builtin_config(d, max_lds, p);
}

bm_status run_norms(const bm_plan_s& p, const float* d_img, float* d_norm, const NormAux& aux,
                    hipStream_t s) {
  const XcGeom& g = p.geom;
  hipError_t e;
  if (plan_needs_centers(p) && !aux.centers) return fail(BM_EINVAL, "no centring slot");
  if (p.desc.precision == BM_PREC_FP16X3 && !aux.amax) return fail(BM_EINVAL, "no max map slot");
  if (aux.centers) {
    e = launch_centers(d_img, g.C, g.H, g.W, aux.centers, s);
    if (e != hipSuccess) return hip_fail(e, "centring launch");
  }
  NormGeom ng{g.H, g.W, g.C, g.P, g.Hv, g.Wv, p.desc.precision == BM_PREC_BF16X4 ? 1 : 0};
  // 3D: one norm map (and max map) per d-plane slab, stacked by depth
  const size_t plane = (size_t)g.H * g.W, nmap = (size_t)g.Hv * g.Wv;
  const size_t tiles = (size_t)norm_tile_count(p.desc);
  for (int z = 0; z < p.Z; ++z) {
    e = launch_norm(d_img + z * plane, d_norm + z * nmap, ng, aux.centers,
                    aux.amax ? aux.amax + z * tiles : nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "norm launch");
  }
  return BM_OK;
}

bm_status run_cross_topk(const bm_plan_s& p, const float* d_img, const float* d_norm,
                         const NormAux& aux, int32_t* d_idx, float* d_dist, hipStream_t s) {
  const bm_desc& d = p.desc;
  if (d.precision == BM_PREC_FP16X3 && !aux.amax) return fail(BM_EINVAL, "no max map slot");
  if (plan_is_3d(p)) {
    const DepthGeom dg{p.Z, (p.depth_c - 1) / 2, p.depth_c, (int)norm_tile_count(d)};
    hipError_t e = launch_xcorr_depth(d.precision, d.channels, (d.patch + 1) / 2, p.kr,
                                      p.geom.NT, d_img, d_norm, aux.amax, d_idx, d_dist, p.geom,
                                      dg, s);
    if (e != hipSuccess) return hip_fail(e, "3D cross-term launch");
    return BM_OK;
  }
  hipError_t e = p.geom.fast
                     ? launch_xcorr_fast(d.precision, d.channels, (d.patch + 1) / 2, p.kr,
                                         p.geom.NT, d_img, d_norm, aux.centers, aux.amax, d_idx,
                                         d_dist, p.geom, s)
                     : launch_xcorr_f32(p.ks_bucket, p.kr, d_img, d_norm, aux.centers, d_idx,
                                        d_dist, p.geom, s);
  if (e != hipSuccess) return hip_fail(e, "cross-term launch");
  return BM_OK;
}

bm_status run_match(const bm_plan_s& p, const float* d_img, int32_t* d_idx, float* d_dist,
                    void* ws, hipStream_t s) {
  if (!ws) return fail(BM_EINVAL, "no workspace");
  float* nrm = static_cast<float*>(ws);
  const NormAux aux = plan_aux(p, ws);
  bm_status st = run_norms(p, d_img, nrm, aux, s);
  if (st != BM_OK) return st;
  return run_cross_topk(p, d_img, nrm, aux, d_idx, d_dist, s);
}

}  // namespace bmk
