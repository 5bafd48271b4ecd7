// Host side of libbm.so: argument checks, plan geometry, workspace, kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/bm.h"
#include "bm_internal.h"
#include "plan.h"

namespace bmk {

static thread_local std::string g_err;

bm_status fail(bm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

bm_status hip_fail(hipError_t e, const char* what) {
  return fail(BM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

bm_status validate_desc(const bm_desc* d) {
  if (!d) return fail(BM_EINVAL, "desc is NULL");
  if (d->height < 1 || d->width < 1) return fail(BM_EINVAL, "height/width must be >= 1");
  const bool d3 = d->window_depth != 0 || d->patch_depth != 0;
  if (d3) {
    if (d->window_depth < 1) return fail(BM_EINVAL, "window_depth must be >= 1 (0 for 2D)");
    if (d->channels < 1 || d->channels > 65536)
      return fail(BM_EINVAL, "3D: channels (volume planes) must be in [1, 65536]");
    if (d->patch_depth < 1 || d->patch_depth > d->channels)
      return fail(BM_EINVAL, "patch_depth must be in [1, channels]");
    if (d->patch_depth > 4) return fail(BM_ENOTSUP, "3D search takes patch_depth <= 4");
    if (d->flags) return fail(BM_ENOTSUP, "3D search takes no flags");
  } else if (d->channels < 1 || d->channels > 8) {
    return fail(BM_EINVAL, "channels must be in [1, 8]");
  }
  if (d->patch < 1 || d->patch > 16) return fail(BM_EINVAL, "patch must be in [1, 16]");
  if (d->patch > d->height || d->patch > d->width)
    return fail(BM_EINVAL, "patch %d larger than the image", d->patch);
  if (d->stride < 1) return fail(BM_EINVAL, "stride must be >= 1");
  if (d->window < 1) return fail(BM_EINVAL, "window must be >= 1");
  if (d->k < 1 || d->k > kMaxK) return fail(BM_EINVAL, "k must be in [1, %d]", kMaxK);
  if (d->precision < BM_PREC_FP32 || d->precision > BM_PREC_FP16X3)
    return fail(BM_EINVAL, "unknown precision %d", d->precision);
  if ((int64_t)d->height * d->width * d->channels >= (int64_t)1 << 31)
    return fail(BM_EINVAL, "image too large for 32-bit indexing");
  if (d->flags & ~(BM_FLAG_CENTER | BM_FLAG_NCC))
    return fail(BM_EINVAL, "unknown flag bits 0x%x", d->flags);
  if ((d->flags & BM_FLAG_CENTER) && (d->flags & BM_FLAG_NCC))
    return fail(BM_EINVAL, "centring changes the normalized cross-correlation");
  const int pe = d->patch + (d->patch & 1);
  const int pc = d3 ? d->patch_depth : d->channels;
  if (pc * (pe / 2) * (pe / 2) > kMaxSteps)
    return fail(BM_ENOTSUP, "channels * ceil(patch/2)^2 = %d exceeds %d", pc * (pe / 2) * (pe / 2),
                kMaxSteps);
  return BM_OK;
}

// Fill the launch geometry.  Generic kernel: a workgroup of wy x wx waves, one 4 x 4
// reference block per wave, channel-plane strip.  Specialised kernel (`fast`): one
// reference block per workgroup shared by wy waves (wx unused), channel-interleaved strip
// rows of kFastRS floats.  `cap`: candidate buffer entries per reference.
void fill_geom(const bm_desc& d, int wy, int wx, int cap, bool fast, XcGeom& g,
               bool fast_norm_strip) {
  memset(&g, 0, sizeof(g));
  g.H = d.height;
  g.W = d.width;
  g.C = d.channels;
  g.P = d.patch;
  g.Pe = d.patch + (d.patch & 1);
  g.s = d.stride;
  g.r = d.window / 2;  // even windows: one more offset before the reference than after
  g.wspan = d.window - 1;
  g.K = d.k;
  g.Hv = d.height - d.patch + 1;
  g.Wv = d.width - d.patch + 1;
  g.nry = (d.height - d.patch) / d.stride + 1;
  g.nrx = (d.width - d.patch) / d.stride + 1;
  g.fast = fast ? 1 : 0;
  g.p1_step = 2;
  if (fast) {
    wx = 1;
    g.WS = wy;
  }
  g.WY = wy;
  g.WX = wx;
  const int rows_per_wg = fast ? kRefBlock : kRefBlock * wy;
  const int cols_per_wg = fast ? kRefBlock : kRefBlock * wx;
  g.nwg_y = (g.nry + rows_per_wg - 1) / rows_per_wg;
  g.nwg_x = (g.nrx + cols_per_wg - 1) / cols_per_wg;
  g.nwg_total = g.nwg_y * g.nwg_x;
  const int span = 3 * g.s + g.wspan + 1;  // candidate positions across a 4-reference block
  g.NT = (span + kTileN - 1) / kTileN;
  g.NH = (fast ? 0 : 4 * g.s * (wy - 1)) + span;
  g.NW = (fast ? 0 : 4 * g.s * (wx - 1)) + kTileN * g.NT;
  g.NRS = g.NW;
  // pixels beyond the patch that the operand reads still touch: the split layout reads whole
  // 4-row x 8-column blocks (zero weight outside the patch) and they must be staged values
  const bool split = fast && d.precision != BM_PREC_FP32;
  const int prow = split ? 4 * ((g.Pe + 3) / 4) : g.Pe;
  const int pcol = split ? 8 * ((g.Pe + 7) / 8) : g.Pe;
  g.SH = g.NH + prow - 1;
  g.SW = g.NW + pcol - 1;
  g.prec = d.precision;
  g.metric = (d.flags & BM_FLAG_NCC) ? 1 : 0;
  g.RS = fast ? (d.precision == BM_PREC_FP32 ? kFastRS : split_rw(d.channels)) : g.SW;
  g.PLANE = g.SH * g.RS;
  g.CAP = cap;
  const int h2 = g.Pe / 2;
  g.KS = g.C * h2 * h2;
  for (int t = 0; t < g.KS; ++t) {
    const int c = t / (h2 * h2);
    const int rem = t - c * h2 * h2;
    const int l2 = rem / h2;
    const int m2 = rem - l2 * h2;
    g.step_off[t] = c * g.PLANE + 2 * l2 * g.RS + 2 * m2;
    uint32_t mask = 0;
    for (int gp = 0; gp < 4; ++gp) {
      const int l = 2 * l2 + (gp >> 1);
      const int m = 2 * m2 + (gp & 1);
      if (l < g.P && m < g.P) mask |= 1u << gp;
    }
    g.step_mask[t] = mask;
  }
  const int nw = wy * wx;
  const int rows_per_img_row = (fast && d.precision != BM_PREC_FP32) ? 2 * g.C : g.C;
  const int strip_bytes = rows_per_img_row * g.SH * g.RS * 4;
  // the specialised BM kernels read candidate norms from the norm map (L2); the generic
  // kernel and non-local means stage them in LDS
  const int norm_bytes =
      (fast && !fast_norm_strip && !lane_norm_strip(d.channels)) ? 0 : g.NH * g.NRS * 4;
  int buf_bytes = nw * 16 * cap * 8;
  if (fast) {
    buf_bytes = nw * (16 * cap * 8 + 64);  // per wave: cap entries per reference + counters
    const int kr = d.k <= 16 ? 1 : 2;
    const int tl_bytes = nw * 4 * (2 * kr) * 64 * 4 + 4 * 64 * 4;  // bounding lists + bounds
    const int list_bytes = nw * 4 * kr * 64 * 8;        // final-list exchange
    buf_bytes = buf_bytes > tl_bytes ? buf_bytes : tl_bytes;
    buf_bytes = buf_bytes > list_bytes ? buf_bytes : list_bytes;
  }
  g.lds_strip_off = 0;
  g.lds_norm_off = (strip_bytes + 15) & ~15;
  g.lds_buf_off = (g.lds_norm_off + norm_bytes + 15) & ~15;
  g.lds_bytes = g.lds_buf_off + buf_bytes;
}

}  // namespace bmk

namespace bmk {
hipError_t prepare_xcorr_depth(int prec, int c, int h2, int kr, int nt, int lds_bytes);
hipError_t launch_nlm(const float* img, const float* nrm, float* patch, float* theta,
                      const XcGeom& g, float b, hipStream_t stream);
hipError_t launch_gather(const float* img, const int32_t* idx, float* groups, const GroupGeom& g,
                         hipStream_t s);
long long aggregate_workspace_bytes(const GroupGeom& g);
void aggregate_tiling(GroupGeom& g);
hipError_t launch_aggregate(const float* groups, const int32_t* idx, float* out, void* ws,
                            const GroupGeom& g, hipStream_t s);

static GroupGeom group_geom(const bm_plan_s& p) {
  GroupGeom g;
  g.C = p.geom.C;
  g.H = p.geom.H;
  g.W = p.geom.W;
  g.P = p.geom.P;
  g.Hv = p.geom.Hv;
  g.Wv = p.geom.Wv;
  g.K = p.geom.K;
  g.n_ref = (long long)p.geom.nry * p.geom.nrx;
  const long long n = g.n_ref * g.K + 1;
  int bits = 0;
  while ((1ll << bits) < n) ++bits;
  g.cnt_bits = bits;
  g.s = p.geom.s;
  g.r = p.geom.r;
  g.wspan = p.geom.wspan;
  g.nry = p.geom.nry;
  g.nrx = p.geom.nrx;
  aggregate_tiling(g);
  return g;
}
}  // namespace bmk

using namespace bmk;

extern "C" {

const char* bm_status_str(bm_status s) {
  switch (s) {
    case BM_OK: return "BM_OK";
    case BM_EINVAL: return "BM_EINVAL";
    case BM_ENOMEM: return "BM_ENOMEM";
    case BM_EDEVICE: return "BM_EDEVICE";
    case BM_EAGAIN: return "BM_EAGAIN";
    case BM_EBUSY: return "BM_EBUSY";
    case BM_ENOTFOUND: return "BM_ENOTFOUND";
    case BM_ECANCELED: return "BM_ECANCELED";
    case BM_ENOTSUP: return "BM_ENOTSUP";
  }
  return "BM_UNKNOWN";
}

const char* bm_last_error(void) { return last_error(); }

bm_status bm_plan(const bm_desc* desc, bm_plan_t* out) {
  if (!out) return fail(BM_EINVAL, "out is NULL");
  *out = nullptr;
  bm_status st = validate_desc(desc);
  if (st != BM_OK) return st;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  int max_lds = 0;
  e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  bm_plan_s* p = new (std::nothrow) bm_plan_s();
  if (!p) return fail(BM_ENOMEM, "host allocation failed");
  p->desc = slab_desc(*desc);
  p->device = dev;
  if (desc->window_depth > 0) {
    p->depth_q = desc->channels;
    p->depth_c = desc->window_depth;
    p->Z = desc->channels - desc->patch_depth + 1;
  }
  st = choose_config(p->desc, max_lds, p);
  if (st == BM_OK && plan_is_3d(*p)) {
    if (!p->geom.fast) {
      st = fail(BM_ENOTSUP, "3D search needs patch 3..8 (5..8 split), K <= 32 and "
                            "17 <= 3*stride + window <= 48");
    } else {
      // the 3D kernel stages candidate norms in LDS with each slab's strip; the 2D
      // configuration was sized without that strip, so if it no longer fits, take the
      // largest block (waves, then buffer capacity) at or below it that does
      XcGeom g3;
      fill_geom(p->desc, p->cfg.wy, 1, p->cfg.cap, true, g3);
      if (g3.lds_bytes > max_lds) {
        bool found = false;
        for (int ws = p->cfg.wy; ws >= 1 && !found; ws = ws > 1 ? ws / 2 : 0)
          for (int cap : {p->cfg.cap, 48, 32}) {
            if (cap > p->cfg.cap || (ws == p->cfg.wy && cap == p->cfg.cap)) continue;
            fill_geom(p->desc, ws, 1, cap, true, g3);
            if (g3.lds_bytes <= max_lds) {
              p->cfg.wy = ws;
              p->cfg.cap = cap;
              found = true;
              break;
            }
          }
        if (!found) fill_geom(p->desc, p->cfg.wy, 1, p->cfg.cap, true, g3);
      }
      g3.p1_step = p->cfg.p1;
      if (g3.lds_bytes > max_lds) {
        st = fail(BM_ENOTSUP, "3D tile needs %d bytes of LDS (limit %d)", g3.lds_bytes, max_lds);
      } else {
        p->geom = g3;
        e = prepare_xcorr_depth(p->desc.precision, p->desc.channels, (p->desc.patch + 1) / 2,
                                p->kr, p->geom.NT, p->geom.lds_bytes);
        if (e != hipSuccess) st = hip_fail(e, "hipFuncSetAttribute");
      }
    }
    if (st == BM_OK && (int64_t)p->geom.nwg_total * p->Z >= ((int64_t)1 << 31))
      st = fail(BM_EINVAL, "3D problem too large for one launch");
  }
  if (st != BM_OK) {
    delete p;
    return st;
  }
  p->ws_bytes = plan_workspace_bytes(*p);
  if (p->ws_bytes > 0) {
    e = hipMalloc(&p->ws, p->ws_bytes);
    if (e != hipSuccess) {
      delete p;
      (void)hipGetLastError();
      return fail(BM_ENOMEM, "workspace hipMalloc(%lld): %s", (long long)p->ws_bytes,
                  hipGetErrorString(e));
    }
  }
  *out = p;
  return BM_OK;
}

bm_status bm_plan_info(bm_plan_t plan, int64_t* n_ref, int64_t* workspace_bytes) {
  if (!plan) return fail(BM_EINVAL, "plan is NULL");
  if (n_ref) *n_ref = (int64_t)plan->Z * plan->geom.nry * plan->geom.nrx;
  if (workspace_bytes) *workspace_bytes = plan->ws_bytes;
  return BM_OK;
}

bm_status bm_plan_destroy(bm_plan_t plan) {
  if (!plan) return fail(BM_EINVAL, "plan is NULL");
  if (plan->ws) (void)hipFree(plan->ws);
  delete plan;
  return BM_OK;
}

bm_status bm_norms(bm_plan_t plan, const float* d_img, float* d_norm, void* stream) {
  if (!plan) return fail(BM_EINVAL, "plan is NULL");
  if (!d_img || !d_norm) return fail(BM_EINVAL, "NULL device pointer");
  return run_norms(*plan, d_img, d_norm, plan_aux(*plan, plan->ws), (hipStream_t)stream);
}

bm_status bm_cross_topk(bm_plan_t plan, const float* d_img, const float* d_norm,
                        int32_t* d_idx, float* d_dist, void* stream) {
  if (!plan) return fail(BM_EINVAL, "plan is NULL");
  if (!d_img || !d_norm || !d_idx || !d_dist) return fail(BM_EINVAL, "NULL device pointer");
  return run_cross_topk(*plan, d_img, d_norm, plan_aux(*plan, plan->ws), d_idx, d_dist,
                        (hipStream_t)stream);
}

bm_status bm_gather(bm_plan_t plan, const float* d_img, const int32_t* d_idx, float* d_groups,
                    void* stream) {
  if (!plan) return fail(BM_EINVAL, "plan is NULL");
  if (plan_is_3d(*plan)) return fail(BM_ENOTSUP, "not available for a 3D plan");
  if (!d_img || !d_idx || !d_groups) return fail(BM_EINVAL, "NULL device pointer");
  hipError_t e = launch_gather(d_img, d_idx, d_groups, group_geom(*plan), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gather launch");
  return BM_OK;
}

bm_status bm_aggregate_workspace(bm_plan_t plan, int64_t* bytes) {
  if (!plan || !bytes) return fail(BM_EINVAL, "NULL argument");
  if (plan_is_3d(*plan)) return fail(BM_ENOTSUP, "not available for a 3D plan");
  *bytes = aggregate_workspace_bytes(group_geom(*plan));
  return BM_OK;
}

bm_status bm_aggregate(bm_plan_t plan, const float* d_groups, const int32_t* d_idx, float* d_out,
                       void* d_workspace, void* stream) {
  if (!plan) return fail(BM_EINVAL, "plan is NULL");
  if (plan_is_3d(*plan)) return fail(BM_ENOTSUP, "not available for a 3D plan");
  if (!d_groups || !d_idx || !d_out) return fail(BM_EINVAL, "NULL device pointer");
  const GroupGeom g = group_geom(*plan);
  hipStream_t s = (hipStream_t)stream;
  void* ws = d_workspace;
  bool own = false;
  if (!ws) {
    if (hipMalloc(&ws, aggregate_workspace_bytes(g)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(BM_ENOMEM, "aggregation workspace");
    }
    own = true;
  }
  hipError_t e = launch_aggregate(d_groups, d_idx, d_out, ws, g, s);
  bm_status st = e == hipSuccess ? BM_OK : hip_fail(e, "aggregation launch");
  if (own) {
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(ws);
    if (st == BM_OK && e2 != hipSuccess) st = hip_fail(e2, "hipStreamSynchronize");
  }
  return st;
}

bm_status bm_nlm(bm_plan_t plan, const float* d_img, float b, float* d_patch, float* d_theta,
                 void* d_workspace, void* stream) {
  if (!plan) return fail(BM_EINVAL, "plan is NULL");
  if (plan_is_3d(*plan)) return fail(BM_ENOTSUP, "not available for a 3D plan");
  if (!d_img || !d_patch) return fail(BM_EINVAL, "NULL device pointer");
  if (!(b > 0.f) || !std::isfinite(b) || !(b * b > 0.f) || !std::isfinite(b * b))
    return fail(BM_EINVAL, "b must be finite and > 0");
  const bm_desc& d = plan->desc;
  if (!plan->geom.fast || d.precision != BM_PREC_FP32 || d.flags != 0)
    return fail(BM_ENOTSUP, "NLM needs a float32 plan without flags inside the specialised "
                            "kernel's envelope");
  void* ws = d_workspace ? d_workspace : plan->ws;
  if (!ws) return fail(BM_EINVAL, "no workspace");
  hipStream_t s = (hipStream_t)stream;
  float* nrm = static_cast<float*>(ws);
  bm_status st = run_norms(*plan, d_img, nrm, plan_aux(*plan, ws), s);
  if (st != BM_OK) return st;
  XcGeom g;
  fill_geom(d, plan->cfg.wy < 4 ? plan->cfg.wy : 4, 1, plan->cfg.cap, true, g, true);
  hipError_t e = launch_nlm(d_img, nrm, d_patch, d_theta, g, b, s);
  if (e != hipSuccess) return hip_fail(e, "NLM launch");
  return BM_OK;
}

bm_status bm_match(bm_plan_t plan, const float* d_img, int32_t* d_idx, float* d_dist,
                   void* d_workspace, void* stream) {
  if (!plan) return fail(BM_EINVAL, "plan is NULL");
  if (!d_img || !d_idx || !d_dist) return fail(BM_EINVAL, "NULL device pointer");
  void* ws = d_workspace ? d_workspace : plan->ws;
  hipStream_t s = (hipStream_t)stream;
  return run_match(*plan, d_img, d_idx, d_dist, ws, s);
}

}  // extern "C"
