// Plan object and the host helpers shared by the single-image, batch and serving paths.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/bm.h"
#include "bm_internal.h"

namespace bmk {

// Kernel configuration of a plan.
struct TileCfg {
  bool fast = false;  // specialised kernel (C <= 4, patch 3..8, K <= 32, span <= 48 columns)
  int wy = 1, wx = 1; // generic: wave grid per workgroup; specialised: wy waves per block
  int cap = 32;       // candidate buffer entries per reference
  int p1 = 2;         // specialised: bounding-sweep row step
};

// "fast ws=4 p1=2 cap=32" or "generic wy=2 wx=2 cap=64"; false on a malformed string.
bool parse_cfg(const char* text, TileCfg* out);
void format_cfg(const TileCfg& c, char* out, int len);

}  // namespace bmk

struct bm_plan_s {
  bm_desc desc;
  int device = 0;
  bmk::XcGeom geom;
  bmk::TileCfg cfg;     // configuration in use
  int ks_bucket = 0;    // compiled step count of the generic kernel
  int kr = 1;           // list registers per reference (K <= 16 * kr)
  void* ws = nullptr;   // plan-owned workspace (norm map)
  int64_t ws_bytes = 0;
  int cfg_source = 0;   // 0 built-in rule, 1 autotuner table, 2 BM_CFG override
  // 3D search: `desc` is then the 2D problem of one d-plane slab (channels = d) and these
  // hold the volume's planes q, the depth window c and the slab count Z = q - d + 1
  int depth_q = 0, depth_c = 0, Z = 1;
};

inline bool plan_is_3d(const bm_plan_s& p) { return p.depth_c > 0; }

namespace bmk {

bm_status fail(bm_status s, const char* fmt, ...);
bm_status hip_fail(hipError_t e, const char* what);
const char* last_error();
bm_status validate_desc(const bm_desc* d);
// fast_norm_strip: the specialised layout with an LDS norm strip (non-local means, the 3D
// kernels and the float32 batch tiers)
void fill_geom(const bm_desc& d, int wy, int wx, int cap, bool fast, XcGeom& g,
               bool fast_norm_strip = false);

bool fast_eligible(const bm_desc& d);
// The 2D problem of one slab of a 3D descriptor (channels = patch_depth); 2D: d itself.
bm_desc slab_desc(const bm_desc& d);
bm_status choose_config(const bm_desc& d, int max_lds, bm_plan_s* p);
bm_status apply_config(const bm_desc& d, const TileCfg& c, int max_lds, bm_plan_s* p);
int64_t plan_workspace_bytes(const bm_plan_s& p);
// Workspace of a descriptor (norm map, centring slot, per-tile max map); the auxiliary
// slots sit in a region of 256 + align256(norm_tile_count * 4) bytes after the norm map.
int64_t norm_tile_count(const bm_desc& d);
int64_t desc_workspace_bytes(const bm_desc& d);
bool plan_needs_centers(const bm_plan_s& p);
// auxiliary outputs of the norm pass inside an auxiliary region (aux_at) or a plan
// workspace (plan_aux); unused slots are null
NormAux aux_at(const bm_plan_s& p, void* slot);
NormAux plan_aux(const bm_plan_s& p, void* ws);
// norms (and, when the plan centres, the centring constants first)
bm_status run_norms(const bm_plan_s& p, const float* d_img, float* d_norm, const NormAux& aux,
                    hipStream_t s);
bm_status run_cross_topk(const bm_plan_s& p, const float* d_img, const float* d_norm,
                         const NormAux& aux, int32_t* d_idx, float* d_dist, hipStream_t s);
bm_status run_match(const bm_plan_s& p, const float* d_img, int32_t* d_idx, float* d_dist,
                    void* ws, hipStream_t s);

}  // namespace bmk
