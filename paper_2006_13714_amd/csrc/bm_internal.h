// Internal definitions shared by the host library and the gfx950 kernels.
#pragma once

#include <stdint.h>

namespace bmk {

// Largest contraction handled in registers: k-steps of 4 elements (fp32 matrix op) for
// one reference patch.  C * ceil(P/2)^2 <= 64, i.e. C * Pe^2 <= 256 with Pe = P rounded up
// to even.
constexpr int kMaxSteps = 64;
constexpr int kMaxK = 64;
constexpr int kRefBlock = 4;      // a wave owns a 4 x 4 block of references
constexpr int kTileN = 16;        // candidates per matrix tile (one row segment)
constexpr int kFastRS = 80;       // LDS row stride (words) of the specialised float32 kernel
constexpr int kSplitRW = 64;      // LDS row stride (words) of the specialised split kernels
// Split-form row stride by channel count: the widest strip row is 3 * 16 + 8 - 1 = 55 words;
// one channel uses exactly that (so a 4-wave block fits four workgroups per compute unit),
// more channels keep 64 so that an operand's rows stay within the reads' offset range.
constexpr int split_rw(int C) { return C == 1 ? 55 : kSplitRW; }

// Output tile of the norm pass.  Tile (tx, ty) stages the input window rows
// [16 ty, 16 ty + 16 + P - 1) x columns [64 tx, 64 tx + 64 + P - 1), clipped to the image,
// so every pixel lies in the tile (min(x / 64, ntx - 1), min(y / 16, nty - 1)).
constexpr int kNormTX = 64;
constexpr int kNormTY = 16;

// Geometry of one fused cross-term / distance / top-K launch.  All sizes in elements.
struct XcGeom {
  int H, W, C, P, Pe, s, r, K;  // r: candidate offsets before the reference (floor(Wn/2))
  int wspan;            // Wn - 1: offsets run from -r to -r + wspan on each axis
  int Hv, Wv;           // valid patch positions per axis
  int nry, nrx;         // reference grid
  int WY, WX;           // wave grid inside a workgroup (each wave: 4 x 4 references)
  int fast;             // 1: specialised kernel (one reference block per workgroup,
                        //    channel-interleaved strip rows with row stride kFastRS)
  int WS;               // specialised kernel: waves sharing one reference block
  int p1_step;          // specialised kernel: bounding sweep visits every p1_step-th row
  int nwg_y, nwg_x, nwg_total;
  int NT;               // 16-wide candidate tiles per candidate row (per wave, max)
  int SH, SW, RS, PLANE;  // pixel strip in LDS: rows, cols, row stride, channel stride
  int NH, NW, NRS;      // patch-norm strip in LDS: rows, cols, row stride
  int CAP;              // candidate buffer entries per reference
  int KS;               // real k-steps (the rest of the template's steps are zero-padded)
  int lds_strip_off, lds_norm_off, lds_buf_off, lds_bytes;
  // k-step table: LDS offset of each step relative to a patch's top-left corner, and the
  // mask of lane groups (bit g) whose element lies inside the P x P patch (odd P pads).
  int step_off[kMaxSteps];
  uint32_t step_mask[kMaxSteps];
  int prec;             // BM_PREC_* of the launch
  int metric;           // 0 Euclidean, 1 normalized cross-correlation
};

// 3D search: Z = q - d + 1 slabs (reference depths), the depth window holds depths
// z - before .. z - before + c - 1 (clipped to 0..Z-1), `tiles` max-map entries per slab.
struct DepthGeom {
  int Z, before, c, tiles;
};

// The fields of XcGeom that the specialised kernel reads (kernel argument of the
// single-image launch; per-image record of the batch launch).
struct FastGeom {
  int H, W, Hv, Wv, P, s, r, K;
  int wspan;  // window offsets -r .. -r + wspan
  int nry, nrx, nwg_x, nwg_total;
  int SH, SW, NH, CAP, p1_step;
  int lds_strip_off, lds_norm_off, lds_buf_off;
  int ntx, nty;  // tile grid of the norm pass (its per-tile max |x| map)
  int metric;    // 0 Euclidean, 1 normalized cross-correlation
};

inline FastGeom fast_geom(const XcGeom& g) {
  FastGeom f;
  f.H = g.H; f.W = g.W; f.Hv = g.Hv; f.Wv = g.Wv; f.P = g.P; f.s = g.s; f.r = g.r; f.K = g.K;
  f.wspan = g.wspan;
  f.nry = g.nry; f.nrx = g.nrx; f.nwg_x = g.nwg_x; f.nwg_total = g.nwg_total;
  f.SH = g.SH; f.SW = g.SW; f.NH = g.NH; f.CAP = g.CAP; f.p1_step = g.p1_step;
  f.lds_strip_off = g.lds_strip_off; f.lds_norm_off = g.lds_norm_off;
  f.lds_buf_off = g.lds_buf_off;
  f.ntx = (g.Wv + kNormTX - 1) / kNormTX;
  f.nty = (g.Hv + kNormTY - 1) / kNormTY;
  f.metric = g.metric;
  return f;
}

// Largest workgroup (waves) of the specialised kernel for a precision form and channel
// count: 8 waves per reference block, except the 4-channel float32 bodies, whose registers
// leave room for one wave per SIMD only.
constexpr int fast_max_waves(int prec, int C) { return (prec == 0 && C == 4) ? 4 : 8; }

// Waves per reference block the built-in rule starts from: the split forms' strips for
// 2..4 channels leave room for one workgroup per compute unit, which then needs 8 waves to
// keep two per SIMD; the other classes keep several 4-wave workgroups per compute unit.
constexpr int fast_default_waves(int prec, int C) { return (prec != 0 && C >= 2) ? 8 : 4; }

// Whether the specialised kernel stages the candidate norms in LDS with the pixel strip
// (per slab in 3D) or reads them from the norm map one tile ahead: multi-channel blocks,
// which take one or two workgroups per compute unit anyway and sweep large maps, stage
// them; one-channel blocks read the (L2-resident) map, which leaves LDS for more
// workgroups per compute unit.
constexpr bool lane_norm_strip(int C) { return C >= 2; }

// Kernel tier of the persistent batch launch for a precision form and channel count, and
// the largest workgroup (waves) of each tier: float32 1 channel (tier 3), 2..3 channels (0),
// 4 channels (1); split forms 1 channel (0), 2..4 channels (2).
constexpr int batch_tier(int prec, int C) {
  return prec == 0 ? (C == 4 ? 1 : (C == 1 ? 3 : 0)) : (C == 1 ? 0 : 2);
}
constexpr int batch_max_waves(int tier) { return tier == 2 ? 8 : 4; }
// Whether a batch tier stages the candidate norms in LDS (else it reads them from each
// image's norm map a row ahead, as the single-image kernels do): the split forms' tiers
// read the map (less LDS per block, more blocks per compute unit), the float32 tiers,
// which gain nothing from it, keep the strip.
constexpr bool batch_norm_strip(int prec, int tier) { return (void)prec, (void)tier, false; }

struct NormGeom {
  int H, W, C, P, Hv, Wv;
  int round_bf16;  // 1: norms of the values rounded to the bfloat16 hi + lo split (the
                   // norms the bfloat16 split form's distance assembly pairs with its
                   // cross term); 0: of the values themselves
};

// Group gather / aggregation geometry (one plan's image, patch and K).
struct GroupGeom {
  int C, H, W, P, Hv, Wv, K;
  long long n_ref;
  int cnt_bits;  // ceil(log2(n_ref * K + 1)): headroom of the fixed-point sums
  int s, r, nry, nrx;  // reference grid and candidate offsets before a reference
  int wspan;           // window offsets -r .. -r + wspan
  // aggregation tiles: tb x tb references per workgroup, whose windows cover a region of
  // th x tw pixels accumulated in LDS (tb = 0: no tiling)
  int tb, th, tw, ntx, nty;
};

// Per-image outputs of the norm pass that the cross-term pass reads besides the norm map:
// the centring constants (null unless centring) and the per-tile max |x - centre| map
// (null unless the float16 split form, which derives its pre-scale from it).
struct NormAux {
  float* centers;
  float* amax;
};

}  // namespace bmk
