// Fused window-masked cross-correlation + distance assembly + top-K for gfx950, with one
// reference per lane (specialised for C <= 4 channels, patch side 3..8, K <= 32 and a
// candidate span of NT * 16 columns per 4 x 4 reference block).
//
// Per reference X_i and in-window candidate X_j it evaluates Lemma 2 (Sec. III-B),
//     d_ij = ||X_i||^2 + ||X_j||^2 - 2 <X_i, X_j>,
// with <X_i, X_j> the window-restricted Self-Convolution of Eq. (eq:selfConv) (footnote to
// Eq. (eq:unifySelfConv)) summed over channels (Sec. IV, S(.)) on the matrix cores, and
// keeps the K smallest (Theorem 1, Euclidean branch).  The normalized cross-correlation
// metric (Eq. equ:cor, Lemma 1) ranks by <X_i, X_j> / ||X_j|| instead.
//
//  * One workgroup = one 4 x 4 block of references, shared by S waves; the pixel strip
//    covering the block's windows is staged in LDS once (per slab in 3D), and the
//    candidate norms are read from the norm map (L2-resident) one tile ahead.  Candidate rows are dealt round-robin to the waves, so each wave
//    meets the candidates of every reference in increasing j.
//  * Matrix tile: 16 candidates (a 16-wide row segment) x 16 references, the candidates
//    as the row operand: lane (g, p) holds reference p (block position (p / 4, p % 4))
//    against candidates 4 g .. 4 g + 3 of the segment.  Each lane therefore owns one
//    reference: its threshold, window mask and admission state are per-lane values, not
//    per-group arrays.
//  * Score s = <X_i, X_j> - ||X_j||^2 / 2 (in the float16 form scaled by 2^2k): the
//    float32 chain accumulates onto -||X_j||^2 / 2, the split forms add it to their chain
//    with one fused multiply-add, so admission is one comparison s > thr per pair.  The distance d = ||X_i||^2 - 2 s (one fused multiply-add) is
//    formed only for admitted pairs and in the bounding sweep, bit for bit the same in
//    both.  thr = (||X_i||^2 - th) / 2 rounded down, th the reference's admission bound,
//    so every pair with d < th passes (a few more may; the merge orders them exactly).
//    Window columns outside the reference's range get thr = +inf; window rows are a
//    per-row lane mask.
//  * Selection: a bounding sweep over the rows inside every reference's window (every
//    p1-th row of each wave) keeps each lane's 2 KR smallest d; the K-th smallest of a
//    reference's lane lists over its four lanes and all waves bounds its K-th distance
//    from above (the values come from distinct candidates).  The selecting sweep appends
//    admitted (d, j) to the lane's own LDS buffer (no cross-lane compaction); full buffers
//    are merged, one reference per 16-lane group and round, into sorted per-reference
//    lists by the DPP bitonic networks of topk.h, and the lists' K-th distances tighten
//    the thresholds.  The waves' lists are merged exactly at the end.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>
#include <stdint.h>

#include "bm_internal.h"
#include "contract.h"
#include "select.h"
#include "topk.h"
#include "xcorr_common.h"

namespace bmk {

// Largest float strictly below x (x itself for -inf and NaN; -0 and +0 give the negative
// denormal).
__device__ __forceinline__ float next_down(float x) {
  const int b = __float_as_int(x);
  if (!(x > -INFINITY)) return x;
  if (x == 0.f) return __int_as_float(0x80000001);
  return __int_as_float(x > 0.f ? b - 1 : b + 1);
}

template <int KR>
struct LaneSelect {
  static constexpr int TL = 2 * KR;
  // round R: the 16-lane group g holds the sorted list of reference 4 g + R
  float Ld[4][KR];
  int Lj[4][KR];
  float tl[TL];  // bounding sweep: this lane's smallest distances
  float th;      // this lane's reference: strict admission bound on d
};

// Threshold on the score s (in-window columns): s > thr admits every pair with
// base - 2 s < th (rounding of base - th is taken downwards).
__device__ __forceinline__ float score_threshold(float base, float th, bool col_ok) {
  return col_ok ? 0.5f * next_down(base - th) : INFINITY;
}

template <class CT, int C, int KR, int NT, bool D3 = false>
__device__ __forceinline__ void lane_block(const float* __restrict__ img,
                                           const float* __restrict__ nrm,
                                           const float* __restrict__ centers,
                                           const float* __restrict__ amax,
                                           int* __restrict__ out_idx,
                                           float* __restrict__ out_dist, const FastGeom& g,
                                           int blk, unsigned char* lds,
                                           const DepthWin* dw = nullptr) {
  constexpr int CRS = CT::CRS;
  constexpr int NB = CT::NB;
  using BReg = typename CT::BReg;
  constexpr int NA = CT::NA;
  constexpr int TL = LaneSelect<KR>::TL;
  static_assert(NT >= 1 && NT <= 4, "tile columns");
  constexpr bool NSTRIP = lane_norm_strip(C);
  constexpr int NW = kTileN * NT;  // norm strip row length
  uint32_t* strip = reinterpret_cast<uint32_t*>(lds + g.lds_strip_off);
  float* nstrip = reinterpret_cast<float*>(lds + g.lds_norm_off);  // NSTRIP only
  unsigned char* bufs = lds + g.lds_buf_off;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int S = blockDim.x >> 6;
  // this wave's candidate buffers: CAP entries per reference, then 16 entry counters
  const int CAP = g.CAP;
  Entry* wbuf = reinterpret_cast<Entry*>(bufs + (size_t)wave * (16 * CAP * 8 + 64));
  int* wcnt = reinterpret_cast<int*>(wbuf + 16 * CAP);

  const int by = blk / g.nwg_x;
  const int bx = blk - by * g.nwg_x;
  const int s = g.s, r = g.r, wsp = g.wspan;
  const int RYw = kRefBlock * by, RXw = kRefBlock * bx;
  const int ryw = s * RYw, rxw = s * RXw;
  const int SY0 = ryw - r, SX0 = rxw - r;

  // centring constants; the float16 form's power-of-two pre-scale 2^k (largest staged
  // magnitude below 2^14); scores and distances carry 2^2k, removed at the output
  float center[8];
  float scale = 1.f, sq = 1.f, isq = 1.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) center[c] = (centers && c < C) ? centers[c] : 0.f;
  if constexpr (CT::kScaled) {
    const int y0 = max(SY0, 0), y1 = min(SY0 + g.SH, g.H) - 1;
    const int x0 = max(SX0, 0), x1 = min(SX0 + g.SW, g.W) - 1;
    float m;
    if constexpr (D3)
      m = strip_absmax(dw->amax + (size_t)dw->z0 * dw->tiles, g, y0, y1, x0, x1, lane,
                       dw->z1 - dw->z0 + 1, dw->tiles);
    else
      m = strip_absmax(amax, g, y0, y1, x0, x1, lane);
    const int e = m > 0.f ? ilogbf(m) + 1 : 0;
    const int k = max(-60, min(60, 14 - e));
    scale = ldexpf(1.f, k);
    sq = ldexpf(1.f, 2 * k);
    isq = ldexpf(1.f, -2 * k);
  }
  const bool ncc = g.metric != 0;
  const float hsq = -0.5f * sq;  // the score's norm term: -||X_j||^2 2^2k / 2

  // ---- stage the strip (and with NSTRIP the raw candidate norms, 0 outside the valid
  //      positions); otherwise candidate norms come from the norm map of the slab being
  //      swept (`nm_cur`)
  const float* nm_cur = nrm;
  const int nm_last = g.Hv * g.Wv - 1;
  auto stage_slab = [&](const float* __restrict__ im, const float* __restrict__ nm)
                        __attribute__((always_inline)) {
    CT::stage(strip, im, g, SY0, SX0, wave, S, lane, center, scale);
    if constexpr (NSTRIP) {
      for (int y0 = wave; y0 < g.NH; y0 += 4 * S) {
        for (int x = lane; x < NW; x += 64) {
          const int qx = SX0 + x;
          const bool xok = (qx >= 0) & (qx < g.Wv);
          float nv[4];
          bool ok[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int qy = SY0 + y0 + u * S;
            ok[u] = (y0 + u * S < g.NH) & (qy >= 0) & (qy < g.Hv) & xok;
            nv[u] = nm[ok[u] ? (size_t)qy * g.Wv + qx : 0];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (y0 + u * S < g.NH) nstrip[(y0 + u * S) * NW + x] = ok[u] ? nv[u] : 0.f;
        }
      }
    } else {
      (void)nm;
    }
  };
  stage_slab(img, nrm);
  __syncthreads();

  const int a_max = min(3, g.nry - 1 - RYw);
  const int b_max = min(3, g.nrx - 1 - RXw);
  const int P = g.P, W = g.W;
  const int p16 = lane & 15;  // this lane's reference
  const int gp = lane >> 4;   // this lane's quarter of each candidate segment
  const int ra = p16 >> 2, rb = p16 & 3;
  const int lane_off = CT::lane_off(gp);

  // ---- operand A: reference p16 (block position (ra, rb))
  typename CT::AReg A[NA];
  const int plane = CT::plane_off(g);
  CT::load_a(A, strip, (s * ra + r) * CRS + (s * rb + r) + lane_off, gp, P, plane);

  // ---- this lane's reference: norm, validity, column masks
  const bool ref_ok = (ra <= a_max) & (rb <= b_max);
  const float nref = nrm[(size_t)min(ryw + s * ra, g.Hv - 1) * g.Wv + min(rxw + s * rb, g.Wv - 1)];
  const float base = ncc ? 0.f : nref * sq;  // d = base - 2 s
  const int xs = rxw - r;  // first candidate column of the block
  bool colok[NT][4];
#pragma unroll
  for (int tx = 0; tx < NT; ++tx)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int cx = kTileN * tx + 4 * gp + k;
      colok[tx][k] = ref_ok & ((unsigned)(cx - s * rb) <= (unsigned)wsp) &
                     ((unsigned)(xs + cx) < (unsigned)g.Wv);
    }

  LaneSelect<KR> sel;
#pragma unroll
  for (int R = 0; R < 4; ++R)
#pragma unroll
    for (int q = 0; q < KR; ++q) {
      sel.Ld[R][q] = INFINITY;
      sel.Lj[R][q] = kNoIndex;
    }
#pragma unroll
  for (int i = 0; i < TL; ++i) sel.tl[i] = INFINITY;
  sel.th = ref_ok ? INFINITY : -INFINITY;

  const int qy_lo = max(0, ryw - r);
  const int qy_hi = min(g.Hv - 1, ryw + s * a_max - r + wsp);
  const int bl = lane_off + p16;  // operand B lane offset within a strip row

  int jofs = 0;  // candidate index of (slab, row 0, column 0)
  auto over_slabs = [&](auto&& body) __attribute__((always_inline)) {
    if constexpr (!D3) {
      body();
    } else {
      for (int zc = dw->z0; zc <= dw->z1; ++zc) {
        __syncthreads();  // every wave is done with the strip
        stage_slab(dw->vol + (size_t)zc * g.H * g.W, dw->nrm + (size_t)zc * g.Hv * g.Wv);
        __syncthreads();
        nm_cur = dw->nrm + (size_t)zc * g.Hv * g.Wv;
        jofs = zc * g.H * g.W;
        body();
      }
    }
  };

  // Lanes whose reference row has candidate row qy inside its window (a lane mask).
  const int row0 = ryw + s * ra - r;
  auto row_ok = [&](int qy) __attribute__((always_inline)) {
    return (unsigned)(qy - row0) <= (unsigned)wsp;
  };

  // One sweep over rows first, first + stride, ... <= last of this wave.  The previous
  // tile's scores go to `arith(sc, tx, qy)` (branch-free, interleaved with this tile's
  // matrix ops) and its result to `post(res, tx, qy)` (may branch) after them.
  // BOUND: the bounding sweep's shorter chain (contract.h), whose scores take the inflated
  // norm term `hs`.
  auto sweep = [&](auto BOUNDc, float hs, int first, int stride, int last, auto&& arith,
                   auto&& post) __attribute__((always_inline)) {
    constexpr bool BOUND = decltype(BOUNDc)::value;
    if (first > last) return;
    const int nrows = (last - first) / stride + 1;
    BReg bufA[NB], bufB[NB];
    constexpr int NAC = CT::NACC_T;
    f4 accp[NAC];
#pragma unroll
    for (int q = 0; q < NAC; ++q) accp[q] = f4{0.f, 0.f, 0.f, 0.f};
    f4 p_n = {0.f, 0.f, 0.f, 0.f};  // the previous tile's norm-strip values
    int p_tx = 0, p_qy = first;
    bool have_prev = false;
    int qy = first;
    CT::load_b(bufA, strip, (qy - SY0) * CRS + bl, plane);
    // raw candidate norms of a tile: candidates 4 gp .. 4 gp + 3 of its segment.  Columns
    // outside the image read neighbouring map entries (or, at the map's two ends, clamped
    // ones): finite values the column masks exclude.
    auto load_norms = [&](int row, int tx) __attribute__((always_inline)) {
      if constexpr (NSTRIP)
        return *reinterpret_cast<const f4*>(nstrip + (row - SY0) * NW + kTileN * tx + 4 * gp);
      const int lin = row * g.Wv + xs + kTileN * tx + 4 * gp;
      f4 v;
      if ((lin >= 0) & (lin <= nm_last - 3)) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = nm_cur[lin + k];
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = nm_cur[min(max(lin + k, 0), nm_last)];
      }
      return v;
    };
    f4 ninit = load_norms(qy, 0);
    // scores of the previous tile: Euclidean <X_i, X_j> - ||X_j||^2 / 2 (float32: started
    // from the norm term in the chain; split forms: added here, one fused multiply-add),
    // NCC <X_i, X_j> / ||X_j|| (the hardware reciprocal square root, within an ulp or two:
    // far inside the NCC tolerance; equal outputs of distinct keys are re-sorted by index
    // at the end)
    auto scores = [&]() __attribute__((always_inline)) {
      const f4 c = CT::combine(accp);
      f4 o;
      if (ncc) {
        // the 16 lanes of a row share candidates 4 g .. 4 g + 3: lane k < 4 of the row forms
        // candidate k's factor (every lane computes one), and a row broadcast hands it on
        const int own = p16 & 3;
        const float nk = own == 0 ? p_n[0] : (own == 1 ? p_n[1] : (own == 2 ? p_n[2] : p_n[3]));
        const float rk = nk > 0.f ? isq * rsqrtf(nk) : 0.f;
        const int ri = __float_as_int(rk);
        o[0] = c[0] * __int_as_float(__builtin_amdgcn_update_dpp(0, ri, 0x150, 0xF, 0xF, false));
        o[1] = c[1] * __int_as_float(__builtin_amdgcn_update_dpp(0, ri, 0x151, 0xF, 0xF, false));
        o[2] = c[2] * __int_as_float(__builtin_amdgcn_update_dpp(0, ri, 0x152, 0xF, 0xF, false));
        o[3] = c[3] * __int_as_float(__builtin_amdgcn_update_dpp(0, ri, 0x153, 0xF, 0xF, false));
      } else if constexpr (CT::kInitInChain) {
        o = c;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = fmaf(hs, p_n[k], c[k]);
      }
      return o;
    };
    auto tile = [&](auto TXc, BReg (&cur)[NB], BReg (&nxt)[NB]) __attribute__((always_inline)) {
      constexpr int TX = decltype(TXc)::value;
      __builtin_amdgcn_sched_barrier(0);
      const int nqy = (TX + 1 < NT) ? qy : min(qy + stride, last);
      const int ntx = (TX + 1 < NT) ? TX + 1 : 0;
      const int nrb = (nqy - SY0) * CRS + bl + kTileN * ntx;
      f4 init = {0.f, 0.f, 0.f, 0.f};
      if constexpr (CT::kInitInChain) {
        if (!ncc) {
#pragma unroll
          for (int k = 0; k < 4; ++k) init[k] = hs * ninit[k];
        }
      }
      f4 acc[NAC];
      // split forms: the waves issuing a tile's matrix chain (with the previous tile's score
      // arithmetic interleaved) go first, ahead of waves in their buffer writes, merges or
      // staging, so the matrix pipe is fed while those wait (2% on one-channel blocks)
      if constexpr (CT::kSplit) __builtin_amdgcn_s_setprio(1);
      CT::template chain_t<BOUND>(A, cur, nxt, strip, nrb, plane, init, acc);
      const f4 ncur = ninit;
      ninit = load_norms(nqy, ntx);
      const auto res = arith(scores(), p_tx, p_qy);
      CT::template schedule<BOUND>();
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (CT::kSplit) __builtin_amdgcn_s_setprio(0);
      if (have_prev) post(res, p_tx, p_qy);
#pragma unroll
      for (int q = 0; q < NAC; ++q) accp[q] = acc[q];
      p_n = ncur;
      p_tx = TX;
      p_qy = qy;
      have_prev = true;
    };
    auto tile_par = [&](auto TXc, auto PARc) __attribute__((always_inline)) {
      constexpr int TX = decltype(TXc)::value;
      constexpr int PAR = decltype(PARc)::value;
      if constexpr (((PAR + TX) & 1) == 0) tile(TXc, bufA, bufB);
      else tile(TXc, bufB, bufA);
    };
    auto row = [&](auto PARc) __attribute__((always_inline)) {
      tile_par(std::integral_constant<int, 0>{}, PARc);
      if constexpr (NT > 1) tile_par(std::integral_constant<int, 1>{}, PARc);
      if constexpr (NT > 2) tile_par(std::integral_constant<int, 2>{}, PARc);
      if constexpr (NT > 3) tile_par(std::integral_constant<int, 3>{}, PARc);
      qy += stride;
    };
    int i = 0;
    if constexpr (NT % 2 == 0) {
      for (; i < nrows; ++i) row(std::integral_constant<int, 0>{});
    } else {
      for (; i + 1 < nrows; i += 2) {
        row(std::integral_constant<int, 0>{});
        row(std::integral_constant<int, 1>{});
      }
      if (i < nrows) row(std::integral_constant<int, 0>{});
    }
    post(arith(scores(), p_tx, p_qy), p_tx, p_qy);  // drain
  };

  // the column mask of tile column tx (wave-uniform tx: scalar selects of lane masks)
  auto col_mask = [&](int tx, int k) __attribute__((always_inline)) {
    bool m = colok[0][k];
#pragma unroll
    for (int q = 1; q < NT; ++q)
      if (tx == q) m = colok[q][k];
    return m;
  };

  // ---- sweep 1: bounding lists over the rows inside every reference row's window (a
  //      subset of each window: its K-th smallest bounds the window's from above).  In 3D
  //      it visits the reference's own slab only (still staged).  A form with a shorter
  //      bounding chain (contract.h) gives each distance up to kBoundRel (N_i + N_j) +
  //      kBoundAbs away from the selecting sweep's; the sweep adds that margin (in its norm
  //      terms), so its values bound the selecting sweep's distances of the same
  //      candidates from above.  NCC keeps the selecting sweep's chain.
  {
    const int b_lo = max(0, ryw + s * a_max - r);
    const int b_hi = min(g.Hv - 1, ryw - r + wsp);
    const int p1 = g.p1_step;
    auto sweep1 = [&](auto BOUNDc) __attribute__((always_inline)) {
      constexpr bool BOUND = decltype(BOUNDc)::value;
      const float grow = BOUND ? 1.f + CT::kBoundRel : 1.f;
      const float base1 = BOUND ? fmaf(base, CT::kBoundRel, base) + CT::kBoundAbs : base;
      sweep(BOUNDc, hsq * grow, b_lo + wave * p1, S * p1, b_hi,
            [&](const f4& sc, int tx, int) __attribute__((always_inline)) {
              f4 d;
#pragma unroll
              for (int k = 0; k < 4; ++k)
                d[k] = col_mask(tx, k) ? fmaf(-2.f, sc[k], base1) : INFINITY;
              return d;
            },
            [&](const f4& d, int, int) __attribute__((always_inline)) {
#pragma unroll
              for (int k = 0; k < 4; ++k) lane_insert<TL>(sel.tl, d[k]);
            });
    };
    if constexpr (CT::kBoundChain) {
      if (ncc) sweep1(std::false_type{});
      else sweep1(std::true_type{});
    } else {
      sweep1(std::false_type{});
    }
  }

  // ---- bound: reference p's values (its four lanes' lists in every wave) are merged by
  //      the wave that owns round p % 4 (round R: group g takes reference 4 g + R)
  {
    float* tlx = reinterpret_cast<float*>(bufs);  // [S][TL][64]
    float* thx = tlx + S * TL * 64;               // [16]
#pragma unroll
    for (int i = 0; i < TL; ++i) tlx[(wave * TL + i) * 64 + lane] = sel.tl[i];
    __syncthreads();
    const int nval = S * TL * 4;  // values per reference
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      if ((R % S) != wave) continue;
      const int p = 4 * gp + R;
      float L[KR];
#pragma unroll
      for (int q = 0; q < KR; ++q) L[q] = INFINITY;
      for (int b0 = 0; b0 < nval; b0 += 16) {
        const int v = b0 + p16;  // v = (w * TL + i) * 4 + quarter
        const float x = v < nval ? tlx[(v >> 2) * 64 + p + 16 * (v & 3)] : INFINITY;
        merge_batch_d<KR>(L, x, p16);
      }
      const float bound = next_up(kth_distance<KR>(L, g.K));
      if (p16 == 0) thx[p] = bound;
    }
    __syncthreads();
    sel.th = fminf(sel.th, thx[p16]);
    __syncthreads();  // the exchange area is the candidate buffers
    if (lane < 16) wcnt[lane] = 0;
  }

  // admission: score > thr on in-window columns
  float thr;
  auto set_thresholds = [&]() __attribute__((always_inline)) {
    thr = score_threshold(base, sel.th, true);
  };
  set_thresholds();

  // Merge this wave's candidate buffers into the round lists (round R: group g takes
  // reference 4 g + R), then lower each lane's threshold to its reference's list K-th
  // distance.
  bool flushed = false;  // a buffer flush happened in the selecting sweep (wave-uniform)
  constexpr int kFlushedBit = 1 << 24, kCountMask = kFlushedBit - 1;
  auto flush = [&]() __attribute__((always_inline)) {
    flushed = true;
    float kth[4];
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      const int p = 4 * gp + R;
      const int n = wcnt[p] & kCountMask;
      for (int e0 = 0; __any(e0 < n); e0 += 16) {
        const int e = e0 + p16;
        float cd = INFINITY;
        int cj = kNoIndex;
        if (e < n) {
          const Entry x = wbuf[p * CAP + e];
          cd = x.d;
          cj = x.j;
        }
        merge_batch<KR>(sel.Ld[R], sel.Lj[R], cd, cj, p16);
      }
      kth[R] = kth_distance<KR>(sel.Ld[R], g.K);
    }
    if (lane < 16) wcnt[lane] = 0;
    // this lane's reference p16 sits in group p16 / 4, round p16 % 4
    float mine = INFINITY;
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      const float v = __shfl(kth[R], 16 * ra);
      if (rb == R) mine = v;
    }
    sel.th = fminf(sel.th, mine);  // never loosen
    set_thresholds();
  };

  // ---- sweep 2: select
  over_slabs([&]() __attribute__((always_inline)) {
    const int jbase = jofs + xs + 4 * gp;
    sweep(std::false_type{}, hsq, qy_lo + wave, S, qy_hi,
          [&](const f4& sc, int tx, int qy) __attribute__((always_inline)) {
            const bool rok = row_ok(qy);
            Admit a;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              a.d[k] = sc[k];
              a.pass[k] = rok & col_mask(tx, k) & (sc[k] > thr);
            }
            return a;
          },
          [&](const Admit& a, int tx, int qy) __attribute__((always_inline)) {
            if (__any(a.pass[0] | a.pass[1] | a.pass[2] | a.pass[3])) {
              // this lane's passes go to its reference's buffer: one LDS atomic reserves
              // them (the four lanes of a reference share the buffer), then one write each
              const int c = (int)a.pass[0] + (int)a.pass[1] + (int)a.pass[2] + (int)a.pass[3];
              int slot = 0;
              if (c > 0) slot = atomicAdd(&wcnt[p16], c);
              const int jt = jbase + qy * W + kTileN * tx;
              Entry* dst = wbuf + p16 * CAP;
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                if (a.pass[k]) {
                  dst[slot] = Entry{fmaf(-2.f, a.d[k], base), jt + k};
                  ++slot;
                }
              }
              // a tile adds at most 16 entries to one reference
              if (__any(slot > CAP - 16)) flush();
            }
          });
  });
  // ---- final merge.  If no wave of the block flushed during the sweep (the usual case),
  //      the owner of round R (wave R mod S) merges every wave's buffered entries of its
  //      four references at once.  Otherwise each wave flushes its buffers into its lists
  //      and the owner merges the other waves' (sorted) lists.
  //      The flag travels in a high bit of each wave's counters (no LDS beyond the layout's).
  if (flushed && lane < 16) wcnt[lane] |= kFlushedBit;
  bool any_flushed = true;
  if (S > 1) {
    __syncthreads();
    const size_t wst = (size_t)16 * CAP * 8 + 64;
    int fl = 0;
    for (int w = 0; w < S; ++w) fl |= reinterpret_cast<const int*>(bufs + w * wst + (size_t)16 * CAP * 8)[0];
    any_flushed = (__builtin_amdgcn_readfirstlane(fl) & kFlushedBit) != 0;
    // every wave has read the flags before a flush below clears its counters (a wave
    // reading a cleared flag would take the other path)
    __syncthreads();
  }
  if (!any_flushed) {
    const size_t wstride = (size_t)16 * CAP * 8 + 64;
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      if ((R % S) != wave) continue;
      const int p = 4 * gp + R;
      int off[8];
      int tot = 0;
      for (int w = 0; w < S; ++w) {
        off[w] = tot;
        tot += reinterpret_cast<const int*>(bufs + w * wstride + (size_t)16 * CAP * 8)[p] & kCountMask;
      }
      for (int e0 = 0; __any(e0 < tot); e0 += 16) {
        const int e = e0 + p16;
        float cd = INFINITY;
        int cj = kNoIndex;
        if (e < tot) {
          int w = 0;
          for (int u = 1; u < S; ++u) w = e >= off[u] ? u : w;
          const Entry x = reinterpret_cast<const Entry*>(bufs + w * wstride)[p * CAP + e - off[w]];
          cd = x.d;
          cj = x.j;
        }
        merge_batch<KR>(sel.Ld[R], sel.Lj[R], cd, cj, p16);
      }
    }
  } else {
    flush();
  }
  if (S > 1 && any_flushed) {
    Entry* lx = reinterpret_cast<Entry*>(bufs);  // [S][4][KR][64]
    __syncthreads();
#pragma unroll
    for (int R = 0; R < 4; ++R)
#pragma unroll
      for (int q = 0; q < KR; ++q)
        lx[((wave * 4 + R) * KR + q) * 64 + lane] = Entry{sel.Ld[R][q], sel.Lj[R][q]};
    __syncthreads();
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      if ((R % S) != wave) continue;
      for (int w = 0; w < S; ++w) {
        if (w == wave) continue;
#pragma unroll
        for (int q = 0; q < KR; ++q) {
          const Entry e = lx[((w * 4 + R) * KR + q) * 64 + lane];
          merge_sorted<KR>(sel.Ld[R], sel.Lj[R], e.d, e.j, p16);
        }
      }
    }
  }
#pragma unroll
  for (int R = 0; R < 4; ++R) {
    if ((R % S) != wave) continue;
    // reference (row gp, column R) of the block
    const bool ok = (gp <= a_max) & (R <= b_max);
    if (!ok) continue;
    const size_t ref = (size_t)(RYw + gp) * g.nrx + (RXw + R);
    const float outk = ncc ? [&] {
      const float n = nrm[(size_t)(ryw + s * gp) * g.Wv + (rxw + s * R)];
      return n > 0.f ? 1.f / sqrtf(n) : 0.f;
    }() : 0.f;
    float o[KR];
    int oj[KR];
    bool neg = false;
#pragma unroll
    for (int q = 0; q < KR; ++q) {
      const bool none = sel.Lj[R][q] == kNoIndex;
      const float d = sel.Ld[R][q];
      neg |= d < 0.f;
      o[q] = none ? INFINITY
                  : (ncc ? fminf(fmaxf(fmaf(outk, d, 2.f), 0.f), 4.f) : fmaxf(d * isq, 0.f));
      oj[q] = sel.Lj[R][q];
    }
    // outputs are a monotone map of the keys that can tie distinct keys (NCC rounding and
    // clamp, the clamp of negative Euclidean keys): re-sort by (value, index)
    if (ncc || __any(neg)) sort_list<KR>(o, oj, p16);
#pragma unroll
    for (int q = 0; q < KR; ++q) {
      const int e = 16 * q + p16;
      if (e < g.K) {
        const bool none = oj[q] == kNoIndex;
        out_idx[ref * g.K + e] = none ? -1 : oj[q];
        out_dist[ref * g.K + e] = none ? INFINITY : o[q];
      }
    }
  }
}

}  // namespace bmk
