// Fused window-masked cross-correlation + distance assembly + top-K for gfx950, specialised
// for C <= 4 channels, patch side 3..8, K <= 32 and a candidate span of NT * 16 columns per
// 4-reference block.  The contraction policy (contract.h) selects float32 products or the
// hi/lo split forms (bfloat16 or float16, three products, float32 accumulation).
//
// Per reference X_i and in-window candidate X_j it evaluates Lemma 2 (Sec. III-B),
//     d_ij = ||X_j||^2 + ||X_i||^2 - 2 <X_i, X_j>,
// where <X_i, X_j> is the window-restricted Self-Convolution of Eq. (eq:selfConv) (footnote
// to Eq. (eq:unifySelfConv)) summed over channels (Sec. IV, S(.)), computed on the matrix
// cores, and keeps the K smallest (Theorem 1, Euclidean branch).
//
//  * One workgroup = one 4 x 4 block of references, shared by S waves.  The workgroup
//    stages the pixel strip covering the block's search windows (all channels, rows
//    interleaved by channel, compile-time row stride) in LDS once; the candidate norms are
//    read from the norm map a row ahead of use, or (NSTRIP) staged as a norm strip too.
//    Candidate rows are dealt round-robin to the S waves, so each wave visits the
//    candidates of every reference in increasing j.
//  * Matrix tile: 16 references x 16 candidates (a 16-wide row segment).  Operand A
//    (reference patches) stays in registers; operand B is read from the strip with one base
//    register per row and immediate offsets (adjacent lanes read adjacent pixels: no
//    im2col).  The accumulator of a split form carries the pre-scale squared, which the
//    distance assembly removes exactly (power of two).
//  * Window mask: folded into the norms.  ||X_i||^2 is replaced by +inf for tile columns
//    outside reference i's column range (precomputed per tile column) and ||X_j||^2 by
//    +inf for rows outside the row range (per row), so an excluded pair has d = +inf.
//  * Software pipeline: each tile's matrix ops are interleaved with the epilogue
//    arithmetic of the previous tile and the LDS reads of the next one.
//  * Metric: Euclidean (Lemma 2) or normalized cross-correlation (Eq. equ:cor, Lemma 1).
//    For NCC the candidate norms become -1/||X_j|| (times the split forms' post-scale), so the
//    same epilogue multiply-add yields e'' = -<X_i, X_j> / ||X_j||, which orders a
//    reference's candidates exactly like 2 - 2 NCC; outputs are 2 - 2 NCC = 2 + 2 e'' / ||X_i||.
//  * Selection (select.h): a bounding sweep over every p1-th candidate row of each wave,
//    a lane-wise merge of the S waves' bounding lists into one upper bound on each K-th
//    distance, a selecting sweep over all rows, and an exact merge of the S waves' lists.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>
#include <stdint.h>

#include "bm_internal.h"
#include "contract.h"
#include "select.h"

namespace bmk {

// Upper bound of max |x - centre| over the strip rows [y0, y1] x columns [x0, x1] (image
// coordinates, already clipped) in `nmap` stacked per-tile maps of the norm pass (`stride`
// entries apart): the largest entry over the tiles that hold those pixels.  The lanes read
// the entries in parallel and a wave-wide max reduces them; the result is the same in
// every lane and every wave.
__device__ __forceinline__ float strip_absmax(const float* __restrict__ amax, const FastGeom& g,
                                              int y0, int y1, int x0, int x1, int lane,
                                              int nmap = 1, size_t stride = 0) {
  const int ty0 = min(y0 / kNormTY, g.nty - 1), ty1 = min(y1 / kNormTY, g.nty - 1);
  const int tx0 = min(x0 / kNormTX, g.ntx - 1), tx1 = min(x1 / kNormTX, g.ntx - 1);
  const int nx = tx1 - tx0 + 1, per = nx * (ty1 - ty0 + 1);
  float m = 0.f;
  for (int i = lane; i < per * nmap; i += 64) {
    const int k = i / per, e = i - k * per;
    const int ty = ty0 + e / nx, tx = tx0 + e - (e / nx) * nx;
    m = fmaxf(m, amax[k * stride + (size_t)ty * g.ntx + tx]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  return m;
}

// Candidate slabs of a 3D search (Sec. IV, 3D Self-Convolution): the reference's d-channel
// slab is the one passed to fast_block as `img` / `nrm`; its candidates come from the
// d-channel slabs z0..z1 of the volume (channel planes of H x W), each with its own norm map
// (Hv x Wv) and, in the float16 form, its own per-tile max map.
struct DepthWin {
  const float* vol;
  const float* nrm;
  const float* amax;
  int z0, z1;
  int tiles;  // entries of one slab's max map
};

// One 4 x 4 reference block `blk` (row-major over the block grid) of one image, computed by
// the whole workgroup (blockDim.x / 64 waves).  `centers` holds the per-channel centring
// constants or is null; `amax` is the norm pass's per-tile max map (float16 form only).
// Every thread of the workgroup must call it (it synchronises).  With D3 the candidates
// are those of the slabs in `dw` (visited in increasing depth, restaged per slab, one
// selection state across all of them) and indices are volume positions (z' H + qy) W + qx.
// NSTRIP: candidate norms staged in LDS with the pixel strip (the layout's norm strip)
// instead of read from the norm map a row ahead.  The single-image kernels and the split
// forms' batch tiers read the map, whose smaller LDS footprint lets more workgroups share a
// compute unit; the 3D kernels and the float32 batch tiers stage the strip.
template <class CT, int C, int KR, int NT, bool D3 = false, bool NSTRIP = true>
__device__ __forceinline__ void fast_block(const float* __restrict__ img,
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
  constexpr int TL = RefSelect<KR>::TL;
  static_assert(NT >= 1 && NT <= 4, "tile columns");
  constexpr int NW = kTileN * NT;  // norm strip row length
  uint32_t* strip = reinterpret_cast<uint32_t*>(lds + g.lds_strip_off);
  float* nstrip = reinterpret_cast<float*>(lds + g.lds_norm_off);  // NSTRIP only
  Entry* buf_all = reinterpret_cast<Entry*>(lds + g.lds_buf_off);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int S = blockDim.x >> 6;  // waves sharing the reference block

  const int by = blk / g.nwg_x;
  const int bx = blk - by * g.nwg_x;
  const int s = g.s, r = g.r;
  const int RYw = kRefBlock * by, RXw = kRefBlock * bx;
  const int ryw = s * RYw, rxw = s * RXw;  // pixel position of the block's reference (0,0)
  const int SY0 = ryw - r, SX0 = rxw - r;   // strip origin (may be negative)

  // centring constants; the float16 form's power-of-two pre-scale 2^k keeps the largest
  // staged magnitude of this block's strip below 2^14, and the distance assembly removes
  // it exactly (factor 2^-2k)
  float center[8];
  float scale = 1.f, mc = -2.f;  // d = mc * acc + (||X_i||^2 + ||X_j||^2)
#pragma unroll
  for (int c = 0; c < 8; ++c) center[c] = (centers && c < C) ? centers[c] : 0.f;
  if constexpr (CT::kScaled) {
    const int y0 = max(SY0, 0), y1 = min(SY0 + g.SH, g.H) - 1;
    const int x0 = max(SX0, 0), x1 = min(SX0 + g.SW, g.W) - 1;
    float m;
    if constexpr (D3)  // one scale for every slab the block stages (the reference's included)
      m = strip_absmax(dw->amax + (size_t)dw->z0 * dw->tiles, g, y0, y1, x0, x1, threadIdx.x & 63,
                       dw->z1 - dw->z0 + 1, dw->tiles);
    else
      m = strip_absmax(amax, g, y0, y1, x0, x1, threadIdx.x & 63);
    const int e = m > 0.f ? ilogbf(m) + 1 : 0;  // m < 2^e
    const int k = max(-60, min(60, 14 - e));
    scale = ldexpf(1.f, k);
    mc = -2.f * ldexpf(1.f, -2 * k);
  }
  const bool ncc = g.metric != 0;  // wave-uniform
  const float post = -0.5f * mc;   // removes the split forms' pre-scale (power of two)

  // Candidate norms as the epilogue uses them: Euclidean ||X_j||^2 (+inf outside the valid
  // positions), NCC -post/||X_j|| (0 for a zero patch and outside the valid positions,
  // which the column masks exclude).  Without NSTRIP they are read from the norm map (L2
  // resident) a row ahead of use.
  const float npost = -post;
  auto cand_norm = [&](float n, bool ok) __attribute__((always_inline)) {
    return ncc ? ((ok & (n > 0.f)) ? npost / sqrtf(n) : 0.f) : (ok ? n : INFINITY);
  };
  const float* nm_cur = nrm;  // norm map of the candidates' slab

  // ---- stage the strip (policy layout; zero outside the image) and, with NSTRIP, the norm
  //      strip (four rows per pass, loads unconditional (clamped) and masked afterwards)
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
            if (y0 + u * S < g.NH) nstrip[(y0 + u * S) * NW + x] = cand_norm(nv[u], ok[u]);
        }
      }
    }
  };
  stage_slab(img, nrm);
  __syncthreads();

  const int a_max = min(3, g.nry - 1 - RYw);
  const int b_max = min(3, g.nrx - 1 - RXw);
  const int P = g.P, r2 = g.wspan, W = g.W;  // window offsets -r .. -r + r2
  const int p16 = lane & 15;  // operand A row / operand B column / output column
  const int gp = lane >> 4;   // lane group: 2x2 element of a step; output reference row
  const int lane_off = CT::lane_off(gp);

  // ---- operand A: reference i = p16 -> block position (i/4, i%4); zero the padding
  //      elements of odd patch sides
  typename CT::AReg A[NA];
  const int plane = CT::plane_off(g);  // split forms: hi plane -> lo plane
  CT::load_a(A, strip, (s * (p16 >> 2) + r) * CRS + (s * (p16 & 3) + r) + lane_off, gp, P,
             plane);

  // ---- selection state for references (row gp, column v); norms with the column part of
  //      the window folded in
  RefSelect<KR> sel;
  bool valid[4];
  float nrx[NT][4];
  {
    float norms[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // reference (ryw + s gp, rxw + s v); padding references read a clamped position
      const int ry = min(ryw + s * gp, g.Hv - 1), rx = min(rxw + s * v, g.Wv - 1);
      norms[v] = cand_norm(nrm[(size_t)ry * g.Wv + rx], true);
      valid[v] = (gp <= a_max) & (v <= b_max);
    }
    sel.init(buf_all + (size_t)wave * 16 * g.CAP, g.CAP, g.K, lane, norms, valid);
    // NCC outputs 2 - 2 NCC = 2 + (2/||X_i||) e''; norms[v] holds -post/||X_i|| here
    sel.ncc = ncc;
#pragma unroll
    for (int v = 0; v < 4; ++v) sel.outk[v] = -2.f * norms[v] / post;
    // column masks: the reference's window columns and the image's valid columns
#pragma unroll
    for (int tx = 0; tx < NT; ++tx)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool inw = (unsigned)(kTileN * tx + p16 - s * v) <= (unsigned)r2;
        const bool colok = (unsigned)(rxw - r + kTileN * tx + p16) < (unsigned)g.Wv;
        nrx[tx][v] = (inw & colok) ? (ncc ? 0.f : norms[v]) : INFINITY;
      }
  }

  const int qy_lo = max(0, ryw - r);
  const int qy_hi = min(g.Hv - 1, ryw + s * a_max - r + r2);
  const int xs = rxw - r;  // first candidate column of the block
  const int bl = lane_off + p16;  // operand B lane offset within a strip row
  bool colok_t[NT];               // this lane's candidate column of tile t is a valid position
#pragma unroll
  for (int t = 0; t < NT; ++t) colok_t[t] = (unsigned)(xs + kTileN * t + p16) < (unsigned)g.Wv;

  // Candidate index of (slab, row 0, column 0): 0 in 2D; set per slab by over_slabs.
  int jofs = 0;
  // Runs `body` once (2D), or once per candidate slab after restaging the strips (3D).
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

  // One sweep over rows first, first + stride, ... (<= qy_hi) of this wave.  `arith` runs
  // inside the pipelined region on the previous tile; `post` may branch.
  auto sweep = [&](int first, int stride, auto&& arith, auto&& post) __attribute__((always_inline)) {
    if (first > qy_hi) return;
    const int nrows = (qy_hi - first) / stride + 1;
    BReg bufA[NB], bufB[NB];
    f4 accp = {0.f, 0.f, 0.f, 0.f};
    // carried description of the previous tile (a virtual +inf row before the first)
    float p_ybias = INFINITY, p_ns = 0.f;
    int p_nrow = 0, p_jrow = 0, p_tx = 0;
    int qy = first;
    CT::load_b(bufA, strip, (qy - SY0) * CRS + bl, plane);
    // raw candidate norms of the current row's tiles and of the next row (loads clamped to a
    // valid position; the column masks are applied when a tile takes its value)
    float ncur[NT], nnxt[NT];
    auto load_norms = [&](float (&dst)[NT], int row) __attribute__((always_inline)) {
      if constexpr (!NSTRIP) {
        const float* src = nm_cur + (size_t)row * g.Wv;
#pragma unroll
        for (int t = 0; t < NT; ++t) dst[t] = src[colok_t[t] ? xs + kTileN * t + p16 : 0];
      } else {
        (void)dst, (void)row;
      }
    };
    load_norms(ncur, qy);
    // tile (qy, TX) with operands in `cur`; loads the next tile into `nxt`
    auto tile = [&](auto TXc, BReg (&cur)[NB], BReg (&nxt)[NB]) __attribute__((always_inline)) {
      constexpr int TX = decltype(TXc)::value;
      __builtin_amdgcn_sched_barrier(0);
      const int nqy = (TX + 1 < NT) ? qy : min(qy + stride, qy_hi);
      const int nrb = (nqy - SY0) * CRS + bl + ((TX + 1 < NT) ? kTileN * (TX + 1) : 0);
      const f4 acc = CT::chain_and_load(A, cur, nxt, strip, nrb, plane);
      const float ns = NSTRIP ? nstrip[p_nrow + p16 + kTileN * p_tx] : p_ns;
      // d = X * acc + (column part + Y): Euclidean X = mc, Y = ||X_j||^2 + row mask;
      // NCC X = -post/||X_j||, Y = row mask
      const float X = ncc ? ns : mc;
      const float Y = ncc ? p_ybias : ns + p_ybias;
      auto res = arith(accp, X, Y, p_tx);
      CT::schedule();
      __builtin_amdgcn_sched_barrier(0);
      post(res, p_jrow + kTileN * p_tx + p16);
      accp = acc;
      p_tx = TX;
      if constexpr (!NSTRIP) p_ns = cand_norm(ncur[TX], colok_t[TX]);
      if constexpr (TX == 0) {
        p_ybias = ((unsigned)(qy - ryw - s * gp + r) <= (unsigned)r2) ? 0.f : INFINITY;
        if constexpr (NSTRIP) p_nrow = (qy - SY0) * NW;
        p_jrow = jofs + qy * W + xs;
      }
    };
    // tile TX of a row with buffer parity PAR uses buffer (PAR + TX) % 2 for its operands
    auto tile_par = [&](auto TXc, auto PARc) __attribute__((always_inline)) {
      constexpr int TX = decltype(TXc)::value;
      constexpr int PAR = decltype(PARc)::value;
      if constexpr (((PAR + TX) & 1) == 0) tile(TXc, bufA, bufB);
      else tile(TXc, bufB, bufA);
    };
    auto row = [&](auto PARc) __attribute__((always_inline)) {
      load_norms(nnxt, min(qy + stride, qy_hi));  // the next row's norms, a row ahead (map)
      tile_par(std::integral_constant<int, 0>{}, PARc);
      if constexpr (NT > 1) tile_par(std::integral_constant<int, 1>{}, PARc);
      if constexpr (NT > 2) tile_par(std::integral_constant<int, 2>{}, PARc);
      if constexpr (NT > 3) tile_par(std::integral_constant<int, 3>{}, PARc);
      qy += stride;
      if constexpr (!NSTRIP)
#pragma unroll
        for (int t = 0; t < NT; ++t) ncur[t] = nnxt[t];
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
    // drain: epilogue of the last tile
    const float ns = NSTRIP ? nstrip[p_nrow + p16 + kTileN * p_tx] : p_ns;
    const float X = ncc ? ns : mc;
    const float Y = ncc ? p_ybias : ns + p_ybias;
    post(arith(accp, X, Y, p_tx), p_jrow + kTileN * p_tx + p16);
  };

  // ---- sweep 1: bounding lists over every p1-th row of this wave.  In 3D it visits the
  //      reference's own slab only (still staged): the K-th smallest distance over a subset
  //      of the window's candidates bounds the K-th smallest over all of them from above,
  //      which is all the selecting sweep needs, and no slab is restaged for it.
  const int p1 = g.p1_step;
  auto over_bound_slabs = [&](auto&& body) __attribute__((always_inline)) {
    if constexpr (D3) {
      nm_cur = nrm;
      jofs = (int)((size_t)(img - dw->vol) / ((size_t)g.H * g.W)) * g.H * g.W;
    }
    body();
  };
  over_bound_slabs([&]() __attribute__((always_inline)) {
  sweep(qy_lo + wave * p1, S * p1,
        [&](const f4& acc, float X, float Y, int tx) __attribute__((always_inline)) {
          float nt[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) nt[v] = nrx[0][v];
#pragma unroll
          for (int q = 1; q < NT; ++q)
            if (tx == q)
#pragma unroll
              for (int v = 0; v < 4; ++v) nt[v] = nrx[q][v];
#pragma unroll
          for (int v = 0; v < 4; ++v)
            lane_insert<TL>(sel.tl[v], fmaf(X, acc[v], nt[v] + Y));
          return 0;
        },
        [&](int, int) __attribute__((always_inline)) {});
  });

  // ---- bound: wave w finishes the reference columns v with v % S == w: it merges the
  //      other waves' lane lists for that column into its own, takes the K-th over the 16
  //      lanes of each group, and publishes the thresholds; every wave then reads all four
  {
    float* tlx = reinterpret_cast<float*>(buf_all);  // [S][4][TL][64]
    float* thx = tlx + S * 4 * TL * 64;              // [4][64]
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int i2 = 0; i2 < TL; ++i2) tlx[((wave * 4 + v) * TL + i2) * 64 + lane] = sel.tl[v][i2];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if ((v % S) != wave) continue;
      for (int w = 0; w < S; ++w) {
        if (w == wave) continue;
#pragma unroll
        for (int i2 = 0; i2 < TL; ++i2)
          lane_insert<TL>(sel.tl[v], tlx[((w * 4 + v) * TL + i2) * 64 + lane]);
      }
      sel.bound_finish_col(v);
      thx[v * 64 + lane] = sel.th[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) sel.th[v] = thx[v * 64 + lane];
    __syncthreads();  // the exchange area is the candidate buffers
  }

  // ---- sweep 2: select
  over_slabs([&]() __attribute__((always_inline)) {
  sweep(qy_lo + wave, S,
        [&](const f4& acc, float X, float Y, int tx) __attribute__((always_inline)) {
          float nt[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) nt[v] = nrx[0][v];
#pragma unroll
          for (int q = 1; q < NT; ++q)
            if (tx == q)
#pragma unroll
              for (int v = 0; v < 4; ++v) nt[v] = nrx[q][v];
          Admit a;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            a.d[v] = fmaf(X, acc[v], nt[v] + Y);
            a.pass[v] = a.d[v] < sel.th[v];
          }
          return a;
        },
        [&](const Admit& a, int jg) __attribute__((always_inline)) { sel.commit(a, jg); });
  });
  sel.flush();

  // ---- exact merge of the S waves' lists: reference column v is finished by wave v mod S,
  //      which merges the other waves' (already sorted) lists for v and writes the outputs
  size_t ref[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) ref[v] = (size_t)(RYw + gp) * g.nrx + (RXw + v);
  if (S > 1) {
    Entry* lx = buf_all;  // [S][4][KR][64]
    __syncthreads();      // every wave is done with its candidate buffers
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int q = 0; q < KR; ++q)
        lx[((wave * 4 + v) * KR + q) * 64 + lane] = Entry{sel.Ld[v][q], sel.Lj[v][q]};
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if ((v % S) != wave) continue;
      for (int w = 0; w < S; ++w) {
        if (w == wave) continue;
#pragma unroll
        for (int q = 0; q < KR; ++q) {
          const Entry e = lx[((w * 4 + v) * KR + q) * 64 + lane];
          merge_sorted<KR>(sel.Ld[v], sel.Lj[v], e.d, e.j, p16);
        }
      }
      sel.write_col(v, out_idx, out_dist, ref[v], valid[v]);
    }
  } else {
    sel.write(out_idx, out_dist, ref, valid);
  }
}

// Waves per SIMD the compiler keeps registers for: the 1-channel split blocks fit four
// 4-wave workgroups per compute unit in LDS, so with K <= 16 (one list register) their
// registers are held to 128 (a few spilled words); with K <= 32 that spills too much.
template <class CT, int C, int KR>
constexpr int fast_waves_per_eu() { return (CT::kSplit && C == 1 && KR == 1) ? 4 : 1; }

// Single image: one workgroup per reference block, XCD-aware block order.
template <class CT, int C, int KR, int NT>
__global__ void __launch_bounds__(64 * fast_max_waves(CT::kSplit ? 1 : 0, C))
__attribute__((amdgpu_waves_per_eu(fast_waves_per_eu<CT, C, KR>())))
xcorr_topk_fast(const float* __restrict__ img, const float* __restrict__ nrm,
                const float* __restrict__ centers, const float* __restrict__ amax,
                int* __restrict__ out_idx, float* __restrict__ out_dist, const FastGeom g) {
  extern __shared__ __align__(16) unsigned char lds[];
  fast_block<CT, C, KR, NT, false, false>(img, nrm, centers, amax, out_idx, out_dist, g,
                                          xcd_remap(blockIdx.x, g.nwg_total), lds);
}

typedef void (*XcFastKernel)(const float*, const float*, const float*, const float*, int*,
                             float*, const FastGeom);

// 3D search over a volume: one workgroup per (reference depth z, 4 x 4 reference block),
// XCD-aware order over both.  Norm maps (and max maps) of every slab are stacked by depth;
// outputs are stacked by reference depth.
template <class CT, int C, int KR, int NT>
__global__ void __launch_bounds__(64 * fast_max_waves(CT::kSplit ? 1 : 0, C))
xcorr_topk_depth(const float* __restrict__ vol, const float* __restrict__ nrm,
                 const float* __restrict__ amax, int* __restrict__ out_idx,
                 float* __restrict__ out_dist, const FastGeom g, const DepthGeom dg) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int t = xcd_remap(blockIdx.x, g.nwg_total * dg.Z);
  const int z = t / g.nwg_total;
  const int blk = t - z * g.nwg_total;
  const size_t slab = (size_t)g.H * g.W, nslab = (size_t)g.Hv * g.Wv;
  const size_t outs = (size_t)g.nry * g.nrx * g.K;
  const int lo = z - dg.before;
  const DepthWin dw{vol, nrm, amax, max(0, lo), min(dg.Z - 1, lo + dg.c - 1), dg.tiles};
  fast_block<CT, C, KR, NT, true, true>(vol + z * slab, nrm + z * nslab, nullptr,
                                  amax ? amax + (size_t)z * dg.tiles : nullptr,
                                  out_idx + z * outs, out_dist + z * outs, g, blk, lds, &dw);
}

typedef void (*XcDepthKernel)(const float*, const float*, const float*, int*, float*,
                              const FastGeom, const DepthGeom);

// policy for (precision, C, H2): 0 float32, 1 bfloat16 split, 2 float16 split
template <int PREC, int C, int H2>
using CtFor = std::conditional_t<PREC == 0, CtF32<C, H2>, CtSplit<C, H2, PREC == 2>>;

template <int PREC, int C, int H2, int KR>
static XcDepthKernel depth_nt(int nt) {
  if constexpr (PREC != 0 && H2 < 3) {
    return nullptr;
  } else {
    switch (nt) {
      case 2: return xcorr_topk_depth<CtFor<PREC, C, H2>, C, KR, 2>;
      case 3: return xcorr_topk_depth<CtFor<PREC, C, H2>, C, KR, 3>;
    }
    return nullptr;
  }
}

template <int PREC, int C>
static XcDepthKernel depth_h2(int h2, int kr, int nt) {
  switch (h2 * 4 + kr) {
    case 2 * 4 + 1: return depth_nt<PREC, C, 2, 1>(nt);
    case 2 * 4 + 2: return depth_nt<PREC, C, 2, 2>(nt);
    case 3 * 4 + 1: return depth_nt<PREC, C, 3, 1>(nt);
    case 3 * 4 + 2: return depth_nt<PREC, C, 3, 2>(nt);
    case 4 * 4 + 1: return depth_nt<PREC, C, 4, 1>(nt);
    case 4 * 4 + 2: return depth_nt<PREC, C, 4, 2>(nt);
  }
  return nullptr;
}

template <int PREC, int C, int H2, int KR>
static XcFastKernel fast_nt(int nt) {
  if constexpr (PREC != 0 && H2 < 3) {
    return nullptr;  // split forms: patch side 5..8
  } else {
    switch (nt) {
      case 2: return xcorr_topk_fast<CtFor<PREC, C, H2>, C, KR, 2>;
      case 3: return xcorr_topk_fast<CtFor<PREC, C, H2>, C, KR, 3>;
    }
    return nullptr;
  }
}

template <int PREC, int C, int H2>
static XcFastKernel fast_kr(int kr, int nt) {
  switch (kr) {
    case 1: return fast_nt<PREC, C, H2, 1>(nt);
    case 2: return fast_nt<PREC, C, H2, 2>(nt);
  }
  return nullptr;
}

// All specialised kernels for one (precision, C): each is its own translation unit.
template <int PREC, int C>
static XcFastKernel fast_h2(int h2, int kr, int nt) {
  switch (h2) {
    case 2: return fast_kr<PREC, C, 2>(kr, nt);
    case 3: return fast_kr<PREC, C, 3>(kr, nt);
    case 4: return fast_kr<PREC, C, 4>(kr, nt);
  }
  return nullptr;
}

}  // namespace bmk
