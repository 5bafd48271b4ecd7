// Fused window-masked cross-correlation + distance assembly + top-K for gfx950 (float32),
// specialised for C <= 4 channels, patch side 3..8, K <= 32 and a candidate span of
// NT * 16 columns per 4-reference block.
//
// Per reference X_i and in-window candidate X_j it evaluates Lemma 2 (Sec. III-B),
//     d_ij = ||X_j||^2 + ||X_i||^2 - 2 <X_i, X_j>,
// where <X_i, X_j> is the window-restricted Self-Convolution of Eq. (eq:selfConv) (footnote
// to Eq. (eq:unifySelfConv)) summed over channels (Sec. IV, S(.)), computed on the matrix
// cores, and keeps the K smallest (Theorem 1, Euclidean branch).
//
//  * One workgroup = one 4 x 4 block of references, shared by S waves.  The workgroup
//    stages the pixel strip covering the block's search windows (all channels, rows
//    interleaved by channel, compile-time row stride) and the norm strip in LDS once.
//    Candidate rows are dealt round-robin to the S waves, so each wave visits the
//    candidates of every reference in increasing j.
//  * Matrix tile: 16 references x 16 candidates (a 16-wide row segment), contracted on
//    v_mfma_f32_16x16x4f32 in steps of 2 x 2 pixels of one channel.  Operand A (reference
//    patches) stays in registers; operand B is read from the strip with one base register
//    per row and immediate offsets (adjacent lanes read adjacent pixels: no im2col).
//  * Window mask: folded into the norms.  ||X_i||^2 is replaced by +inf for tile columns
//    outside reference i's column range (precomputed per tile column) and ||X_j||^2 by
//    +inf for rows outside the row range (per row), so an excluded pair has d = +inf.
//  * Software pipeline: each tile's matrix ops are interleaved with the epilogue
//    arithmetic of the previous tile and the LDS reads of the next one.
//  * Selection (select.h): a bounding sweep over every p1-th candidate row of each wave,
//    a lane-wise merge of the S waves' bounding lists into one upper bound on each K-th
//    distance, a selecting sweep over all rows, and an exact merge of the S waves' lists.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "bm_internal.h"
#include "select.h"

namespace bmk {

template <int C, int H2>
struct FastLayout {
  static constexpr int RS = kFastRS;
  static constexpr int CRS = C * RS;  // one image row across the channels
  static constexpr int KS = C * H2 * H2;
  // step t = ((l2 * H2) + m2) * C + c covers pixels (2*l2 + dy, 2*m2 + dx), dy, dx in {0,1}
  static constexpr int l2(int t) { return t / (H2 * C); }
  static constexpr int m2(int t) { return (t / C) % H2; }
  static constexpr int ch(int t) { return t % C; }
  static constexpr int off(int t) { return (2 * l2(t) * C + ch(t)) * RS + 2 * m2(t); }
};

template <int C, int H2, int KR, int NT>
__global__ void __launch_bounds__(256)
xcorr_topk_fast(const float* __restrict__ img, const float* __restrict__ nrm,
                int* __restrict__ out_idx, float* __restrict__ out_dist, const XcGeom g) {
  using L = FastLayout<C, H2>;
  constexpr int KS = L::KS;
  constexpr int RS = L::RS;
  constexpr int CRS = L::CRS;
  constexpr int TL = RefSelect<KR>::TL;
  static_assert(NT >= 1 && NT <= 4, "tile columns");
  constexpr int NW = kTileN * NT;  // norm strip row length
  extern __shared__ __align__(16) unsigned char lds[];
  float* strip = reinterpret_cast<float*>(lds + g.lds_strip_off);
  float* nstrip = reinterpret_cast<float*>(lds + g.lds_norm_off);
  Entry* buf_all = reinterpret_cast<Entry*>(lds + g.lds_buf_off);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int S = blockDim.x >> 6;  // waves sharing the reference block

  const int blk = xcd_remap(blockIdx.x, g.nwg_total);
  const int by = blk / g.nwg_x;
  const int bx = blk - by * g.nwg_x;
  const int s = g.s, r = g.r;
  const int RYw = kRefBlock * by, RXw = kRefBlock * bx;
  const int ryw = s * RYw, rxw = s * RXw;  // pixel position of the block's reference (0,0)
  const int SY0 = ryw - r, SX0 = rxw - r;   // strip origin (may be negative)

  // ---- stage the strip (rows y*C + c; zero outside the image) and the norm strip (+inf
  //      outside the valid positions)
  for (int row = wave; row < g.SH * C; row += S) {
    const int y = row / C;
    const int c = row - y * C;
    const int iy = SY0 + y;
    const bool yok = (iy >= 0) & (iy < g.H);
    const float cc = g.center[c];
    const float* src = img + ((size_t)c * g.H + (yok ? iy : 0)) * g.W;
    float* dst = strip + row * RS;
    for (int x = lane; x < g.SW; x += 64) {
      const int ix = SX0 + x;
      dst[x] = (yok & (ix >= 0) & (ix < g.W)) ? src[ix] - cc : 0.f;
    }
  }
  for (int y = wave; y < g.NH; y += S) {
    const int qy = SY0 + y;
    const bool yok = (qy >= 0) & (qy < g.Hv);
    const float* src = nrm + (size_t)(yok ? qy : 0) * g.Wv;
    float* dst = nstrip + y * NW;
    for (int x = lane; x < NW; x += 64) {
      const int qx = SX0 + x;
      dst[x] = (yok & (qx >= 0) & (qx < g.Wv)) ? src[qx] : INFINITY;
    }
  }
  __syncthreads();

  const int a_max = min(3, g.nry - 1 - RYw);
  const int b_max = min(3, g.nrx - 1 - RXw);
  const int P = g.P, r2 = 2 * r, W = g.W;
  const int p16 = lane & 15;  // operand A row / operand B column / output column
  const int gp = lane >> 4;   // lane group: 2x2 element of a step; output reference row
  const int lane_off = (gp >> 1) * CRS + (gp & 1);

  // ---- operand A: reference i = p16 -> block position (i/4, i%4); zero the padding
  //      elements of odd patch sides
  float A[KS];
  {
    const int base = (s * (p16 >> 2) + r) * CRS + (s * (p16 & 3) + r) + lane_off;
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      const bool ok = (2 * L::l2(t) + (gp >> 1) < P) & (2 * L::m2(t) + (gp & 1) < P);
      A[t] = ok ? strip[base + L::off(t)] : 0.f;
    }
  }

  // ---- selection state for references (row gp, column v); norms with the column part of
  //      the window folded in
  RefSelect<KR> sel;
  bool valid[4];
  float nrx[NT][4];
  {
    float norms[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      norms[v] = nstrip[(s * gp + r) * NW + s * v + r];
      valid[v] = (gp <= a_max) & (v <= b_max);
    }
    sel.init(buf_all + (size_t)wave * 16 * g.CAP, g.CAP, g.K, lane, norms, valid);
#pragma unroll
    for (int tx = 0; tx < NT; ++tx)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        nrx[tx][v] = ((unsigned)(kTileN * tx + p16 - s * v) <= (unsigned)r2) ? norms[v] : INFINITY;
  }

  const int qy_lo = max(0, ryw - r);
  const int qy_hi = min(g.Hv - 1, ryw + s * a_max + r);
  const int xs = rxw - r;  // first candidate column of the block
  const int bl = lane_off + p16;  // operand B lane offset within a strip row

  // One sweep over rows first, first + stride, ... (<= qy_hi) of this wave.  `arith` runs
  // inside the pipelined region on the previous tile; `post` may branch.
  auto sweep = [&](int first, int stride, auto&& arith, auto&& post) __attribute__((always_inline)) {
    if (first > qy_hi) return;
    const int nrows = (qy_hi - first) / stride + 1;
    float bufA[KS], bufB[KS];
    f4 accp = {0.f, 0.f, 0.f, 0.f};
    // carried description of the previous tile (a virtual +inf row before the first)
    float p_ybias = INFINITY;
    int p_nrow = 0, p_jrow = 0, p_tx = 0;
    int qy = first;
    {
      const int rb = (qy - SY0) * CRS + bl;
#pragma unroll
      for (int t = 0; t < KS; ++t) bufA[t] = strip[rb + L::off(t)];
    }
    // tile (qy, TX) with operands in `cur`; loads the next tile into `nxt`
    auto tile = [&](auto TXc, float (&cur)[KS], float (&nxt)[KS]) __attribute__((always_inline)) {
      constexpr int TX = decltype(TXc)::value;
      __builtin_amdgcn_sched_barrier(0);
      const int nqy = (TX + 1 < NT) ? qy : min(qy + stride, qy_hi);
      const int nrb = (nqy - SY0) * CRS + bl + ((TX + 1 < NT) ? kTileN * (TX + 1) : 0);
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[t], cur[t], acc, 0, 0, 0);
        nxt[t] = strip[nrb + L::off(t)];
      }
      const float nc = nstrip[p_nrow + p16 + kTileN * p_tx] + p_ybias;
      auto res = arith(accp, nc, p_tx);
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix op
        __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // up to two vector ops
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
      }
      __builtin_amdgcn_sched_barrier(0);
      post(res, p_jrow + kTileN * p_tx + p16);
      accp = acc;
      p_tx = TX;
      if constexpr (TX == 0) {
        p_ybias = ((unsigned)(qy - ryw - s * gp + r) <= (unsigned)r2) ? 0.f : INFINITY;
        p_nrow = (qy - SY0) * NW;
        p_jrow = qy * W + xs;
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
    // drain: epilogue of the last tile
    const float nc = nstrip[p_nrow + p16 + kTileN * p_tx] + p_ybias;
    post(arith(accp, nc, p_tx), p_jrow + kTileN * p_tx + p16);
  };

  // ---- sweep 1: bounding lists over every p1-th row of this wave
  const int p1 = g.p1_step;
  sweep(qy_lo + wave * p1, S * p1,
        [&](const f4& acc, float nc, int tx) __attribute__((always_inline)) {
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
            lane_insert<TL>(sel.tl[v], fmaf(-2.f, acc[v], nt[v] + nc));
          return 0;
        },
        [&](int, int) __attribute__((always_inline)) {});

  // ---- bound: lane-wise merge of the S waves' lists, then the K-th over the 16 lanes
  {
    float* tlx = reinterpret_cast<float*>(buf_all);  // [S][4][TL][64]
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int i2 = 0; i2 < TL; ++i2) tlx[((wave * 4 + v) * TL + i2) * 64 + lane] = sel.tl[v][i2];
    __syncthreads();
    for (int w = 0; w < S; ++w) {
      if (w == wave) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int i2 = 0; i2 < TL; ++i2)
          lane_insert<TL>(sel.tl[v], tlx[((w * 4 + v) * TL + i2) * 64 + lane]);
    }
    __syncthreads();  // the exchange area is the candidate buffers
  }
  sel.bound_finish();

  // ---- sweep 2: select
  sweep(qy_lo + wave, S,
        [&](const f4& acc, float nc, int tx) __attribute__((always_inline)) {
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
            a.d[v] = fmaf(-2.f, acc[v], nt[v] + nc);
            a.pass[v] = a.d[v] < sel.th[v];
          }
          return a;
        },
        [&](const Admit& a, int jg) __attribute__((always_inline)) { sel.commit(a, jg); });
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

typedef void (*XcKernel)(const float*, const float*, int*, float*, const XcGeom);

template <int C, int H2, int KR>
static XcKernel fast_nt(int nt) {
  switch (nt) {
    case 2: return xcorr_topk_fast<C, H2, KR, 2>;
    case 3: return xcorr_topk_fast<C, H2, KR, 3>;
  }
  return nullptr;
}

template <int C, int H2>
static XcKernel fast_kr(int kr, int nt) {
  switch (kr) {
    case 1: return fast_nt<C, H2, 1>(nt);
    case 2: return fast_nt<C, H2, 2>(nt);
  }
  return nullptr;
}

// All specialised kernels for C channels (one translation unit per C builds in parallel).
template <int C>
static XcKernel fast_h2(int h2, int kr, int nt) {
  switch (h2) {
    case 2: return fast_kr<C, 2>(kr, nt);
    case 3: return fast_kr<C, 3>(kr, nt);
    case 4: return fast_kr<C, 4>(kr, nt);
  }
  return nullptr;
}

}  // namespace bmk
