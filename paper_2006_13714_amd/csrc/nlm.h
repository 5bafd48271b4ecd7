// Non-local means over each reference's search window for gfx950 (Sec. III-A,
// Eq. (equ:nlm); Prop. 1): for reference X_i and every in-window candidate X_j,
//     w_ij = exp(-||X_j - X_i||^2 / b^2),  Theta_i = sum_j w_ij,
//     Y_i = sum_j w_ij X_j / Theta_i,
// with the distance from Lemma 2 (norm box filter + Self-Convolution cross term).  Prop. 1
// writes the weights as exp((2 C_i - h(.)h - ||X_i||^2) / b^2): this kernel evaluates that
// expression with the cross term on the matrix cores, then forms the weighted patch sum as a
// second dense contraction on the matrix cores.
//
// Same block structure as the specialised BM kernel (xcorr_fast.h): one workgroup per 4 x 4
// block of references, float32 strip and norm strip staged in LDS, candidate rows dealt
// round-robin to the waves.  Per 16 x 16 tile (16 references x 16 candidates):
//   1. cross term: the CtF32 matrix-op chain (16 refs x 16 cands, contraction over patch);
//   2. w = exp2(d * k), k = -log2(e) / b^2, with out-of-window pairs at d = +inf (w = 0);
//      Theta partial sums stay in registers;
//   3. the 16 x 16 weight tile goes through the wave's own LDS area from the accumulator
//      layout (reference x candidate by lane group) to the operand layout;
//   4. weighted patch sum: D[ref][pixel] += sum_cand W[ref][cand] X_cand[pixel] with
//      v_mfma_f32_16x16x4f32, candidate pixels read straight from the strip (16-pixel blocks
//      of 2 patch rows x 8 columns).
// At the end Theta is reduced over the 16 lanes of a group and over the waves, the patch sums
// over the waves (through LDS), and each reference's patch is divided by its Theta.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bm_internal.h"
#include "contract.h"
#include "topk.h"

namespace bmk {

template <int C, int H2, int NT>
__global__ void __launch_bounds__(256)
nlm_fast(const float* __restrict__ img, const float* __restrict__ nrm,
         float* __restrict__ out_patch, float* __restrict__ out_theta, const FastGeom g,
         float kexp) {
  using CT = CtF32<C, H2>;
  constexpr int CRS = CT::CRS;
  constexpr int RS = CT::RW;
  constexpr int NS = CT::NS;
  constexpr int NW = kTileN * NT;
  constexpr int NPB = C * H2;  // 16-pixel blocks per patch: (row pair, channel)
  extern __shared__ __align__(16) unsigned char lds[];
  float* strip = reinterpret_cast<float*>(lds + g.lds_strip_off);
  float* nstrip = reinterpret_cast<float*>(lds + g.lds_norm_off);
  float* wall = reinterpret_cast<float*>(lds + g.lds_buf_off);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int S = blockDim.x >> 6;

  const int blk = xcd_remap(blockIdx.x, g.nwg_total);
  const int by = blk / g.nwg_x;
  const int bx = blk - by * g.nwg_x;
  const int s = g.s, r = g.r;
  const int RYw = kRefBlock * by, RXw = kRefBlock * bx;
  const int ryw = s * RYw, rxw = s * RXw;
  const int SY0 = ryw - r, SX0 = rxw - r;

  // ---- stage the strip (zero outside the image) and the norm strip (+inf outside)
  float center[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) center[c] = 0.f;
  CT::stage(reinterpret_cast<uint32_t*>(strip), img, g, SY0, SX0, wave, S, lane, center, 1.f);
  // norm strip: four rows per pass, loads unconditional (clamped) and masked afterwards
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
        nv[u] = nrm[ok[u] ? (size_t)qy * g.Wv + qx : 0];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (y0 + u * S < g.NH) nstrip[(y0 + u * S) * NW + x] = ok[u] ? nv[u] : INFINITY;
    }
  }
  __syncthreads();

  const int a_max = min(3, g.nry - 1 - RYw);
  const int b_max = min(3, g.nrx - 1 - RXw);
  const int r2 = g.wspan;  // window offsets -r .. -r + r2
  const int p16 = lane & 15;
  const int gp = lane >> 4;
  const int lane_off = CT::lane_off(gp);

  float A[NS];
  CT::load_a(A, reinterpret_cast<const uint32_t*>(strip),
             (s * (p16 >> 2) + r) * CRS + (s * (p16 & 3) + r) + lane_off, gp, g.P);

  // reference norms with the column part of the window and the image's valid columns
  // folded in (+inf: weight 0)
  float nrx[NT][4];
  {
    float norms[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) norms[v] = nstrip[(s * gp + r) * NW + s * v + r];
#pragma unroll
    for (int tx = 0; tx < NT; ++tx)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool inw = (unsigned)(kTileN * tx + p16 - s * v) <= (unsigned)r2;
        const bool colok = (unsigned)(rxw - r + kTileN * tx + p16) < (unsigned)g.Wv;
        nrx[tx][v] = (inw & colok) ? norms[v] : INFINITY;
      }
  }

  const int qy_lo = max(0, ryw - r);
  const int qy_hi = min(g.Hv - 1, ryw + s * a_max - r + r2);
  const int bl = lane_off + p16;
  // operand-B lane offset of the weighted sum: candidate 4t + gp of the tile, pixel
  // (row (p16 / 8) of the pair, column p16 % 8)
  const int boff = ((p16 >> 3) * C) * RS + (p16 & 7) + gp;
  float* wb = wall + wave * 256;  // this wave's 16 x 16 weight tile

  f4 ysum[NPB];
#pragma unroll
  for (int pb = 0; pb < NPB; ++pb) ysum[pb] = f4{0.f, 0.f, 0.f, 0.f};
  float th[4] = {0.f, 0.f, 0.f, 0.f};

  for (int qy = qy_lo + wave; qy <= qy_hi; qy += S) {
    const float ybias = ((unsigned)(qy - ryw - s * gp + r) <= (unsigned)r2) ? 0.f : INFINITY;
    const int rowb = (qy - SY0) * CRS;
#pragma unroll
    for (int tx = 0; tx < NT; ++tx) {
      // 1. cross term of the 16 x 16 tile
      float B[NS];
      CT::load_b(B, reinterpret_cast<const uint32_t*>(strip), rowb + bl + kTileN * tx);
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < NS; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[t], B[t], acc, 0, 0, 0);
      // 2. weights (Lemma 2 distance; masked pairs at +inf give 0)
      const float nc = nstrip[(qy - SY0) * NW + kTileN * tx + p16] + ybias;
      float w[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        w[v] = exp2f(fmaf(-2.f, acc[v], nrx[tx][v] + nc) * kexp);
        th[v] += w[v];
      }
      // 3. accumulator layout (ref 4 gp + v, cand p16) -> operand layout (ref p16, cand k)
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int v = 0; v < 4; ++v) wb[(4 * gp + v) * 16 + p16] = w[v];
      __builtin_amdgcn_wave_barrier();
      float a2[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) a2[t] = wb[p16 * 16 + 4 * t + gp];
      // 4. weighted patch sums
      const int pbase = rowb + boff + kTileN * tx;
#pragma unroll
      for (int pb = 0; pb < NPB; ++pb) {
        const int l2 = pb / C, c = pb - (pb / C) * C;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          ysum[pb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
              a2[t], strip[pbase + (2 * l2 * C + c) * RS + 4 * t], ysum[pb], 0, 0, 0);
      }
    }
  }

  // ---- Theta over the 16 candidate lanes of each group
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) th[v] += __shfl_xor(th[v], o);

  // ---- reduce over the waves through LDS (the strips are no longer needed)
  __syncthreads();
  float* red = reinterpret_cast<float*>(lds);                 // [S][16 refs][NPB * 16]
  float* redt = red + S * 16 * NPB * 16;                        // [S][16 refs]
#pragma unroll
  for (int pb = 0; pb < NPB; ++pb)
#pragma unroll
    for (int i = 0; i < 4; ++i) red[((wave * 16 + 4 * gp + i) * NPB + pb) * 16 + p16] = ysum[pb][i];
  if (p16 == 0)
#pragma unroll
    for (int v = 0; v < 4; ++v) redt[wave * 16 + 4 * gp + v] = th[v];
  __syncthreads();

  // ---- outputs: reference m = 4 a + b of the block -> grid (RYw + a, RXw + b)
  const int P = g.P;
  const int per_ref = C * P * P;
  for (int e = tid; e < 16 * per_ref; e += blockDim.x) {
    const int m = e / per_ref;
    const int rem = e - m * per_ref;
    const int c = rem / (P * P);
    const int l = (rem / P) % P;
    const int mm = rem % P;
    const int a = m >> 2, b = m & 3;
    if (a > a_max || b > b_max) continue;
    float tot = 0.f, sum = 0.f;
    const int pb = (l >> 1) * C + c;
    const int n = (l & 1) * 8 + mm;
    for (int w2 = 0; w2 < S; ++w2) {
      tot += redt[w2 * 16 + m];
      sum += red[((w2 * 16 + m) * NPB + pb) * 16 + n];
    }
    const size_t ref = (size_t)(RYw + a) * g.nrx + (RXw + b);
    out_patch[ref * per_ref + rem] = sum / tot;
    if (rem == 0 && out_theta) out_theta[ref] = tot;
  }
}

typedef void (*NlmKernel)(const float*, const float*, float*, float*, const FastGeom, float);

template <int C, int H2>
static NlmKernel nlm_nt(int nt) {
  switch (nt) {
    case 2: return nlm_fast<C, H2, 2>;
    case 3: return nlm_fast<C, H2, 3>;
  }
  return nullptr;
}

template <int C>
static NlmKernel nlm_h2(int h2, int nt) {
  switch (h2) {
    case 2: return nlm_nt<C, 2>(nt);
    case 3: return nlm_nt<C, 3>(nt);
    case 4: return nlm_nt<C, 4>(nt);
  }
  return nullptr;
}

}  // namespace bmk
