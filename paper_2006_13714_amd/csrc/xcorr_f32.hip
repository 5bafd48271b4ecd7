// Fused window-masked cross-correlation + distance assembly + top-K for gfx950 (float32).
//
// Per reference X_i and in-window candidate X_j the kernel evaluates Lemma 2 (Sec. III-B),
//     d_ij = ||X_j||^2 + ||X_i||^2 - 2 <X_i, X_j>,
// where <X_i, X_j> is the window-restricted Self-Convolution C_i(q, r) of Eq. (eq:selfConv)
// (footnote to Eq. (eq:unifySelfConv): X_{Omega_i} * X_i) summed over channels (Sec. IV,
// S(.)), computed as a dense contraction on the matrix cores, and keeps the K smallest
// (Theorem 1, Euclidean branch).  The similarity map is never written to memory.
//
// Work decomposition
//  * A wave owns a 4 x 4 block of references (grid stride s).  A workgroup of WY x WX waves
//    stages, once, the pixel strip that covers the union of its waves' search windows
//    (all channels) and the matching patch-norm strip in LDS.
//  * Matrix tile = 16 references x 16 candidates (one 16-wide row segment of candidate
//    positions), v_mfma_f32_16x16x4f32, contraction over the patch in steps of 4 elements
//    laid out as 2 x 2 pixel blocks.  The references' patches stay in registers (operand A);
//    candidate patches are read from the LDS strip with per-step offsets (operand B).  The
//    overlapping candidates need no im2col: adjacent lanes read adjacent pixels.
//  * Epilogue per tile: each lane holds 4 references x 1 candidate.  It assembles d in
//    float32, applies the window mask, and compares with the reference's current K-th
//    distance; survivors go to a per-reference LDS buffer via ballot/popcount compaction.
//    Full buffers are merged into the per-reference sorted lists by the wavefront-shuffle
//    bitonic networks of topk.h.  Candidates are visited in increasing j for every
//    reference, so a strict "d < K-th distance" test is exact for the (d, j) order.
#include <hip/hip_runtime.h>
#include <math.h>

#include "bm_internal.h"
#include "topk.h"

namespace bmk {

typedef float f4 __attribute__((ext_vector_type(4)));

struct Entry {
  float d;
  int j;
};

template <int KS, int KR>
__global__ void __launch_bounds__(256)
xcorr_topk_f32(const float* __restrict__ img, const float* __restrict__ nrm,
               int* __restrict__ out_idx, float* __restrict__ out_dist, const XcGeom g) {
  extern __shared__ __align__(16) unsigned char lds[];
  float* strip = reinterpret_cast<float*>(lds + g.lds_strip_off);
  float* nstrip = reinterpret_cast<float*>(lds + g.lds_norm_off);
  Entry* buf_all = reinterpret_cast<Entry*>(lds + g.lds_buf_off);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;

  const int wg = xcd_remap(blockIdx.x, g.nwg_total);
  const int wgy = wg / g.nwg_x;
  const int wgx = wg - wgy * g.nwg_x;
  const int RY0 = wgy * kRefBlock * g.WY;
  const int RX0 = wgx * kRefBlock * g.WX;
  const int SY0 = g.s * RY0 - g.r;  // strip origin in pixels (may be negative)
  const int SX0 = g.s * RX0 - g.r;

  // ---- stage the pixel strip (zero outside the image) and the norm strip (+inf outside
  //      the valid positions), one row per wave iteration, lanes across the row
  for (int row = wave; row < g.C * g.SH; row += nwaves) {
    const int c = row / g.SH;
    const int y = row - c * g.SH;
    const int iy = SY0 + y;
    const bool yok = iy >= 0 && iy < g.H;
    const float cc = g.center[c];
    const float* src = img + ((size_t)c * g.H + (yok ? iy : 0)) * g.W;
    float* dst = strip + c * g.PLANE + y * g.RS;
    for (int x = lane; x < g.SW; x += 64) {
      const int ix = SX0 + x;
      dst[x] = (yok && ix >= 0 && ix < g.W) ? src[ix] - cc : 0.f;
    }
  }
  for (int y = wave; y < g.NH; y += nwaves) {
    const int qy = SY0 + y;
    const bool yok = qy >= 0 && qy < g.Hv;
    const float* src = nrm + (size_t)(yok ? qy : 0) * g.Wv;
    float* dst = nstrip + y * g.NRS;
    for (int x = lane; x < g.NW; x += 64) {
      const int qx = SX0 + x;
      dst[x] = (yok && qx >= 0 && qx < g.Wv) ? src[qx] : INFINITY;
    }
  }
  __syncthreads();  // the only barrier: waves are independent from here on

  const int wy = wave / g.WX;
  const int wx = wave - wy * g.WX;
  const int RYw = RY0 + kRefBlock * wy;
  const int RXw = RX0 + kRefBlock * wx;
  if (RYw >= g.nry || RXw >= g.nrx) return;
  const int ryw = g.s * RYw;  // pixel position of the block's reference (0, 0)
  const int rxw = g.s * RXw;
  const int a_max = min(3, g.nry - 1 - RYw);
  const int b_max = min(3, g.nrx - 1 - RXw);

  const int p16 = lane & 15;  // operand A row / operand B column / output column
  const int gp = lane >> 4;   // lane group: k-element within a step; output reference row
  const int lane_off = (gp >> 1) * g.RS + (gp & 1);

  // ---- operand A: reference i = p16 -> block position (i/4, i%4)
  float A[KS];
  {
    const int ai = p16 >> 2, bi = p16 & 3;
    const int base = (ryw + g.s * ai - SY0) * g.RS + (rxw + g.s * bi - SX0) + lane_off;
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      const bool ok = (g.step_mask[t] >> gp) & 1u;
      A[t] = ok ? strip[base + g.step_off[t]] : 0.f;
    }
  }

  // ---- per-lane output references: (row gp, column v) of the block
  float nr[4], th[4];
  int cnt[4];
  float Ld[4][KR];
  int Lj[4][KR];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const bool ok = gp <= a_max && v <= b_max;
    nr[v] = nstrip[(ryw + g.s * gp - SY0) * g.NRS + (rxw + g.s * v - SX0)];
    th[v] = ok ? INFINITY : -INFINITY;  // -inf: a padding reference admits nothing
    cnt[v] = 0;
#pragma unroll
    for (int q = 0; q < KR; ++q) {
      Ld[v][q] = INFINITY;
      Lj[v][q] = kNoIndex;
    }
  }
  Entry* buf = buf_all + (size_t)wave * 16 * g.CAP;

  const int qy_lo = max(0, ryw - g.r);
  const int qy_hi = min(g.Hv - 1, ryw + g.s * a_max + g.r);
  const int xs = rxw - g.r;  // first tile start (unclipped)
  const int nt = (g.s * b_max + 2 * g.r + 1 + kTileN - 1) / kTileN;
  const int tx_lo = xs < -(kTileN - 1) ? (-xs) / kTileN : 0;
  const int tx_hi = min(nt - 1, (g.Wv - 1 - xs) / kTileN);
  const unsigned long long grp_bits = 0xFFFFull << (16 * gp);
  const unsigned long long below = (1ull << lane) - 1ull;

  auto flush = [&]() {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      for (int ch = 0; __any(ch * 16 < cnt[v]); ++ch) {
        const int e = ch * 16 + p16;
        float cd = INFINITY;
        int cj = kNoIndex;
        if (e < cnt[v]) {
          const Entry x = buf[(4 * gp + v) * g.CAP + e];
          cd = x.d;
          cj = x.j;
        }
        merge_batch<KR>(Ld[v], Lj[v], cd, cj, p16);
      }
      cnt[v] = 0;
      const float kth = kth_distance<KR>(Ld[v], g.K);
      th[v] = (th[v] == -INFINITY) ? -INFINITY : kth;
    }
  };

  for (int qy = qy_lo; qy <= qy_hi; ++qy) {
    const bool yin = abs(qy - ryw - g.s * gp) <= g.r;
    const int srow = (qy - SY0) * g.RS;
    const int nrow = (qy - SY0) * g.NRS;
    for (int tx = tx_lo; tx <= tx_hi; ++tx) {
      const int qx0 = xs + kTileN * tx;
      const int bbase = srow + (qx0 - SX0) + p16 + lane_off;
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < KS; ++t)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[t], strip[bbase + g.step_off[t]], acc, 0, 0, 0);

      const int qx = qx0 + p16;
      const float nc = nstrip[nrow + (qx - SX0)];  // +inf outside the valid positions
      const int jg = qy * g.W + qx;
      const int xrel = qx - rxw;
      bool added = false;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float d = nr[v] + nc - 2.f * acc[v];
        const bool pass = yin && abs(xrel - g.s * v) <= g.r && d < th[v];
        const unsigned long long m = __ballot(pass);
        if (m) {
          const unsigned long long gm = m & grp_bits;
          if (pass) {
            const int pos = cnt[v] + __popcll(gm & below);
            buf[(4 * gp + v) * g.CAP + pos] = Entry{d, jg};
          }
          cnt[v] += __popcll(gm);
          added = true;
        }
      }
      if (added) {
        const int lim = g.CAP - 16;
        if (__any(cnt[0] > lim || cnt[1] > lim || cnt[2] > lim || cnt[3] > lim)) flush();
      }
    }
  }
  flush();

#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (gp <= a_max && v <= b_max) {
      const size_t ref = (size_t)(RYw + gp) * g.nrx + (RXw + v);
#pragma unroll
      for (int q = 0; q < KR; ++q) {
        const int e = 16 * q + p16;
        if (e < g.K) {
          const bool none = Lj[v][q] == kNoIndex;
          out_idx[ref * g.K + e] = none ? -1 : Lj[v][q];
          out_dist[ref * g.K + e] = none ? INFINITY : fmaxf(Ld[v][q], 0.f);
        }
      }
    }
  }
}

// ---- instantiation table --------------------------------------------------------------
typedef void (*XcKernel)(const float*, const float*, int*, float*, const XcGeom);

template <int KS>
static XcKernel pick_kr(int kr) {
  switch (kr) {
    case 1: return xcorr_topk_f32<KS, 1>;
    case 2: return xcorr_topk_f32<KS, 2>;
    case 4: return xcorr_topk_f32<KS, 4>;
  }
  return nullptr;
}

// Step-count buckets compiled for the float32 form (extra steps are zero-padded).
int f32_step_bucket(int ks) {
  static const int b[] = {4, 8, 9, 12, 16, 18, 24, 27, 32, 36, 48, 64};
  for (int x : b)
    if (ks <= x) return x;
  return -1;
}

XcKernel f32_kernel(int ks_bucket, int kr) {
  switch (ks_bucket) {
    case 4: return pick_kr<4>(kr);
    case 8: return pick_kr<8>(kr);
    case 9: return pick_kr<9>(kr);
    case 12: return pick_kr<12>(kr);
    case 16: return pick_kr<16>(kr);
    case 18: return pick_kr<18>(kr);
    case 24: return pick_kr<24>(kr);
    case 27: return pick_kr<27>(kr);
    case 32: return pick_kr<32>(kr);
    case 36: return pick_kr<36>(kr);
    case 48: return pick_kr<48>(kr);
    case 64: return pick_kr<64>(kr);
  }
  return nullptr;
}

hipError_t launch_xcorr_f32(int ks_bucket, int kr, const float* img, const float* nrm, int* idx,
                            float* dist, const XcGeom& g, hipStream_t stream) {
  XcKernel k = f32_kernel(ks_bucket, kr);
  if (!k) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, g.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(g.nwg_total), dim3(64 * g.WY * g.WX), g.lds_bytes, stream, img, nrm,
                     idx, dist, g);
  return hipGetLastError();
}

}  // namespace bmk
