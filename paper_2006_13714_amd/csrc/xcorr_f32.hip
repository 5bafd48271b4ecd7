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
//  * Software pipeline: operand B is double-buffered in registers; the LDS reads of the next
//    tile are issued before the matrix-op chain of the current one.
//  * Epilogue: each lane holds 4 references x 1 candidate and assembles d in float32 with
//    the window mask.  Selection takes two sweeps with bit-identical arithmetic.  Sweep 1
//    keeps, per lane, a branch-free min/max list of its smallest distances; the K-th
//    smallest over the 16 lanes of a reference bounds that reference's K-th distance from
//    above.  Sweep 2 appends only candidates under the bound (about K per reference) to a
//    per-reference LDS buffer via ballot/popcount compaction, and the wavefront-shuffle
//    bitonic networks of topk.h merge them into the sorted (d, j) lists.
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
               const float* __restrict__ centers, int* __restrict__ out_idx,
               float* __restrict__ out_dist, const XcGeom g) {
  extern __shared__ __align__(16) unsigned char lds[];
  float* strip = reinterpret_cast<float*>(lds + g.lds_strip_off);
  float* nstrip = reinterpret_cast<float*>(lds + g.lds_norm_off);
  Entry* buf_all = reinterpret_cast<Entry*>(lds + g.lds_buf_off);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
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
    const bool yok = (iy >= 0) & (iy < g.H);
    const float cc = centers ? centers[c] : 0.f;  // centring constant
    const float* src = img + ((size_t)c * g.H + (yok ? iy : 0)) * g.W;
    float* dst = strip + c * g.PLANE + y * g.RS;
    for (int x = lane; x < g.SW; x += 64) {
      const int ix = SX0 + x;
      dst[x] = (yok & (ix >= 0) & (ix < g.W)) ? src[ix] - cc : 0.f;
    }
  }
  for (int y = wave; y < g.NH; y += nwaves) {
    const int qy = SY0 + y;
    const bool yok = (qy >= 0) & (qy < g.Hv);
    const float* src = nrm + (size_t)(yok ? qy : 0) * g.Wv;
    float* dst = nstrip + y * g.NRS;
    for (int x = lane; x < g.NW; x += 64) {
      const int qx = SX0 + x;
      dst[x] = (yok & (qx >= 0) & (qx < g.Wv)) ? src[qx] : INFINITY;
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
    const bool ok = (gp <= a_max) & (v <= b_max);
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

  // scalars the inner loops use (kept out of the kernel-argument struct so that nothing
  // takes its address)
  const int s = g.s, r = g.r, CAP = g.CAP, K = g.K, W = g.W, NRS = g.NRS, RS = g.RS;
  const int wsp = g.wspan;  // window offsets -r .. -r + wsp
  constexpr int TL = 2 * KR;  // per-lane list length of the bounding pass
  const int qy_lo = max(0, ryw - r);
  const int qy_hi = min(g.Hv - 1, ryw + s * a_max - r + wsp);
  const int xs = rxw - r;  // first tile start (unclipped)
  const int nt = (s * b_max + wsp + 1 + kTileN - 1) / kTileN;
  const int tx_lo = xs < -(kTileN - 1) ? (-xs) / kTileN : 0;
  const int tx_hi = min(nt - 1, (g.Wv - 1 - xs) / kTileN);
  const int n_tx = tx_hi - tx_lo + 1;
  const int n_tiles = (qy_hi - qy_lo + 1) * n_tx;
  const unsigned long long grp_bits = 0xFFFFull << (16 * gp);
  const unsigned long long below = (1ull << lane) - 1ull;
  const int lim = CAP - 16;
  int soff[KS];
#pragma unroll
  for (int t = 0; t < KS; ++t) soff[t] = g.step_off[t];
  const int bcol0 = (xs - SX0) + p16 + lane_off;  // operand B: lane offset inside a row
  const float* nbase = nstrip + (xs - SX0) + p16;

  auto flush = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      for (int ch = 0; __any(ch * 16 < cnt[v]); ++ch) {
        const int e = ch * 16 + p16;
        float cd = INFINITY;
        int cj = kNoIndex;
        if (e < cnt[v]) {
          const Entry x = buf[(4 * gp + v) * CAP + e];
          cd = x.d;
          cj = x.j;
        }
        merge_batch<KR>(Ld[v], Lj[v], cd, cj, p16);
      }
      cnt[v] = 0;
      // never loosen: a list that is not yet full has K-th distance +inf (padding
      // references keep -inf)
      th[v] = fminf(th[v], kth_distance<KR>(Ld[v], K));
    }
  };

  // Pass-2 epilogue, split into a branch-free part (distances, window mask, admission test)
  // that is interleaved with the next tile's matrix ops, and a commit part (ballot,
  // compaction into the buffers, merges) that branches.
  struct Admit {
    float d[4];
    bool pass[4];
  };
  auto admit = [&](const f4& acc, int qy, int tx) __attribute__((always_inline)) {
    Admit a;
    const float nc = nbase[(qy - SY0) * NRS + kTileN * tx];  // +inf off the valid range
    const int xrel = xs + kTileN * tx + p16 - rxw;
    const bool yin = (unsigned)(qy - ryw - s * gp + r) <= (unsigned)wsp;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      a.d[v] = fmaf(-2.f, acc[v], nr[v] + nc);
      a.pass[v] = yin & ((unsigned)(xrel - s * v + r) <= (unsigned)wsp) & (a.d[v] < th[v]);
    }
    return a;
  };
  auto commit = [&](const Admit& a, int qy, int tx) __attribute__((always_inline)) {
    if (__any(a.pass[0] | a.pass[1] | a.pass[2] | a.pass[3])) {
      const int jg = qy * W + xs + kTileN * tx + p16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const unsigned long long m = __ballot(a.pass[v]);
        if (m) {
          const unsigned long long gm = m & grp_bits;
          if (a.pass[v]) {
            const int pos = cnt[v] + __popcll(gm & below);
            buf[(4 * gp + v) * CAP + pos] = Entry{a.d[v], jg};
          }
          cnt[v] += __popcll(gm);
        }
      }
      if (__any((cnt[0] > lim) | (cnt[1] > lim) | (cnt[2] > lim) | (cnt[3] > lim))) flush();
    }
  };

  // One sweep over this wave's candidate tiles, software-pipelined: while the matrix ops
  // of tile it run, the wave computes the branch-free epilogue of tile it-1 and issues the
  // LDS reads of tile it+1 (the scheduling groups interleave one matrix op, a few vector
  // ops and one LDS read).  The last iteration runs the chain on a clamped (in-bounds)
  // repeat of the final tile whose result is discarded.
  auto sweep = [&](auto&& arith, auto&& post) __attribute__((always_inline)) {
    if (n_tiles <= 0) return;
    int qy = qy_lo, tx = tx_lo;
    auto tile_base = [&](int y, int x) __attribute__((always_inline)) {
      return (min(y, qy_hi) - SY0) * RS + bcol0 + kTileN * x;
    };
    float b[KS];
    f4 acc_prev = {0.f, 0.f, 0.f, 0.f};
    {
      const int bb = tile_base(qy, tx);
#pragma unroll
      for (int t = 0; t < KS; ++t) b[t] = strip[bb + soff[t]];
#pragma unroll
      for (int t = 0; t < KS; ++t)
        acc_prev = __builtin_amdgcn_mfma_f32_16x16x4f32(A[t], b[t], acc_prev, 0, 0, 0);
    }
    int pqy = qy, ptx = tx;
    auto advance = [&]() __attribute__((always_inline)) {
      if (++tx > tx_hi) {
        tx = tx_lo;
        ++qy;
      }
    };
    advance();
    {
      const int bb = tile_base(qy, tx);
#pragma unroll
      for (int t = 0; t < KS; ++t) b[t] = strip[bb + soff[t]];
    }
    // one pipeline step: matrix ops of the tile whose operands are in `cur`, the epilogue
    // arithmetic of the previous tile, and the LDS reads of the next tile into `nxt`
    auto step = [&](float (&cur)[KS], float (&nxt)[KS]) __attribute__((always_inline)) {
      __builtin_amdgcn_sched_barrier(0);  // keep each step its own scheduling region
      const int cqy = qy, ctx = tx;
      advance();
      const int nb = tile_base(qy, tx);
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[t], cur[t], acc, 0, 0, 0);
        nxt[t] = strip[nb + soff[t]];
      }
      auto res = arith(acc_prev, pqy, ptx);
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix op
        __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // up to three vector ops
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
      }
      __builtin_amdgcn_sched_barrier(0);
      post(res, pqy, ptx);
      acc_prev = acc;
      pqy = cqy;
      ptx = ctx;
    };
    // unrolled by two so the operand buffers swap roles without register copies
    float b2[KS];
    int it = 1;
    for (; it + 1 <= n_tiles; it += 2) {
      step(b, b2);
      step(b2, b);
    }
    if (it <= n_tiles) step(b, b2);
  };

  // ---- pass 1: bound the K-th distance of every reference.  Each lane keeps the TL
  // smallest in-window distances it sees (distances only); those 16*TL values belong to
  // distinct candidates, so the K-th smallest of them is >= the true K-th distance.
  float tl[4][TL];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < TL; ++i) tl[v][i] = INFINITY;
  sweep(
      [&](const f4& acc, int qy, int tx) __attribute__((always_inline)) {
        const float nc = nbase[(qy - SY0) * NRS + kTileN * tx];
        const int xrel = xs + kTileN * tx + p16 - rxw;
        const bool yin = (unsigned)(qy - ryw - s * gp + r) <= (unsigned)wsp;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float d = fmaf(-2.f, acc[v], nr[v] + nc);
          lane_insert<TL>(tl[v], (yin & ((unsigned)(xrel - s * v + r) <= (unsigned)wsp)) ? d : INFINITY);
        }
        return 0;
      },
      [&](int, int, int) __attribute__((always_inline)) {});
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    float L[KR];
#pragma unroll
    for (int q = 0; q < KR; ++q) L[q] = INFINITY;
#pragma unroll
    for (int i = 0; i < TL; ++i) merge_batch_d<KR>(L, tl[v][i], p16);
    const float bound = kth_distance<KR>(L, K);
    // strict "<" against the next float up admits exactly the candidates with d <= bound
    th[v] = (th[v] == -INFINITY) ? -INFINITY : next_up(bound);
  }

  // ---- pass 2: identical distances; candidates with d <= bound go to the buffers.  A
  // merge (flush) lowers the threshold to the list's K-th distance; from then on every
  // listed candidate precedes the rest in j, so the strict test stays exact.
  sweep(admit, commit);
  flush();

#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if ((gp <= a_max) & (v <= b_max)) {
      const size_t ref = (size_t)(RYw + gp) * g.nrx + (RXw + v);
#pragma unroll
      for (int q = 0; q < KR; ++q) {
        const int e = 16 * q + p16;
        if (e < K) {
          const bool none = Lj[v][q] == kNoIndex;
          out_idx[ref * K + e] = none ? -1 : Lj[v][q];
          out_dist[ref * K + e] = none ? INFINITY : fmaxf(Ld[v][q], 0.f);
        }
      }
    }
  }
}

// ---- instantiation table --------------------------------------------------------------
typedef void (*XcKernel)(const float*, const float*, const float*, int*, float*, const XcGeom);

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

// Allow the kernel the dynamic LDS of its tile (done once, at plan time).
hipError_t prepare_xcorr_f32(int ks_bucket, int kr, int lds_bytes) {
  XcKernel k = f32_kernel(ks_bucket, kr);
  if (!k) return hipErrorInvalidValue;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

hipError_t launch_xcorr_f32(int ks_bucket, int kr, const float* img, const float* nrm,
                            const float* centers, int* idx, float* dist, const XcGeom& g,
                            hipStream_t stream) {
  XcKernel k = f32_kernel(ks_bucket, kr);
  if (!k) return hipErrorInvalidValue;
  (void)hipGetLastError();  // a stale status (e.g. a query's not-ready) must not read as a launch failure
  hipLaunchKernelGGL(k, dim3(g.nwg_total), dim3(64 * g.WY * g.WX), g.lds_bytes, stream, img, nrm,
                     centers, idx, dist, g);
  return hipGetLastError();
}

}  // namespace bmk
