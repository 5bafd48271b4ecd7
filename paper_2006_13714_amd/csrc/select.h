// Per-reference selection state of the fused BM kernels (gfx950, wave64).
//
// Layout: a wave owns a 4 x 4 block of references; after a 16 x 16 matrix tile each lane
// holds the cross terms of references (row gp = lane/16, column v = 0..3) of its block
// against one candidate (lane % 16).  This struct keeps everything those 4 references
// need in that lane: their squared norms, admission thresholds, the bounding-pass lists,
// the LDS candidate buffers and the sorted (d, j) lists of topk.h.
//
// Selection (Theorem 1, Euclidean branch: keep the K smallest distances) runs in two
// sweeps over the candidates with bit-identical arithmetic:
//  1. bound: each lane keeps its TL = 2*KR smallest in-window distances (branch-free
//     min/max chain).  The 16*TL values of a reference come from distinct candidates, so
//     their K-th smallest is >= the reference's true K-th distance.
//  2. select: candidates with d <= bound are compacted (ballot + popcount) into a
//     per-reference LDS buffer and merged into the sorted list; a merge lowers the
//     threshold to the list's K-th distance.  Candidates reach a reference in increasing
//     j, so once the list is full a strict "d < K-th" test is exact for the (d, j) order.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "topk.h"

namespace bmk {

typedef float f4 __attribute__((ext_vector_type(4)));

struct Entry {
  float d;
  int j;
};

struct Admit {
  float d[4];
  bool pass[4];
};

// Wave-wide vote into a scalar register pair (a uniform branch on it needs no vector op).
__device__ __forceinline__ unsigned long long vote(bool p) {
  return __builtin_amdgcn_ballot_w64(p);
}

template <int KR>
struct RefSelect {
  static constexpr int TL = 2 * KR;
  float nr[4];   // squared norms of the 4 references
  float th[4];   // admission threshold (strict); -inf for padding references
  int cnt[4];    // entries waiting in each reference's buffer
  float Ld[4][KR];
  int Lj[4][KR];
  float tl[4][TL];
  Entry* buf;    // this wave's buffers: reference (4*gp + v) at buf[(4*gp+v)*cap]
  Entry* bv[4];  // this lane's reference (4*gp + v) buffer
  int cap, K, p16, gp;
  bool ncc = false;  // outputs 2 - 2 NCC = 2 + outk[v] * key instead of the distance
  float outk[4] = {0.f, 0.f, 0.f, 0.f};
  unsigned long long grp_bits, below;

  __device__ __forceinline__ void init(Entry* wave_buf, int cap_, int K_, int lane,
                                       const float (&norms)[4], const bool (&valid)[4]) {
    buf = wave_buf;
    cap = cap_;
    K = K_;
    p16 = lane & 15;
    gp = lane >> 4;
    grp_bits = 0xFFFFull << (16 * gp);
    below = (1ull << lane) - 1ull;
#pragma unroll
    for (int v = 0; v < 4; ++v) bv[v] = buf + (4 * gp + v) * cap;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      nr[v] = norms[v];
      th[v] = valid[v] ? INFINITY : -INFINITY;
      cnt[v] = 0;
#pragma unroll
      for (int q = 0; q < KR; ++q) {
        Ld[v][q] = INFINITY;
        Lj[v][q] = kNoIndex;
      }
#pragma unroll
      for (int i = 0; i < TL; ++i) tl[v][i] = INFINITY;
    }
  }

  // distance assembly (Lemma 2): d = ||X_i||^2 + ||X_j||^2 - 2 <X_i, X_j>
  __device__ __forceinline__ float dist(const f4& acc, float nc, int v) const {
    return fmaf(-2.f, acc[v], nr[v] + nc);
  }

  // ---- sweep 1
  __device__ __forceinline__ void bound_update(const f4& acc, float nc, const bool (&inw)[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) lane_insert<TL>(tl[v], inw[v] ? dist(acc, nc, v) : INFINITY);
  }

  // threshold of reference column v from its (all-wave) lane lists
  __device__ __forceinline__ void bound_finish_col(int v) {
    float L[KR];
#pragma unroll
    for (int q = 0; q < KR; ++q) L[q] = INFINITY;
#pragma unroll
    for (int i = 0; i < TL; ++i) merge_batch_d<KR>(L, tl[v][i], p16);
    // a strict "<" against the next float up admits exactly d <= bound
    th[v] = fminf(th[v], next_up(kth_distance<KR>(L, K)));
  }

  // ---- sweep 2
  __device__ __forceinline__ Admit admit(const f4& acc, float nc, const bool (&inw)[4]) const {
    Admit a;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      a.d[v] = dist(acc, nc, v);
      a.pass[v] = inw[v] & (a.d[v] < th[v]);
    }
    return a;
  }

  __device__ __forceinline__ void flush() {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      for (int ch = 0; vote(ch * 16 < cnt[v]); ++ch) {
        const int e = ch * 16 + p16;
        float cd = INFINITY;
        int cj = kNoIndex;
        if (e < cnt[v]) {
          const Entry x = bv[v][e];
          cd = x.d;
          cj = x.j;
        }
        merge_batch<KR>(Ld[v], Lj[v], cd, cj, p16);
      }
      cnt[v] = 0;
      // never loosen: a list that is not yet full has K-th distance +inf
      th[v] = fminf(th[v], kth_distance<KR>(Ld[v], K));
    }
  }

  // Append the passing (d, j) of each reference to its buffer in lane order: a lane's slot
  // is the buffered count plus the passing lanes of its group below it (mbcnt).
  __device__ __forceinline__ void commit(const Admit& a, int jg) {
    // the votes are taken on the comparisons themselves (a.pass[v] == a.d[v] < th[v]), so
    // they stay scalar masks
    if (vote((a.d[0] < th[0]) | (a.d[1] < th[1]) | (a.d[2] < th[2]) | (a.d[3] < th[3]))) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool pass = a.d[v] < th[v];
        const unsigned long long m = vote(pass);
        if (m) {
          const unsigned long long gm = m & grp_bits;
          const unsigned lo = (unsigned)gm, hi = (unsigned)(gm >> 32);
          if (pass) {
            const int pos = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, cnt[v]));
            bv[v][pos] = Entry{a.d[v], jg};
          }
          cnt[v] = __builtin_popcount(lo) + (__builtin_popcount(hi) + cnt[v]);
        }
      }
      const int lim = cap - 16;
      if (vote((cnt[0] > lim) | (cnt[1] > lim) | (cnt[2] > lim) | (cnt[3] > lim))) flush();
    }
  }

  // Column v of the sorted lists -> outputs (distance clamped at 0, or 2 - 2 NCC clamped to
  // [0, 4]; padding -> (-1, +inf)).
  __device__ __forceinline__ void write_col(int v, int* out_idx, float* out_dist, size_t ref,
                                            bool valid) const {
    if (!valid) return;
    float o[KR];
    int oj[KR];
#pragma unroll
    for (int q = 0; q < KR; ++q) {
      const bool none = Lj[v][q] == kNoIndex;
      o[q] = none ? INFINITY
                  : (ncc ? fminf(fmaxf(fmaf(outk[v], Ld[v][q], 2.f), 0.f), 4.f)
                         : fmaxf(Ld[v][q], 0.f));
      oj[q] = Lj[v][q];
    }
    // The outputs are a monotone map of the keys (NCC: 2 - 2 NCC; Euclidean: the clamp at
    // 0), but the map can give two distinct keys the same output (NCC rounding and clamp,
    // negative Euclidean keys); sorting the outputs by (value, index) then puts the
    // smaller index first, as the output order requires.  Euclidean lists without a
    // negative key map one to one and skip it.
    bool neg = false;
#pragma unroll
    for (int q = 0; q < KR; ++q) neg |= Ld[v][q] < 0.f;
    if (ncc || vote(neg)) sort_list<KR>(o, oj, p16);
#pragma unroll
    for (int q = 0; q < KR; ++q) {
      const int e = 16 * q + p16;
      if (e < K) {
        const bool none = oj[q] == kNoIndex;
        out_idx[ref * K + e] = none ? -1 : oj[q];
        out_dist[ref * K + e] = none ? INFINITY : o[q];
      }
    }
  }

  __device__ __forceinline__ void write(int* out_idx, float* out_dist, const size_t (&ref)[4],
                                        const bool (&valid)[4]) const {
#pragma unroll
    for (int v = 0; v < 4; ++v) write_col(v, out_idx, out_dist, ref[v], valid[v]);
  }
};

// Window test for one tile: candidate row offset and candidate column offset u (both
// already shifted by +r) lie in [0, 2r] for reference column v at stride s.
__device__ __forceinline__ void window_mask(bool (&inw)[4], bool in_y, int u, int s, int r2) {
#pragma unroll
  for (int v = 0; v < 4; ++v) inw[v] = in_y & ((unsigned)(u - s * v) <= (unsigned)r2);
}

}  // namespace bmk
