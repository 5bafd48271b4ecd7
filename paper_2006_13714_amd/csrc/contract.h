// Contraction policies of the specialised cross-term kernel (xcorr_fast.h): how the joint
// P x P x C patches are laid out in LDS, held in registers and contracted on the matrix cores.
//
// Both policies compute, for a tile of 16 references x 16 candidates, the cross terms
// <X_i, X_j> of Eq. (eq:selfConv) summed over channels (Sec. IV, S(.)), with a float32
// accumulator.  The strip in LDS holds one image row per channel in consecutive strip rows
// of RW 32-bit words; a tile's operand-B reads are one base register (two for the split
// forms: hi and lo planes) plus compile-time immediate offsets.
//
//  CtF32   float32 products, v_mfma_f32_16x16x4f32; a step covers a 2 x 2 pixel block of one
//          channel (lane group g holds pixel (g/2, g%2) of the block).
//  CtSplit x = hi + lo split in bfloat16 (FP16 = false) or float16 after a power-of-two
//          pre-scale (FP16 = true) on v_mfma_f32_16x16x32_{bf16,f16}.  float16: three
//          products hi*hi + hi*lo + lo*hi per element (22 significant bits; the dropped
//          lo*lo is below float32 rounding).  bfloat16: all four products, so the cross term
//          is the exact product of the rounded values hi + lo (16 significant bits), which
//          the distance assembly pairs with the norms of the same rounded values
//          (split16.h).  A lane holds a 4-row x 2-column pixel block per
//          32-element block; the strip stores, per pixel x, the 32-bit word (v[x], v[x+1])
//          of 16-bit parts, so every read is aligned.  The hi parts form one plane (rows:
//          image row, then channel) and the lo parts a second plane SH * C rows later, so the
//          four rows of an operand pair up into two-word reads of one plane and land in the
//          matrix op's operand registers without copies.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bm_internal.h"
#include "split16.h"

namespace bmk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------------------
template <int C, int H2>
struct CtF32 {
  static constexpr int RW = kFastRS;          // words per strip row
  static constexpr int ROWS = C;              // strip rows per image row
  static constexpr int CRS = ROWS * RW;       // words per image row
  static constexpr int NS = C * H2 * H2;      // steps (matrix ops) per tile
  static constexpr int NA = NS;               // operand-A registers
  static constexpr int NB = NS;               // operand-B registers per tile
  static constexpr int NACC = NS >= 32 ? 4 : 2;  // accumulators of the chain
  static constexpr bool kScaled = false;
  static constexpr bool kSplit = false;
  using AReg = float;
  using BReg = float;                          // one operand B per matrix op

  // step t = ((l2 * H2) + m2) * C + c: pixels (2*l2 + dy, 2*m2 + dx), dy, dx in {0,1}
  static constexpr int l2(int t) { return t / (H2 * C); }
  static constexpr int m2(int t) { return (t / C) % H2; }
  static constexpr int ch(int t) { return t % C; }
  static constexpr int off(int t) { return (2 * l2(t) * C + ch(t)) * RW + 2 * m2(t); }

  __device__ static int lane_off(int gp) { return (gp >> 1) * CRS + (gp & 1); }
  __device__ static int plane_off(const FastGeom&) { return 0; }  // one plane

  // strip rows (y*C + c): the centred image values, zero outside the image.  Four rows per
  // pass, loads unconditional (clamped to a valid address, masked afterwards) so they are
  // in flight together.
  __device__ static void stage(uint32_t* strip, const float* img, const FastGeom& g, int SY0,
                               int SX0, int first, int step, int lane, const float* center,
                               float) {
    const int n = g.SH * C;
    for (int row0 = first; row0 < n; row0 += 4 * step) {
      for (int x = lane; x < g.SW; x += 64) {
        const int ix = SX0 + x;
        const bool xok = (ix >= 0) & (ix < g.W);
        float v[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int row = row0 + u * step;
          const int y = row / C;
          const int c = row - y * C;
          const int iy = SY0 + y;
          ok[u] = (row < n) & (iy >= 0) & (iy < g.H) & xok;
          v[u] = img[ok[u] ? ((size_t)c * g.H + iy) * g.W + ix : 0];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int row = row0 + u * step;
          if (row < n)
            reinterpret_cast<float*>(strip)[row * RW + x] = ok[u] ? v[u] - center[row % C] : 0.f;
        }
      }
    }
  }

  // operand A for the reference whose patch starts at strip word `base` (lane offset
  // included); elements outside the P x P patch (odd P) are zero
  __device__ static void load_a(AReg (&A)[NS], const uint32_t* strip, int base, int gp, int P,
                                int = 0) {
    const float* s = reinterpret_cast<const float*>(strip);
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const bool ok = (2 * l2(t) + (gp >> 1) < P) & (2 * m2(t) + (gp & 1) < P);
      A[t] = ok ? s[base + off(t)] : 0.f;
    }
  }

  __device__ static void load_b(float (&B)[NB], const uint32_t* strip, int base, int = 0) {
    const float* s = reinterpret_cast<const float*>(strip);
#pragma unroll
    for (int t = 0; t < NB; ++t) B[t] = s[base + off(t)];
  }

  // the matrix-op chain with the next tile's reads interleaved; `nb` is their base
  __device__ static f4 chain_and_load(const AReg (&A)[NS], const float (&cur)[NB],
                                      float (&nxt)[NB], const uint32_t* strip, int nb, int = 0) {
    const float* s = reinterpret_cast<const float*>(strip);
    // NACC independent accumulators over interleaved steps, added pairwise at the end:
    // each partial sum stays a fraction of the cross term, so its roundings are smaller
    // than those of one accumulator running through all NS steps
    f4 acc[NACC];
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      acc[t % NACC] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[t], cur[t], acc[t % NACC], 0, 0, 0);
      nxt[t] = s[nb + off(t)];
    }
    if constexpr (NACC == 4) return (acc[0] + acc[1]) + (acc[2] + acc[3]);
    else return acc[0] + acc[1];
  }

  // The same chain with the candidates as the row operand: lane (g, p) receives the cross
  // terms of candidates 4 g .. 4 g + 3 of the tile with reference p.  The first accumulator
  // starts from `init`; the accumulators are returned raw and added by combine() one tile
  // later, so nothing waits for the matrix ops here.
  static constexpr int NACC_T = NACC;
  static constexpr bool kInitInChain = true;
  // the bounding sweep runs the same chain (bit-identical distances): no inflation
  static constexpr bool kBoundChain = false;
  static constexpr float kBoundRel = 0.f, kBoundAbs = 0.f;
  template <bool BOUND = false>
  __device__ static void chain_t(const AReg (&A)[NS], const float (&cur)[NB], float (&nxt)[NB],
                                 const uint32_t* strip, int nb, int, const f4& init,
                                 f4 (&acc)[NACC_T]) {
    const float* s = reinterpret_cast<const float*>(strip);
    acc[0] = init;
#pragma unroll
    for (int q = 1; q < NACC; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      acc[t % NACC] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[t], A[t], acc[t % NACC], 0, 0, 0);
      nxt[t] = s[nb + off(t)];
    }
  }
  __device__ static f4 combine(const f4 (&acc)[NACC_T]) {
    if constexpr (NACC == 4) return (acc[0] + acc[1]) + (acc[2] + acc[3]);
    else return acc[0] + acc[1];
  }

  template <bool BOUND = false>
  __device__ static void schedule() {
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix op
      __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // up to two vector ops
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
    }
  }
};

// ---------------------------------------------------------------------------------------
template <bool FP16>
__device__ __forceinline__ void split2(float v, uint32_t& hi, uint32_t& lo) {
  if constexpr (FP16) {
    const _Float16 h = (_Float16)v;
    const _Float16 l = (_Float16)(v - (float)h);
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, l);
  } else {
    hi = bf16_rne_bits(v);
    const float hf = __uint_as_float(hi << 16);
    lo = bf16_rne_bits(v - hf);
  }
}

template <int C, int H2, bool FP16>
struct CtSplit {
  static constexpr int RW = split_rw(C);
  static constexpr int ROWS = C;              // per image row and plane: channel c -> row c
  static constexpr int CRS = ROWS * RW;
  static constexpr int PE = 2 * H2;
  static constexpr int NRB = (PE + 3) / 4;    // 4-row blocks
  static constexpr int NCB = (PE + 7) / 8;    // 8-column blocks
  static constexpr int NKB = C * NRB * NCB;   // 32-element blocks
  static constexpr bool kLL = !FP16;          // bfloat16: lo*lo as a fourth product
  static constexpr int NS = (kLL ? 4 : 3) * NKB;  // matrix ops per tile
  static constexpr int NA = 2 * NKB;          // operand-A vectors (hi, lo per block)
  static constexpr int NB = 2 * NKB;          // operand-B vectors per tile (hi, lo per block)
  static constexpr bool kScaled = FP16;
  static constexpr bool kSplit = true;
  using AReg = u4;                            // 8 x 16-bit parts
  using BReg = u4;                            // held as whole 4-word vectors, so the reads
                                              // land in the matrix op's operand registers

  // block b = ((rb * NCB) + cb) * C + c; word i of block b (in either plane): image row
  // 4*rb + i, columns 8*cb + 2*g, +1 of channel c
  static constexpr int rb(int b) { return b / (NCB * C); }
  static constexpr int cb(int b) { return (b / C) % NCB; }
  static constexpr int ch(int b) { return b % C; }
  static constexpr int woff(int b, int i) {
    return ((4 * rb(b) + i) * ROWS + ch(b)) * RW + 8 * cb(b);
  }

  __device__ static int lane_off(int gp) { return 2 * gp; }
  // words from the hi plane to the lo plane
  __device__ static int plane_off(const FastGeom& g) { return g.SH * CRS; }

  // Strip word x of a row = (v[x], v[x+1]) of the row's 16-bit parts (the pixel pair that
  // starts at x), zero outside the image and past the strip width.  Lane x stages word x
  // (the strip width is at most 64 words): it loads and splits pixel x once and takes the
  // parts of pixel x+1 from lane x+1 (a wave-wide DPP shift; the last lane gets zeros).
  // Four rows per pass, loads unconditional (clamped to a valid address, masked
  // afterwards) so they are in flight together.
  __device__ static void stage(uint32_t* strip, const float* img, const FastGeom& g, int SY0,
                               int SX0, int first, int step, int lane, const float* center,
                               float scale) {
    const int n = g.SH * C;
    const int lo_plane = g.SH * CRS;
    const int x = lane;
    const int ix = SX0 + x;
    const bool xok = (x < g.SW) & (ix >= 0) & (ix < g.W);
    for (int row0 = first; row0 < n; row0 += 4 * step) {
      float v[4];
      bool ok[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = row0 + u * step;
        const int y = row / C;
        const int c = row - y * C;
        const int iy = SY0 + y;
        ok[u] = (row < n) & (iy >= 0) & (iy < g.H) & xok;
        v[u] = img[ok[u] ? ((size_t)c * g.H + iy) * g.W + ix : 0];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = row0 + u * step;
        const float val = ok[u] ? (v[u] - center[row % C]) * scale : 0.f;
        uint32_t h0, l0;
        split2<FP16>(val, h0, l0);
        // DPP wave_shl:1 -- lane i reads lane i + 1; lane 63 keeps the zero
        const uint32_t h1 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)h0, 0x130, 0xF, 0xF, false);
        const uint32_t l1 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)l0, 0x130, 0xF, 0xF, false);
        if ((row < n) & (x < g.SW)) {
          const int y = row / C;
          const int c = row - y * C;
          uint32_t* dhi = strip + (y * ROWS + c) * RW;
          dhi[x] = h0 | (h1 << 16);
          dhi[lo_plane + x] = l0 | (l1 << 16);
        }
      }
    }
  }

  // operand A: per block, hi words then lo words; halves outside the P x P patch are zero
  __device__ static void load_a(AReg (&A)[2 * NKB], const uint32_t* strip, int base, int gp,
                                int P, int lo) {
#pragma unroll
    for (int b = 0; b < NKB; ++b) {
      const int c0 = 8 * cb(b) + 2 * gp;
      const uint32_t keep = (c0 < P ? 0xFFFFu : 0u) | (c0 + 1 < P ? 0xFFFF0000u : 0u);
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        const uint32_t* pl = strip + base + (part ? lo : 0);
        u4 w;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool rok = 4 * rb(b) + i < P;
          w[i] = rok ? (pl[woff(b, i)] & keep) : 0u;
        }
        A[2 * b + part] = w;
      }
    }
  }

  __device__ static void load_b(u4 (&B)[NB], const uint32_t* strip, int base, int lo) {
    const uint32_t* sh = strip + base;
    const uint32_t* sl = strip + base + lo;
#pragma unroll
    for (int b = 0; b < NKB; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        B[2 * b][i] = sh[woff(b, i)];
        B[2 * b + 1][i] = sl[woff(b, i)];
      }
  }

  __device__ static f4 mfma(const u4& a, const u4& b, const f4& c) {
    if constexpr (FP16)
      return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a),
                                                    __builtin_bit_cast(h8, b), c, 0, 0, 0);
    else
      return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                     __builtin_bit_cast(bf8, b), c, 0, 0, 0);
  }

  __device__ static f4 chain_and_load(const AReg (&A)[2 * NKB], const u4 (&cur)[NB],
                                      u4 (&nxt)[NB], const uint32_t* strip, int nb, int lo) {
    const uint32_t* sh = strip + nb;
    const uint32_t* sl = strip + nb + lo;
    // The small products first, then hi * hi: the accumulator only reaches the size of the
    // cross term in the last NKB ops, so fewer roundings happen at that size.
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < NKB; ++b) {
      if constexpr (kLL) acc = mfma(A[2 * b + 1], cur[2 * b + 1], acc);  // lo * lo
      acc = mfma(A[2 * b], cur[2 * b + 1], acc);      // hi * lo
      acc = mfma(A[2 * b + 1], cur[2 * b], acc);      // lo * hi
#pragma unroll
      for (int i = 0; i < 4; ++i) nxt[2 * b][i] = sh[woff(b, i)];
#pragma unroll
      for (int i = 0; i < 4; ++i) nxt[2 * b + 1][i] = sl[woff(b, i)];
    }
#pragma unroll
    for (int b = 0; b < NKB; ++b) acc = mfma(A[2 * b], cur[2 * b], acc);  // hi * hi
    return acc;
  }

  // The same chain with the candidates as the row operand: lane (g, p) receives the cross
  // terms of candidates 4 g .. 4 g + 3 of the tile with reference p.  The chain starts
  // from zero (small products first, as above); the caller adds its starting value one
  // tile later, so nothing waits for the matrix ops here.
  //
  // BOUND (bfloat16 only): the bounding sweep's shorter chain, without lo * lo.  The values
  // v = hi + lo of the bfloat16 form have |lo| <= 2^-8 (1 + 2^-7) |v|, so by Cauchy-Schwarz
  // and ||v_i|| ||v_j|| <= (V_i + V_j) / 2 (V = ||v||^2, the norm map's value) the dropped
  // products sum to at most 2^-17 (1 + 2^-6) (V_i + V_j); the float32 accumulation of each
  // chain (at most 4 n <= 1024 roundings of sums of products bounded as above) errs by at
  // most 2^-15 (1 + 2^-6) (V_i + V_j).  A distance d = ... - 2 C therefore moves by less
  // than 2^-12.8 (V_i + V_j) < kBoundRel (V_i + V_j), which the bounding sweep adds to its
  // distances.  (For float16 the one product hi * hi
  // needs a margin of about 2^-10 (V_i + V_j), which admitted more candidates than the
  // saved products gained: it keeps the selecting sweep's chain.)
  static constexpr int NACC_T = 1;
  static constexpr bool kInitInChain = false;
  static constexpr bool kBoundChain = kLL;
  static constexpr float kBoundRel = kLL ? 0x1p-12f : 0.f;
  static constexpr float kBoundAbs = 0.f;
  template <bool BOUND = false>
  __device__ static void chain_t(const AReg (&A)[2 * NKB], const u4 (&cur)[NB], u4 (&nxt)[NB],
                                 const uint32_t* strip, int nb, int lo, const f4&,
                                 f4 (&out)[NACC_T]) {
    const uint32_t* sh = strip + nb;
    const uint32_t* sl = strip + nb + lo;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < NKB; ++b) {
      if constexpr (kLL && !BOUND) acc = mfma(cur[2 * b + 1], A[2 * b + 1], acc);  // lo * lo
      acc = mfma(cur[2 * b + 1], A[2 * b], acc);      // hi (reference) * lo (candidate)
      acc = mfma(cur[2 * b], A[2 * b + 1], acc);      // lo * hi
#pragma unroll
      for (int i = 0; i < 4; ++i) nxt[2 * b][i] = sh[woff(b, i)];
#pragma unroll
      for (int i = 0; i < 4; ++i) nxt[2 * b + 1][i] = sl[woff(b, i)];
    }
#pragma unroll
    for (int b = 0; b < NKB; ++b) acc = mfma(cur[2 * b], A[2 * b], acc);  // hi * hi
    out[0] = acc;
  }
  __device__ static f4 combine(const f4 (&acc)[NACC_T]) { return acc[0]; }

  template <bool BOUND = false>
  __device__ static void schedule() {
    constexpr int NSB = (BOUND && kLL) ? 3 * NKB : NS;  // matrix ops of the chain
#pragma unroll
    for (int t = 0; t < NSB; ++t) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix op
      __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // up to two vector ops
      __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);  // up to three LDS reads
    }
  }
};

}  // namespace bmk
