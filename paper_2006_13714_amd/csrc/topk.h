// Wavefront-shuffle top-K for the fused BM kernels (gfx950, wave64).
//
// Theorem 1 (Euclidean branch) keeps, for each reference, the support of the K largest
// b_i = vec(C_i) - h(.)h/2, which is the set of the K smallest distances.  Here each
// reference owns one 16-lane group of a wavefront.  Its current best list of 16*KR entries
// lives in KR register pairs (distance, candidate index) of that group: element e = 16*r + p
// sits in register r of lane p, sorted ascending by the key (d, j), a strict total order
// because j is unique per reference.  New candidates arrive in batches of 16 (one per lane),
// are sorted by a bitonic network and merged into the list by bitonic merges; the 16 largest
// of (last list register, batch) are dropped.  Unused slots hold (+inf, INT_MAX).
//
// Lane exchanges inside a 16-lane row use DPP only (xor 1, 2: quad permutes; xor 4: row
// rotates by 4 and 12 selected by lane bit 2; xor 8: row rotate by 8; xor 15: row mirror),
// so the networks run at VALU speed instead of paying LDS-crossbar latency per stage.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmk {

constexpr int kNoIndex = 0x7fffffff;

template <int M>
__device__ __forceinline__ int xor_lane(int v) {
  if constexpr (M == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  else if constexpr (M == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  else if constexpr (M == 4) {
    // row_ror:N reads lane (i - N) mod 16 of the row
    const int lo = __builtin_amdgcn_mov_dpp(v, 0x12C, 0xF, 0xF, false);  // lane i + 4
    const int hi = __builtin_amdgcn_mov_dpp(v, 0x124, 0xF, 0xF, false);  // lane i - 4
    return (threadIdx.x & 4) ? hi : lo;
  }
  else if constexpr (M == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
  else return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);  // M == 15
}

template <int M>
__device__ __forceinline__ float xor_lane(float v) {
  return __int_as_float(xor_lane<M>(__float_as_int(v)));
}

__device__ __forceinline__ bool key_less(float ad, int aj, float bd, int bj) {
  return (ad < bd) | ((ad == bd) & (aj < bj));
}

// Compare-exchange with the lane at xor distance M inside a 16-lane row.  The two keys are
// distinct or the two entries are identical (j is unique per reference; padding entries are
// all (+inf, INT_MAX)), so "keep the smaller" takes the partner exactly when the partner's
// key is smaller, and "keep the larger" exactly when it is not: one comparison chain and a
// mask comparison instead of two chains and a select between them.
template <int M>
__device__ __forceinline__ void cmpx(float& d, int& j, bool keep_min) {
  const float pd = xor_lane<M>(d);
  const int pj = xor_lane<M>(j);
  const bool take = key_less(pd, pj, d, j) == keep_min;
  d = take ? pd : d;
  j = take ? pj : j;
}

template <int K, int M>
__device__ __forceinline__ void sort_stage(float& d, int& j, int p, bool asc) {
  const bool blk_asc = ((p & K) == 0) == asc;  // K == 16: a single block, direction `asc`
  cmpx<M>(d, j, ((p & M) == 0) == blk_asc);
}

// Sort 16 entries (one per lane of the row); ascending if `asc`.
__device__ __forceinline__ void sort16(float& d, int& j, int p, bool asc) {
  sort_stage<2, 1>(d, j, p, asc);
  sort_stage<4, 2>(d, j, p, asc);
  sort_stage<4, 1>(d, j, p, asc);
  sort_stage<8, 4>(d, j, p, asc);
  sort_stage<8, 2>(d, j, p, asc);
  sort_stage<8, 1>(d, j, p, asc);
  sort_stage<16, 8>(d, j, p, asc);
  sort_stage<16, 4>(d, j, p, asc);
  sort_stage<16, 2>(d, j, p, asc);
  sort_stage<16, 1>(d, j, p, asc);
}

// Turn a bitonic sequence of 16 into ascending order.
__device__ __forceinline__ void bitonic_merge16(float& d, int& j, int p) {
  cmpx<8>(d, j, (p & 8) == 0);
  cmpx<4>(d, j, (p & 4) == 0);
  cmpx<2>(d, j, (p & 2) == 0);
  cmpx<1>(d, j, (p & 1) == 0);
}

// Merge a batch (cd, cj), one entry per lane, into the sorted list (Ld, Lj)[KR].
template <int KR>
__device__ __forceinline__ void merge_batch(float (&Ld)[KR], int (&Lj)[KR], float cd, int cj,
                                            int p) {
  sort16(cd, cj, p, /*asc=*/false);
  {
    // 16 smallest of (last list register, batch): the elementwise minimum of an ascending
    // and a descending run is bitonic.
    const bool lt = key_less(Ld[KR - 1], Lj[KR - 1], cd, cj);
    float sd = lt ? Ld[KR - 1] : cd;
    int sj = lt ? Lj[KR - 1] : cj;
    bitonic_merge16(sd, sj, p);
    cd = sd;
    cj = sj;
  }
#pragma unroll
  for (int r = 0; r < KR - 1; ++r) {
    // merge two ascending runs of 16: the low half stays in register r, the high half
    // carries on to the next register
    const float rd = xor_lane<15>(cd);
    const int rj = xor_lane<15>(cj);
    const bool lt = key_less(Ld[r], Lj[r], rd, rj);
    float lo_d = lt ? Ld[r] : rd, hi_d = lt ? rd : Ld[r];
    int lo_j = lt ? Lj[r] : rj, hi_j = lt ? rj : Lj[r];
    bitonic_merge16(lo_d, lo_j, p);
    bitonic_merge16(hi_d, hi_j, p);
    Ld[r] = lo_d;
    Lj[r] = lo_j;
    cd = hi_d;
    cj = hi_j;
  }
  Ld[KR - 1] = cd;
  Lj[KR - 1] = cj;
}

// Sort a list of 16 * KR entries (KR <= 2) by (d, j) ascending: element e = 16 r + p in
// register r of lane p.  Used where a monotone map of sorted keys can create equal values
// whose indices are then out of order.
template <int KR>
__device__ __forceinline__ void sort_list(float (&d)[KR], int (&j)[KR], int p) {
  static_assert(KR == 1 || KR == 2, "lists of 16 or 32");
  if constexpr (KR == 1) {
    sort16(d[0], j[0], p, true);
  } else {
    sort16(d[0], j[0], p, true);
    sort16(d[1], j[1], p, false);
    // ascending against descending: the lane-wise smaller entries are the 16 smallest,
    // and both halves are bitonic
    const bool lt = key_less(d[0], j[0], d[1], j[1]);
    const float lo_d = lt ? d[0] : d[1], hi_d = lt ? d[1] : d[0];
    const int lo_j = lt ? j[0] : j[1], hi_j = lt ? j[1] : j[0];
    d[0] = lo_d, j[0] = lo_j, d[1] = hi_d, j[1] = hi_j;
    bitonic_merge16(d[0], j[0], p);
    bitonic_merge16(d[1], j[1], p);
  }
}

// ---- distance-only networks (no indices): used to bound the K-th distance ------------
// Distances only: min or max by a compare and a select (no NaN ever reaches these networks,
// so the min/max of the IEEE functions and their operand canonicalisation are not needed).
template <int M>
__device__ __forceinline__ void cmpx_d(float& d, bool keep_min) {
  const float pd = xor_lane<M>(d);
  d = ((pd < d) == keep_min) ? pd : d;
}

template <int K, int M>
__device__ __forceinline__ void sort_stage_d(float& d, int p, bool asc) {
  const bool blk_asc = ((p & K) == 0) == asc;
  cmpx_d<M>(d, ((p & M) == 0) == blk_asc);
}

__device__ __forceinline__ void sort16_d(float& d, int p, bool asc) {
  sort_stage_d<2, 1>(d, p, asc);
  sort_stage_d<4, 2>(d, p, asc);
  sort_stage_d<4, 1>(d, p, asc);
  sort_stage_d<8, 4>(d, p, asc);
  sort_stage_d<8, 2>(d, p, asc);
  sort_stage_d<8, 1>(d, p, asc);
  sort_stage_d<16, 8>(d, p, asc);
  sort_stage_d<16, 4>(d, p, asc);
  sort_stage_d<16, 2>(d, p, asc);
  sort_stage_d<16, 1>(d, p, asc);
}

__device__ __forceinline__ void bitonic_merge16_d(float& d, int p) {
  cmpx_d<8>(d, (p & 8) == 0);
  cmpx_d<4>(d, (p & 4) == 0);
  cmpx_d<2>(d, (p & 2) == 0);
  cmpx_d<1>(d, (p & 1) == 0);
}

// Keep the 16*KR smallest of (list, batch), sorted; distances only.
template <int KR>
__device__ __forceinline__ void merge_batch_d(float (&L)[KR], float c, int p) {
  sort16_d(c, p, false);
  float m = fminf(L[KR - 1], c);
  bitonic_merge16_d(m, p);
  c = m;
#pragma unroll
  for (int r = 0; r < KR - 1; ++r) {
    const float rc = xor_lane<15>(c);
    float lo = fminf(L[r], rc), hi = fmaxf(L[r], rc);
    bitonic_merge16_d(lo, p);
    bitonic_merge16_d(hi, p);
    L[r] = lo;
    c = hi;
  }
  L[KR - 1] = c;
}

// Smallest float strictly greater than x (x itself for +inf and NaN).
__device__ __forceinline__ float next_up(float x) {
  const int b = __float_as_int(x);
  if (!(x < INFINITY)) return x;
  if (x == 0.f) return __int_as_float(1);
  return __int_as_float(x > 0.f ? b + 1 : b - 1);
}

// Insert x into a lane-private ascending list of T distances (branch-free min/max chain).
template <int T>
__device__ __forceinline__ void lane_insert(float (&t)[T], float x) {
#pragma unroll
  for (int i = 0; i < T - 1; ++i) {
    const float lo = fminf(t[i], x);
    x = fmaxf(t[i], x);
    t[i] = lo;
  }
  t[T - 1] = fminf(t[T - 1], x);
}

// Merge an ascending run of 16 (one entry per lane) into the sorted list: the same
// network as merge_batch without the initial sort.
template <int KR>
__device__ __forceinline__ void merge_sorted(float (&Ld)[KR], int (&Lj)[KR], float cd, int cj,
                                             int p) {
  cd = xor_lane<15>(cd);  // descending
  cj = xor_lane<15>(cj);
  {
    const bool lt = key_less(Ld[KR - 1], Lj[KR - 1], cd, cj);
    float sd = lt ? Ld[KR - 1] : cd;
    int sj = lt ? Lj[KR - 1] : cj;
    bitonic_merge16(sd, sj, p);
    cd = sd;
    cj = sj;
  }
#pragma unroll
  for (int r = 0; r < KR - 1; ++r) {
    const float rd = xor_lane<15>(cd);
    const int rj = xor_lane<15>(cj);
    const bool lt = key_less(Ld[r], Lj[r], rd, rj);
    float lo_d = lt ? Ld[r] : rd, hi_d = lt ? rd : Ld[r];
    int lo_j = lt ? Lj[r] : rj, hi_j = lt ? rj : Lj[r];
    bitonic_merge16(lo_d, lo_j, p);
    bitonic_merge16(hi_d, hi_j, p);
    Ld[r] = lo_d;
    Lj[r] = lo_j;
    cd = hi_d;
    cj = hi_j;
  }
  Ld[KR - 1] = cd;
  Lj[KR - 1] = cj;
}

// Distance of list element K-1 (the admission threshold), broadcast within the row.
template <int KR>
__device__ __forceinline__ float kth_distance(const float (&Ld)[KR], int K) {
  const int r = (K - 1) >> 4;
  const int p = (K - 1) & 15;
  float v = Ld[0];
#pragma unroll
  for (int q = 1; q < KR; ++q)
    if (q == r) v = Ld[q];
  return __shfl(v, p, 16);
}

// XCD-aware workgroup order: the hardware hands workgroup i to XCD (i mod 8); give each
// XCD a contiguous run of logical tiles so neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int i, int n) {
  const int q = n >> 3;
  if (i < (q << 3)) return (i & 7) * q + (i >> 3);
  return i;
}

}  // namespace bmk
