// Wavefront-shuffle top-K for the fused BM kernels (gfx950, wave64).
//
// Theorem 1 (Euclidean branch) keeps, for each reference, the support of the K largest
// b_i = vec(C_i) - h(.)h/2, which is the set of the K smallest distances.  Here each
// reference owns one 16-lane group of a wavefront.  Its current best list of 16*KR entries
// lives in KR register pairs (distance, candidate index) of that group: element e = 16*r + p
// sits in register r of lane p, sorted ascending by the key (d, j), which is a strict total
// order because j is unique per reference.  New candidates arrive in batches of 16 (one per
// lane), are sorted with a bitonic network built from lane-xor shuffles, and are merged
// into the list by bitonic merges; the 16 largest of (last list register, batch) are
// dropped.  Unused slots hold (+inf, INT_MAX).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmk {

constexpr int kNoIndex = 0x7fffffff;

__device__ __forceinline__ bool key_less(float ad, int aj, float bd, int bj) {
  return ad < bd || (ad == bd && aj < bj);
}

// Compare-exchange with the lane at xor distance m inside a 16-lane group.
__device__ __forceinline__ void cmpx(float& d, int& j, int m, bool keep_min) {
  const float pd = __shfl_xor(d, m, 16);
  const int pj = __shfl_xor(j, m, 16);
  const bool take = keep_min ? key_less(pd, pj, d, j) : key_less(d, j, pd, pj);
  d = take ? pd : d;
  j = take ? pj : j;
}

// Sort 16 entries (one per lane of the group); ascending if `asc`.
__device__ __forceinline__ void sort16(float& d, int& j, int p, bool asc) {
#pragma unroll
  for (int k = 2; k <= 16; k <<= 1) {
#pragma unroll
    for (int m = k >> 1; m > 0; m >>= 1) {
      const bool blk_asc = ((p & k) == 0) == asc;  // k == 16: one block, direction `asc`
      const bool lower = (p & m) == 0;
      cmpx(d, j, m, lower == blk_asc);
    }
  }
}

// Turn a bitonic sequence of 16 into ascending order.
__device__ __forceinline__ void bitonic_merge16(float& d, int& j, int p) {
#pragma unroll
  for (int m = 8; m > 0; m >>= 1) cmpx(d, j, m, (p & m) == 0);
}

// Merge a batch (cd, cj), one entry per lane, into the sorted list (Ld, Lj)[KR].
template <int KR>
__device__ __forceinline__ void merge_batch(float (&Ld)[KR], int (&Lj)[KR], float cd, int cj,
                                            int p) {
  sort16(cd, cj, p, /*asc=*/false);
  // 16 smallest of (last list register, batch): elementwise min of an ascending and a
  // descending sequence is bitonic.
  {
    const bool lt = key_less(Ld[KR - 1], Lj[KR - 1], cd, cj);
    float sd = lt ? Ld[KR - 1] : cd;
    int sj = lt ? Lj[KR - 1] : cj;
    bitonic_merge16(sd, sj, p);
    cd = sd;
    cj = sj;  // (cd, cj) now ascending
  }
#pragma unroll
  for (int r = 0; r < KR - 1; ++r) {
    // merge two ascending 16-runs: low half stays in register r, high half carries on
    const float rd = __shfl_xor(cd, 15, 16);
    const int rj = __shfl_xor(cj, 15, 16);
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

// Distance of list element K-1 (the admission threshold), broadcast within the group.
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
