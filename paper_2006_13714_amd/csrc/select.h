// Entry types shared by the fused BM kernels' selection (Theorem 1, Euclidean branch: keep
// the K smallest distances): a buffered (distance, candidate index) pair and the four
// candidate scores of one lane after a matrix tile with their admission flags.
#pragma once

#include <hip/hip_runtime.h>

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

}  // namespace bmk
