// Device helpers shared by the libgbs kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "gbs.h"

namespace gbs {

constexpr int kMaxOrder = GBS_MAX_ORDER;
// Largest grid of a one-subset-per-thread launch; beyond it threads stride.
constexpr uint64_t kMaxGrid = 1ull << 30;

// Packed lower-triangular index of (i, j), i >= j.
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }
__host__ __device__ constexpr int tri_size(int n) { return n * (n + 1) / 2; }

__host__ __device__ constexpr int popcount_c(unsigned x) {
  return x == 0 ? 0 : (int)(x & 1u) + popcount_c(x >> 1);
}

// Status word written by kernels: the first non-positive or non-finite pivot.
struct DeviceStatus {
  int32_t flag;   // 0 = ok
  int32_t order;  // subset order of the first failure seen
  int64_t rank;   // its colex rank
};

__device__ __forceinline__ void latch_failure(DeviceStatus* st, int order, int64_t rank) {
  if (atomicCAS(&st->flag, 0, 1) == 0) {
    st->order = order;
    st->rank = rank;
  }
}

// 1/sqrt(x) in FP64: hardware estimate refined by two Newton steps
// y <- y + y (1 - x y^2) / 2, each step squaring the relative error.
__device__ __forceinline__ double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  return y;
}

// Colex unranking.  bin[k * ld + n] = C(n, k) for k = 1..D, n = 0..M.
// Writes s[0] < s[1] < ... < s[D-1] with sum_j C(s[j], j+1) = r.
template <int D, typename Table>
__device__ __forceinline__ void colex_unrank(uint64_t r, int M, const Table* bin, int ld,
                                             int (&s)[D]) {
  int hi = M;  // exclusive upper bound for the current element
#pragma unroll
  for (int j = D - 1; j >= 0; --j) {
    const Table* col = bin + (j + 1) * ld;
    int lo = j;
    int h = hi - 1;
    while (lo < h) {
      int mid = (lo + h + 1) >> 1;
      if ((uint64_t)col[mid] <= r) lo = mid; else h = mid - 1;
    }
    s[j] = lo;
    r -= (uint64_t)col[lo];
    hi = lo;
  }
}

}  // namespace gbs
