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

// Packed lower triangle of an N x N symmetric matrix.
template <int N>
struct Tri {
  double a[tri_size(N)];
};

// Schur complement of the leading 2x2 block P of A (n x n, n >= 4):
//   S = A_rr - A_r0 P^{-1} A_0r,  P^{-1} = adj(P) / det(P).
// Returns det(P); inv_det = 1/det(P) is supplied by the caller (it usually
// has det(P)^(-1/2) already).
template <int n>
__device__ __forceinline__ void schur_leading_block(const Tri<n>& A, double inv_det, Tri<n - 2>& S) {
  const double a00 = A.a[0], a10 = A.a[1], a11 = A.a[2];
  double u0[n], u1[n];
#pragma unroll
  for (int i = 2; i < n; ++i) {
    const double c0 = A.a[tri(i, 0)], c1 = A.a[tri(i, 1)];
    u0[i] = fma(a11, c0, -a10 * c1) * inv_det;
    u1[i] = fma(a00, c1, -a10 * c0) * inv_det;
  }
#pragma unroll
  for (int i = 2; i < n; ++i) {
#pragma unroll
    for (int j = 2; j <= i; ++j) {
      S.a[tri(i - 2, j - 2)] =
          fma(-A.a[tri(i, 1)], u1[j], fma(-A.a[tri(i, 0)], u0[j], A.a[tri(i, j)]));
    }
  }
}

// Gather the 2n x 2n principal block of the interleaved Q for modes s[0..n-1]
// (in the given order: block i of the result is mode s[i]).
template <int n>
__device__ __forceinline__ void gather_q(const double* __restrict__ Qi, int M, const int* s,
                                         Tri<2 * n>& A) {
  const size_t ldq = 2 * (size_t)M;
#pragma unroll
  for (int i = 0; i < n; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      const double* q = Qi + (size_t)(2 * s[i]) * ldq + 2 * s[j];
      const double2 q0 = *reinterpret_cast<const double2*>(q);
      const double2 q1 = *reinterpret_cast<const double2*>(q + ldq);
      A.a[tri(2 * i, 2 * j)] = q0.x;
      A.a[tri(2 * i + 1, 2 * j)] = q1.x;
      A.a[tri(2 * i + 1, 2 * j + 1)] = q1.y;
      if (i != j) A.a[tri(2 * i, 2 * j + 1)] = q0.y;
    }
  }
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
