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

// 1/sqrt(x) in FP64: the hardware estimate refined by one Halley step.
__device__ __forceinline__ double rsqrt_f64(double x) {
  // The instruction's estimate y is good to about 2^-25 relative; one step of
  // Halley's iteration for x y^2 = 1, y <- y (1 + e/2 + 3e^2/8) with
  // e = 1 - x y^2, leaves an error of order e^3 below the final rounding
  // (measured within 1 ulp, like two Newton steps, at five operations
  // instead of eight).
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// Packed lower triangle of an N x N symmetric matrix.
template <int N>
struct Tri {
  double a[tri_size(N)];
};

template <int N>
struct TriF {
  float a[tri_size(N)];
};

// Gather the normalised deviation F = E_S (FP32, zero diagonal blocks) for
// modes s[0..n-1] in the given order.
template <int n>
__device__ __forceinline__ void gather_e(const float* __restrict__ E, int M, const int* s,
                                         TriF<2 * n>& F) {
  const size_t lde = 2 * (size_t)M;
#pragma unroll
  for (int i = 0; i < n; ++i) {
    F.a[tri(2 * i, 2 * i)] = 0.0f;
    F.a[tri(2 * i + 1, 2 * i)] = 0.0f;
    F.a[tri(2 * i + 1, 2 * i + 1)] = 0.0f;
#pragma unroll
    for (int j = 0; j < i; ++j) {
      const float* q = E + (size_t)(2 * s[i]) * lde + 2 * s[j];
      const float2 q0 = *reinterpret_cast<const float2*>(q);
      const float2 q1 = *reinterpret_cast<const float2*>(q + lde);
      F.a[tri(2 * i, 2 * j)] = q0.x;
      F.a[tri(2 * i, 2 * j + 1)] = q0.y;
      F.a[tri(2 * i + 1, 2 * j)] = q1.x;
      F.a[tri(2 * i + 1, 2 * j + 1)] = q1.y;
    }
  }
}

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

// Displaced states: the share of mu^T Q^{-1} mu taken by the leading 2x2 pivot
// P of A, given the mean v over A's rows (v[0..1] on P):
//   w = P^{-1} v_P,  returns v_P . w,  vr[i - 2] = v[i] - A_{i,P} w  (i >= 2),
// so vr is the mean over the rows of the Schur complement A / P and the
// quadratic form splits as v_P^T P^{-1} v_P + vr^T (A / P)^{-1} vr (block
// elimination of the bordered matrix [[A, v], [v^T, 0]]).  inv_det = 1/det(P).
template <int n>
__device__ __forceinline__ double pivot_mean(const Tri<n>& A, double inv_det, const double* v,
                                             double* vr) {
  const double a00 = A.a[0], a10 = A.a[1], a11 = A.a[2];
  const double w0 = fma(a11, v[0], -a10 * v[1]) * inv_det;
  const double w1 = fma(a00, v[1], -a10 * v[0]) * inv_det;
#pragma unroll
  for (int i = 2; i < n; ++i)
    vr[i - 2] = fma(-A.a[tri(i, 1)], w1, fma(-A.a[tri(i, 0)], w0, v[i]));
  return fma(v[0], w0, v[1] * w1);
}

// The first moments of modes s[0..n-1] (in the given order) from the
// interleaved mean vector (x_k at 2k, p_k at 2k+1).
template <int n>
__device__ __forceinline__ void gather_mean(const double* __restrict__ mi, const int* s,
                                            double (&v)[2 * n]) {
#pragma unroll
  for (int i = 0; i < n; ++i) {
    const double2 m = *reinterpret_cast<const double2*>(mi + 2 * (size_t)s[i]);
    v[2 * i] = m.x;
    v[2 * i + 1] = m.y;
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

// As gather_q, for a block order in which block V's mode varies fastest across
// the lanes of a wavefront (consecutive colex ranks differ in their smallest
// mode): the blocks in V's block row are read from the transposed position
// (a row shared by the wavefront, consecutive columns) and V's diagonal block
// from the per-mode table Qd (x-x, p-x, p-p entries, 4 doubles per mode), so
// every load instruction is coalesced or a broadcast.
template <int n, int V>
__device__ __forceinline__ void gather_q_coalesced(const double* __restrict__ Qi,
                                                   const double* __restrict__ Qd, int M,
                                                   const int* s, Tri<2 * n>& A) {
  const size_t ldq = 2 * (size_t)M;
#pragma unroll
  for (int i = 0; i < n; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      if (i == V && j == V) {
        const double2 d0 = *reinterpret_cast<const double2*>(Qd + 4 * (size_t)s[i]);
        const double2 d1 = *reinterpret_cast<const double2*>(Qd + 4 * (size_t)s[i] + 2);
        A.a[tri(2 * i, 2 * i)] = d0.x;
        A.a[tri(2 * i + 1, 2 * i)] = d0.y;
        A.a[tri(2 * i + 1, 2 * i + 1)] = d1.x;
      } else if (i == V) {
        // block (V, j) = transpose of block (j, V)
        const double* q = Qi + (size_t)(2 * s[j]) * ldq + 2 * s[i];
        const double2 q0 = *reinterpret_cast<const double2*>(q);        // (j_x, V_x), (j_x, V_p)
        const double2 q1 = *reinterpret_cast<const double2*>(q + ldq);  // (j_p, V_x), (j_p, V_p)
        A.a[tri(2 * i, 2 * j)] = q0.x;
        A.a[tri(2 * i + 1, 2 * j)] = q0.y;
        A.a[tri(2 * i, 2 * j + 1)] = q1.x;
        A.a[tri(2 * i + 1, 2 * j + 1)] = q1.y;
      } else {
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
}

// The same for the normalised FP32 deviation E (symmetric, zero diagonal blocks).
template <int n, int V>
__device__ __forceinline__ void gather_e_coalesced(const float* __restrict__ E, int M, const int* s,
                                                   TriF<2 * n>& F) {
  const size_t lde = 2 * (size_t)M;
#pragma unroll
  for (int i = 0; i < n; ++i) {
    F.a[tri(2 * i, 2 * i)] = 0.0f;
    F.a[tri(2 * i + 1, 2 * i)] = 0.0f;
    F.a[tri(2 * i + 1, 2 * i + 1)] = 0.0f;
#pragma unroll
    for (int j = 0; j < i; ++j) {
      if (i == V) {
        const float* q = E + (size_t)(2 * s[j]) * lde + 2 * s[i];
        const float2 q0 = *reinterpret_cast<const float2*>(q);
        const float2 q1 = *reinterpret_cast<const float2*>(q + lde);
        F.a[tri(2 * i, 2 * j)] = q0.x;
        F.a[tri(2 * i + 1, 2 * j)] = q0.y;
        F.a[tri(2 * i, 2 * j + 1)] = q1.x;
        F.a[tri(2 * i + 1, 2 * j + 1)] = q1.y;
      } else {
        const float* q = E + (size_t)(2 * s[i]) * lde + 2 * s[j];
        const float2 q0 = *reinterpret_cast<const float2*>(q);
        const float2 q1 = *reinterpret_cast<const float2*>(q + lde);
        F.a[tri(2 * i, 2 * j)] = q0.x;
        F.a[tri(2 * i, 2 * j + 1)] = q0.y;
        F.a[tri(2 * i + 1, 2 * j)] = q1.x;
        F.a[tri(2 * i + 1, 2 * j + 1)] = q1.y;
      }
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

// Colex unranking by estimate and correction.  At level j the element is the
// largest x < hi with C(x, j) <= r; since C(x, j) ~ (x - (j-1)/2)^j / j!, the
// estimate x ~ (j! r)^(1/j) + (j-1)/2 (FP32) is within a step or two, and exact
// integer comparisons against the binomial table finish the search.
// col_j(x) = bin[j * ld + x] = C(x, j).
template <int D, typename Tab>
__device__ __forceinline__ void colex_unrank_est(uint64_t r, int M, const Tab* bin, int ld,
                                                 int (&s)[D]) {
  constexpr float kFact[6] = {1.f, 1.f, 2.f, 6.f, 24.f, 120.f};
  int hi = M;
#pragma unroll
  for (int j = D; j >= 1; --j) {
    const Tab* col = bin + j * ld;
    int x;
    if (j == 1) {
      x = (int)r;
    } else {
      const float fr = (float)r;
      float est;
      if (j == 2) {
        est = 0.5f * (1.0f + __builtin_amdgcn_sqrtf(fmaf(8.0f, fr, 1.0f)));
      } else {
        const float lg = __builtin_amdgcn_logf(fr * kFact[j]) * (1.0f / (float)j);
        est = __builtin_amdgcn_exp2f(lg) + 0.5f * (float)(j - 1);
      }
      x = (int)est;
      x = x < j - 1 ? j - 1 : (x > hi - 1 ? hi - 1 : x);
      while (x + 1 < hi && (uint64_t)col[x + 1] <= r) ++x;
      while (x > j - 1 && (uint64_t)col[x] > r) --x;
    }
    s[j - 1] = x;
    r -= (uint64_t)col[x];
    hi = x;
  }
}

// Load from a uniform base pointer at a 32-bit element index (byte offset < 2^32).
__device__ __forceinline__ double load_at(const double* __restrict__ base, uint32_t idx) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + (idx << 3));
}
__device__ __forceinline__ double load_at(const double* __restrict__ base, uint64_t idx) {
  return base[idx];
}
// Two doubles at a 32-bit byte offset (16-byte aligned) from a uniform base.
__device__ __forceinline__ double2 load2_at(const double* __restrict__ base, uint32_t byte_off) {
  return *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ __forceinline__ void store_at(double* __restrict__ base, uint32_t idx, double v) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + (idx << 3)) = v;
}
__device__ __forceinline__ void store_at(double* __restrict__ base, uint64_t idx, double v) {
  base[idx] = v;
}

}  // namespace gbs
