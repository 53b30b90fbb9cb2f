// Adjoint (vector-Jacobian product) of the correlator/cumulant path.
//
// Forward chain, for all subsets up to order K (m = mu for click, c for parity):
//   p(T) = det(Q_T)^(-1/2)                                   (App. D.1)
//   m(B) = sum_{T subset B} a(B,T) p(T),  a = (-1)^|T| (click) or (-1)^|B| (-2)^|T| (parity)
//   k(S) = sum_{pi partition of S} w(pi) prod_{B in pi} m(B) (Eq. cumulant_corr_main)
// Reverse, given the upstream gradients gm(S) (correlators) and gk(S) (cumulants):
//   mbar(B) = gm(B) + gk(B) + sum_{X disjoint from B, 1 <= |X| <= K-|B|} gk(B + X) D1(X),
//      where d k(S)/d m(B) = D1(S \ B) and, for X non-empty,
//      D1(X) = sum_{pi partition of X} (-1)^|pi| |pi|! prod_{B' in pi} m(B')
//      (the partitions of S having B as a block are pi' + {B}, pi' a partition of
//      S \ B, with weight w(|pi'| + 1) = (-1)^|pi'| |pi'|!);
//   pbar(T) = sum_{B superset of T, |B| <= K} a(B,T) mbar(B);
//   d p(T) / d Q_T = -p(T) Q_T^{-1} / 2   (d log det A = tr(A^{-1} dA)),
//   so the 2x2 block (i, j) of dL/dsigma is
//      G_ij = sum_{T containing i and j} -pbar(T) p(T) [Q_T^{-1}]_{ij} / 2.
// Every sum is a gather owned by one wavefront (the superset sums by their
// target subset, G_ij by its mode pair) reduced in a fixed order: no atomics,
// results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "gbs_internal.h"

namespace gbs {

namespace {

constexpr int kWave = 64;

// Set partitions of {0..n-1}, n <= 4, as block masks (restricted growth strings).
struct PartTable {
  int count[5];
  int nblocks[5][15];
  unsigned char blocks[5][15][4];
};

constexpr PartTable make_partitions() {
  PartTable t{};
  for (int n = 1; n <= 4; ++n) {
    int lab[4] = {0, 0, 0, 0};
    int total = 1;
    for (int i = 0; i < n; ++i) total *= n;
    int cnt = 0;
    for (int code = 0; code < total; ++code) {
      int c = code;
      for (int i = 0; i < n; ++i) {
        lab[i] = c % n;
        c /= n;
      }
      // restricted growth: lab[0] = 0, lab[i] <= 1 + max(lab[0..i-1])
      bool ok = lab[0] == 0;
      int mx = 0;
      for (int i = 1; i < n && ok; ++i) {
        if (lab[i] > mx + 1) ok = false;
        if (lab[i] > mx) mx = lab[i];
      }
      if (!ok) continue;
      t.nblocks[n][cnt] = mx + 1;
      for (int b = 0; b < 4; ++b) t.blocks[n][cnt][b] = 0;
      for (int i = 0; i < n; ++i) t.blocks[n][cnt][lab[i]] |= (unsigned char)(1u << i);
      ++cnt;
    }
    t.count[n] = cnt;
  }
  return t;
}

__constant__ PartTable kParts = make_partitions();

__device__ __forceinline__ uint64_t binom_at(const uint64_t* __restrict__ bin, int n, int k) {
  return bin[k * kBinLd + n];
}

__device__ __forceinline__ uint64_t rank_sorted(const uint64_t* __restrict__ bin, const int* s,
                                                int n) {
  uint64_t r = 0;
  for (int j = 0; j < n; ++j) r += binom_at(bin, s[j], j + 1);
  return r;
}

// j-subset of [0, universe) with colex rank r, ascending.
__device__ __forceinline__ void unrank_dyn(const uint64_t* __restrict__ bin, uint64_t r, int j,
                                           int universe, int* x) {
  int hi = universe;
  for (int t = j - 1; t >= 0; --t) {
    int lo = t, h = hi - 1;
    while (lo < h) {
      const int mid = (lo + h + 1) >> 1;
      if (binom_at(bin, mid, t + 1) <= r) lo = mid; else h = mid - 1;
    }
    x[t] = lo;
    r -= binom_at(bin, lo, t + 1);
    hi = lo;
  }
}

// Modes of a j-subset of the complement of B (sorted, size k): complement
// index -> mode, skipping B's elements in increasing order.
__device__ __forceinline__ void complement_modes(const int* xc, int j, const int* B, int k, int* x) {
  for (int t = 0; t < j; ++t) {
    int m = xc[t];
    for (int i = 0; i < k; ++i)
      if (B[i] <= m) ++m;
    x[t] = m;
  }
}

// Sorted union of two sorted disjoint sets.
__device__ __forceinline__ int merge_sorted(const int* a, int na, const int* b, int nb, int* out) {
  int i = 0, j = 0, n = 0;
  while (i < na || j < nb) {
    if (j >= nb || (i < na && a[i] < b[j])) out[n++] = a[i++];
    else out[n++] = b[j++];
  }
  return n;
}

// Flat index over all X of sizes jmin..jmax within a universe of u modes.
__device__ __forceinline__ void flat_to_sized(const uint64_t* __restrict__ bin, uint64_t i, int jmin,
                                              int jmax, int u, int* j, uint64_t* r) {
  for (int t = jmin; t <= jmax; ++t) {
    const uint64_t c = binom_at(bin, u, t);
    if (i < c) {
      *j = t;
      *r = i;
      return;
    }
    i -= c;
  }
  *j = -1;
  *r = 0;
}

__device__ __forceinline__ uint64_t count_sized(const uint64_t* __restrict__ bin, int jmin, int jmax,
                                                int u) {
  uint64_t c = 0;
  for (int t = jmin; t <= jmax; ++t) c += binom_at(bin, u, t);
  return c;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Workgroups of up to this many threads share one superset sum (the sigma-bar
// kernel, whose per-superset inverse needs about 200 registers, up to
// kSigmaThreads).
constexpr int kSumThreads = 1024;
constexpr int kSigmaThreads = 256;

// Sum over the workgroup in a fixed order (lanes by the butterfly, then the
// waves in index order): deterministic for a given launch shape.  Valid in
// thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[kSumThreads / kWave];
  __syncthreads();  // thread 0 has read the previous call's partial sums
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) part[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += part[i];
  return t;
}

struct Offsets {
  int64_t off[kMaxOrder + 2];  // start of order-d block, off[1] = 0
};

// A superset sum of n terms split over nsplit workgroups (blockIdx.y): chunk y
// takes the terms [n y / nsplit, n (y + 1) / nsplit).  With nsplit > 1 each
// workgroup writes its partial sum to part[(item * nsplit + y) * width + e] and
// a finishing kernel adds the partials in chunk order, so the result stays
// deterministic for a given launch shape.
__device__ __forceinline__ void chunk_range(uint64_t n, uint64_t* lo, uint64_t* hi) {
  *lo = n * blockIdx.y / gridDim.y;
  *hi = n * (blockIdx.y + 1) / gridDim.y;
}

// ---------------------------------------------------------------------------
// D1(X) for every non-empty X with |X| <= K - 1 (one thread per X).
__global__ void d1_kernel(const double* __restrict__ m, int M, int K, Offsets o,
                          const uint64_t* __restrict__ bin, double* __restrict__ d1) {
  const int64_t total = o.off[K];  // orders 1..K-1
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int j = 1;
    while (idx >= o.off[j + 1]) ++j;
    const uint64_t r = (uint64_t)(idx - o.off[j]);
    int x[kMaxOrder];
    unrank_dyn(bin, r, j, M, x);
    double mv[16];
    mv[0] = 1.0;
    for (unsigned mask = 1; mask < (1u << j); ++mask) {
      int sub[kMaxOrder], n = 0;
      for (int t = 0; t < j; ++t)
        if (mask & (1u << t)) sub[n++] = x[t];
      mv[mask] = m[o.off[n] + rank_sorted(bin, sub, n)];
    }
    double acc = 0.0;
    for (int q = 0; q < kParts.count[j]; ++q) {
      const int nb = kParts.nblocks[j][q];
      double w = (nb & 1) ? -1.0 : 1.0;
      for (int f = 2; f <= nb; ++f) w *= f;  // (-1)^nb nb!
      for (int b = 0; b < nb; ++b) w *= mv[kParts.blocks[j][q][b]];
      acc += w;
    }
    d1[idx] = acc;
  }
}

// mbar(B) for every B of order k (one workgroup per B, its threads striding
// over the supersets).
__global__ __launch_bounds__(kSumThreads) void mbar_kernel(int M, int K, int k, Offsets o,
                                                     const uint64_t* __restrict__ bin,
                                                     const double* __restrict__ gm,
                                                     const double* __restrict__ gk,
                                                     const double* __restrict__ d1,
                                                     double* __restrict__ mbar,
                                                     double* __restrict__ part) {
  const uint64_t rb = blockIdx.x;
  int B[kMaxOrder];
  unrank_dyn(bin, rb, k, M, B);
  double acc = 0.0;
  if (gk && k < K) {
    const int u = M - k;
    uint64_t lo, hi;
    chunk_range(count_sized(bin, 1, K - k, u), &lo, &hi);
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      int j;
      uint64_t rx;
      flat_to_sized(bin, i, 1, K - k, u, &j, &rx);
      int xc[kMaxOrder], X[kMaxOrder], U[kMaxOrder];
      unrank_dyn(bin, rx, j, u, xc);
      complement_modes(xc, j, B, k, X);
      const int n = merge_sorted(B, k, X, j, U);
      acc = fma(gk[o.off[n] + rank_sorted(bin, U, n)], d1[o.off[j] + rank_sorted(bin, X, j)], acc);
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) {
    if (gridDim.y > 1) {
      part[rb * gridDim.y + blockIdx.y] = acc;
      return;
    }
    const int64_t at = o.off[k] + (int64_t)rb;
    double v = acc;
    if (gk) v += gk[at];
    if (gm) v += gm[at];
    mbar[at] = v;
  }
}

// The split mbar sums of order k: partials in chunk order, then as mbar_kernel.
__global__ void mbar_finish_kernel(int k, int nsplit, uint64_t count, Offsets o,
                                   const double* __restrict__ gm, const double* __restrict__ gk,
                                   const double* __restrict__ part, double* __restrict__ mbar) {
  const uint64_t rb = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rb >= count) return;
  double v = 0.0;
  for (int y = 0; y < nsplit; ++y) v += part[rb * nsplit + y];
  const int64_t at = o.off[k] + (int64_t)rb;
  if (gk) v += gk[at];
  if (gm) v += gm[at];
  mbar[at] = v;
}

// The top order K has no proper supersets: mbar = gk + gm and
// pbar = (-1)^K mbar (click) or (-2)^K (-1)^K mbar (parity), one thread per subset.
__global__ void top_order_kernel(int64_t off, uint64_t count, int K, int parity,
                                 const double* __restrict__ gm, const double* __restrict__ gk,
                                 double* __restrict__ mbar, double* __restrict__ pbar) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= count) return;
  const int64_t at = off + (int64_t)r;
  double v = 0.0;
  if (gk) v += gk[at];
  if (gm) v += gm[at];
  mbar[at] = v;
  double coef = (K & 1) ? -1.0 : 1.0;
  if (parity) coef *= (K & 1) ? -(double)(1 << K) : (double)(1 << K);
  pbar[at] = coef * v;
}

// pbar(T) for every T of order t (one workgroup per T, its threads striding
// over the supersets).
__global__ __launch_bounds__(kSumThreads) void pbar_kernel(int M, int K, int t, int parity, Offsets o,
                                                     const uint64_t* __restrict__ bin,
                                                     const double* __restrict__ mbar,
                                                     double* __restrict__ pbar,
                                                     double* __restrict__ part) {
  const uint64_t rt = blockIdx.x;
  int T[kMaxOrder];
  unrank_dyn(bin, rt, t, M, T);
  const int u = M - t;
  uint64_t lo, hi;
  chunk_range(count_sized(bin, 0, K - t, u), &lo, &hi);
  double acc = 0.0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    int j;
    uint64_t rx;
    flat_to_sized(bin, i, 0, K - t, u, &j, &rx);
    int xc[kMaxOrder], X[kMaxOrder], U[kMaxOrder];
    unrank_dyn(bin, rx, j, u, xc);
    complement_modes(xc, j, T, t, X);
    const int n = merge_sorted(T, t, X, j, U);
    const double v = mbar[o.off[n] + rank_sorted(bin, U, n)];
    acc += (parity && (n & 1)) ? -v : v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) {
    if (gridDim.y > 1) {
      part[rt * gridDim.y + blockIdx.y] = acc;
      return;
    }
    // click: (-1)^t;  parity: (-2)^t (the (-1)^|B| factor is inside the sum)
    double coef = (t & 1) ? -1.0 : 1.0;
    if (parity) coef *= (double)(1 << t);
    pbar[o.off[t] + (int64_t)rt] = coef * acc;
  }
}

// The split pbar sums of order t: partials in chunk order, then as pbar_kernel.
__global__ void pbar_finish_kernel(int t, int parity, int nsplit, uint64_t count, Offsets o,
                                   const double* __restrict__ part, double* __restrict__ pbar) {
  const uint64_t rt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rt >= count) return;
  double v = 0.0;
  for (int y = 0; y < nsplit; ++y) v += part[rt * nsplit + y];
  double coef = (t & 1) ? -1.0 : 1.0;
  if (parity) coef *= (double)(1 << t);
  pbar[o.off[t] + (int64_t)rt] = coef * v;
}

// Trailing (base) block of Q_T^{-1}: the first NX blocks of `modes` are
// eliminated, the last NB (1 or 2) are the base modes.
template <int NX, int NB>
__device__ __forceinline__ void base_inverse(const double* __restrict__ Qi, int M, const int* modes,
                                             double (&G)[4], bool& bad) {
  constexpr int N = NX + NB;
  Tri<2 * N> A;
  gather_q<N>(Qi, M, modes, A);
  double S[tri_size(2 * NB)];
  if constexpr (NX == 0) {
#pragma unroll
    for (int q = 0; q < tri_size(2 * NB); ++q) S[q] = A.a[q];
  } else {
    Tri<2 * N - 2> A1;
    const double det0 = fma(A.a[0], A.a[2], -A.a[1] * A.a[1]);
    bad |= !(det0 > 0.0);
    schur_leading_block<2 * N>(A, 1.0 / det0, A1);
    if constexpr (NX == 1) {
#pragma unroll
      for (int q = 0; q < tri_size(2 * NB); ++q) S[q] = A1.a[q];
    } else {
      Tri<2 * N - 4> A2;
      const double det1 = fma(A1.a[0], A1.a[2], -A1.a[1] * A1.a[1]);
      bad |= !(det1 > 0.0);
      schur_leading_block<2 * N - 2>(A1, 1.0 / det1, A2);
      if constexpr (NX == 2) {
#pragma unroll
        for (int q = 0; q < tri_size(2 * NB); ++q) S[q] = A2.a[q];
      } else {
        Tri<2 * N - 6> A3;
        const double det2 = fma(A2.a[0], A2.a[2], -A2.a[1] * A2.a[1]);
        bad |= !(det2 > 0.0);
        schur_leading_block<2 * N - 4>(A2, 1.0 / det2, A3);
        if constexpr (NX == 3) {
#pragma unroll
          for (int q = 0; q < tri_size(2 * NB); ++q) S[q] = A3.a[q];
        } else {
          static_assert(NX <= 4, "at most four eliminated blocks");
          Tri<2 * N - 8> A4;
          const double det3 = fma(A3.a[0], A3.a[2], -A3.a[1] * A3.a[1]);
          bad |= !(det3 > 0.0);
          schur_leading_block<2 * N - 6>(A3, 1.0 / det3, A4);
#pragma unroll
          for (int q = 0; q < tri_size(2 * NB); ++q) S[q] = A4.a[q];
        }
      }
    }
  }
  if constexpr (NB == 1) {
    // inverse of the 2x2 Schur complement [[s00, s10], [s10, s11]]
    const double det = fma(S[0], S[2], -S[1] * S[1]);
    bad |= !(det > 0.0);
    const double inv = 1.0 / det;
    G[0] = S[2] * inv;
    G[1] = -S[1] * inv;
    G[2] = -S[1] * inv;
    G[3] = S[0] * inv;
  } else {
    // [[A, Bm], [Bm^T, C]]^{-1} off-diagonal block = -A^{-1} Bm Sc^{-1},
    // Sc = C - Bm^T A^{-1} Bm.  Packed 4x4: A = (0,0),(1,0),(1,1);
    // Bm^T rows 2,3 cols 0,1; C = (2,2),(3,2),(3,3).
    const double a00 = S[tri(0, 0)], a10 = S[tri(1, 0)], a11 = S[tri(1, 1)];
    const double b00 = S[tri(2, 0)], b01 = S[tri(3, 0)], b10 = S[tri(2, 1)], b11 = S[tri(3, 1)];
    // Bm = [[b00, b01], [b10, b11]] (rows: A's modes, cols: C's modes)
    const double da = fma(a00, a11, -a10 * a10);
    bad |= !(da > 0.0);
    const double ia = 1.0 / da;
    const double ai00 = a11 * ia, ai01 = -a10 * ia, ai11 = a00 * ia;
    // Y = A^{-1} Bm
    const double y00 = ai00 * b00 + ai01 * b10, y01 = ai00 * b01 + ai01 * b11;
    const double y10 = ai01 * b00 + ai11 * b10, y11 = ai01 * b01 + ai11 * b11;
    // Sc = C - Bm^T Y
    const double c00 = S[tri(2, 2)] - (b00 * y00 + b10 * y10);
    const double c01 = S[tri(3, 2)] - (b00 * y01 + b10 * y11);
    const double c11 = S[tri(3, 3)] - (b01 * y01 + b11 * y11);
    const double dc = fma(c00, c11, -c01 * c01);
    bad |= !(dc > 0.0);
    const double ic = 1.0 / dc;
    const double si00 = c11 * ic, si01 = -c01 * ic, si11 = c00 * ic;
    // -Y Sc^{-1}
    G[0] = -(y00 * si00 + y01 * si01);
    G[1] = -(y00 * si01 + y01 * si11);
    G[2] = -(y10 * si00 + y11 * si01);
    G[3] = -(y10 * si01 + y11 * si11);
  }
}

template <int NB>
__device__ __forceinline__ void base_inverse_dispatch(const double* __restrict__ Qi, int M,
                                                      const int* modes, int nx, double (&G)[4],
                                                      bool& bad) {
  switch (nx) {
    case 0: base_inverse<0, NB>(Qi, M, modes, G, bad); break;
    case 1: base_inverse<1, NB>(Qi, M, modes, G, bad); break;
    case 2: base_inverse<2, NB>(Qi, M, modes, G, bad); break;
    case 3: base_inverse<3, NB>(Qi, M, modes, G, bad); break;
    default: if constexpr (NB == 1) base_inverse<4, 1>(Qi, M, modes, G, bad); break;
  }
}

// Mode pair of a sigma-bar item: the diagonal pairs (i, i), or the pairs i < j
// in colex order (item j (j - 1) / 2 + i).
__device__ __forceinline__ void pair_of(int64_t pid, int diag, int* pi_, int* pj_) {
  if (diag) {
    *pi_ = *pj_ = (int)pid;
    return;
  }
  int j = (int)((1.0 + sqrt(8.0 * (double)pid + 1.0)) / 2.0);
  while ((int64_t)j * (j - 1) / 2 > pid) --j;
  while ((int64_t)(j + 1) * j / 2 <= pid) ++j;
  *pi_ = (int)(pid - (int64_t)j * (j - 1) / 2);
  *pj_ = j;
}

// The 2x2 block (i, j) of dL/dsigma (interleaved (2i + a, 2j + b) -> xxpp
// (i + a M, j + b M)) and, for i != j, its mirror.
__device__ __forceinline__ void store_sigma_block(double* __restrict__ gsig, int M, int i, int j,
                                                  const double (&acc)[4]) {
  const size_t n2 = 2 * (size_t)M;
  const size_t xi = i, pi = i + M, xj = j, pj = j + M;
  gsig[xi * n2 + xj] = acc[0];
  gsig[xi * n2 + pj] = acc[1];
  gsig[pi * n2 + xj] = acc[2];
  gsig[pi * n2 + pj] = acc[3];
  if (i != j) {
    gsig[xj * n2 + xi] = acc[0];
    gsig[pj * n2 + xi] = acc[1];
    gsig[xj * n2 + pi] = acc[2];
    gsig[pj * n2 + pi] = acc[3];
  }
}

// One wavefront per mode pair (i <= j): the 2x2 block of dL/dsigma.
// One workgroup per mode pair (i, j): the diagonal pairs (many more supersets,
// wide workgroups) and the pairs i < j (colex, blockIdx = j (j - 1) / 2 + i)
// are separate launches.
__global__ __launch_bounds__(kSigmaThreads) void sigma_bar_kernel(const double* __restrict__ Qi,
                                                                int M, int K, int diag, Offsets o,
                                                                const uint64_t* __restrict__ bin,
                                                                const double* __restrict__ ptab,
                                                                const double* __restrict__ pbar,
                                                                double* __restrict__ gsig,
                                                                DeviceStatus* __restrict__ st,
                                                                double* __restrict__ part) {
  const int64_t pid = blockIdx.x;
  int i, j;
  pair_of(pid, diag, &i, &j);
  int base[2] = {i, j};
  const int nb = (i == j) ? 1 : 2;
  const int u = M - nb;
  uint64_t lo, hi;
  chunk_range(count_sized(bin, 0, K - nb, u), &lo, &hi);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  bool bad = false;
  for (uint64_t q = lo + threadIdx.x; q < hi; q += blockDim.x) {
    int jx;
    uint64_t rx;
    flat_to_sized(bin, q, 0, K - nb, u, &jx, &rx);
    int xc[kMaxOrder], X[kMaxOrder], T[kMaxOrder];
    unrank_dyn(bin, rx, jx, u, xc);
    complement_modes(xc, jx, base, nb, X);
    const int n = merge_sorted(base, nb, X, jx, T);
    const int64_t at = o.off[n] + (int64_t)rank_sorted(bin, T, n);
    const double w = -0.5 * pbar[at] * ptab[at];
    int modes[kMaxOrder];
    for (int t = 0; t < jx; ++t) modes[t] = X[t];
    for (int t = 0; t < nb; ++t) modes[jx + t] = base[t];
    double G[4];
    if (nb == 1) base_inverse_dispatch<1>(Qi, M, modes, jx, G, bad);
    else base_inverse_dispatch<2>(Qi, M, modes, jx, G, bad);
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[e] = fma(w, G[e], acc[e]);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) acc[e] = block_sum(acc[e]);
  if (bad) latch_failure(st, 0, (int64_t)j * (j + 1) / 2 + i);  // pair index, i <= j
  if (threadIdx.x == 0 && gridDim.y > 1) {
#pragma unroll
    for (int e = 0; e < 4; ++e) part[((size_t)pid * gridDim.y + blockIdx.y) * 4 + e] = acc[e];
  } else if (threadIdx.x == 0) {
    store_sigma_block(gsig, M, i, j, acc);
  }
}

// The split sigma-bar sums: partials in chunk order, then as sigma_bar_kernel.
__global__ void sigma_finish_kernel(int M, int diag, int nsplit, uint64_t count,
                                    const double* __restrict__ part, double* __restrict__ gsig) {
  const uint64_t pid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pid >= count) return;
  int i, j;
  pair_of((int64_t)pid, diag, &i, &j);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int y = 0; y < nsplit; ++y)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[e] += part[(pid * nsplit + y) * 4 + e];
  store_sigma_block(gsig, M, i, j, acc);
}

}  // namespace

hipError_t launch_adjoint(int M, int K, int flags, const double* Qi, const uint64_t* binom,
                          const double* m, const double* ptab, const double* gm, const double* gk,
                          double* d1, double* mbar, double* pbar, double* gsig, DeviceStatus* st,
                          double* part, hipStream_t s) {
  Offsets o{};
  o.off[1] = 0;
  for (int d = 1; d <= kMaxOrder; ++d) o.off[d + 1] = o.off[d] + (d <= K ? (int64_t)host_binom(M, d) : 0);
  hipError_t e = hipSuccess;
  const int parity = (flags & GBS_PARITY) ? 1 : 0;
  if (K >= 2 && gk) {
    e = timing_begin(s, GBS_STAGE_ADJOINT, 0);
    const int64_t n1 = o.off[K];
    const int grid = (int)std::min<int64_t>((n1 + 255) / 256, 65535);
    if (e == hipSuccess) hipLaunchKernelGGL(d1_kernel, dim3(grid), dim3(256), 0, s, m, M, K, o, binom, d1);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = timing_end(s);
  }
  // threads per workgroup for a sum over n supersets: whole wavefronts, at most kSumThreads
  auto threads_for = [](uint64_t n, int cap = kSumThreads) {
    const uint64_t w = std::max<uint64_t>(1, std::min<uint64_t>((n + kWave - 1) / kWave,
                                                                (uint64_t)(cap / kWave)));
    return (unsigned)(w * kWave);
  };
  auto supersets = [&](int k, int jmin) {  // sum_{j = jmin}^{K-k} C(M - k, j)
    uint64_t n = 0;
    for (int j = jmin; j <= K - k; ++j) n += host_binom(M - k, j);
    return n;
  };
  // workgroups per sum: a launch of fewer than kAdjointSplitItems long sums
  // (the order-1 subsets, the diagonal mode pairs) would leave compute units
  // idle, so each sum is split into chunks of at least 512 terms
  auto split_for = [](uint64_t items, uint64_t n) -> unsigned {
    if (items >= (uint64_t)kAdjointSplitItems) return 1u;
    const uint64_t want = ((uint64_t)kAdjointSplitItems + items - 1) / items;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>({want, (uint64_t)kAdjointMaxSplit, n / 512}));
  };
  auto finish_grid = [](uint64_t items) { return dim3((unsigned)((items + 255) / 256)); };
  for (int k = 1; k < K && e == hipSuccess; ++k) {
    e = timing_begin(s, GBS_STAGE_ADJOINT, k);
    const uint64_t items = host_binom(M, k), n = supersets(k, 1);
    const unsigned ns = gk ? split_for(items, n) : 1u;
    if (e == hipSuccess)
      hipLaunchKernelGGL(mbar_kernel, dim3((unsigned)items, ns),
                         dim3(gk ? threads_for((n + ns - 1) / ns) : kWave), 0, s, M, K, k, o,
                         binom, gm, gk, d1, mbar, part);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess && ns > 1)
      hipLaunchKernelGGL(mbar_finish_kernel, finish_grid(items), dim3(256), 0, s, k, (int)ns,
                         items, o, gm, gk, part, mbar);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = timing_end(s);
  }
  if (e == hipSuccess) {  // order K: mbar and pbar together
    e = timing_begin(s, GBS_STAGE_ADJOINT, K);
    const uint64_t cnt = host_binom(M, K);
    if (e == hipSuccess)
      hipLaunchKernelGGL(top_order_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                         o.off[K], cnt, K, parity, gm, gk, mbar, pbar);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = timing_end(s);
  }
  for (int t = 1; t < K && e == hipSuccess; ++t) {
    e = timing_begin(s, GBS_STAGE_ADJOINT, t);
    const uint64_t items = host_binom(M, t), n = supersets(t, 0);
    const unsigned ns = split_for(items, n);
    if (e == hipSuccess)
      hipLaunchKernelGGL(pbar_kernel, dim3((unsigned)items, ns), dim3(threads_for((n + ns - 1) / ns)),
                         0, s, M, K, t, parity, o, binom, mbar, pbar, part);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess && ns > 1)
      hipLaunchKernelGGL(pbar_finish_kernel, finish_grid(items), dim3(256), 0, s, t, parity,
                         (int)ns, items, o, part, pbar);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = timing_end(s);
  }
  if (e == hipSuccess) {
    e = timing_begin(s, GBS_STAGE_ADJOINT, 0);
    // supersets of {i} (diagonal) and of {i, j}: sum_j C(M - nb, j), j <= K - nb
    auto sets = [&](int nb) {
      uint64_t n = 0;
      for (int q = 0; q <= K - nb; ++q) n += host_binom(M - nb, q);
      return n;
    };
    for (int diag = 1; diag >= 0 && e == hipSuccess; --diag) {
      const uint64_t items = diag ? (uint64_t)M : (uint64_t)M * (M - 1) / 2;
      if (items == 0) continue;
      const uint64_t n = sets(diag ? 1 : 2);
      const unsigned ns = split_for(items, n);
      hipLaunchKernelGGL(sigma_bar_kernel, dim3((unsigned)items, ns),
                         dim3(threads_for((n + ns - 1) / ns, kSigmaThreads)), 0, s, Qi, M, K, diag,
                         o, binom, ptab, pbar, gsig, st, part);
      e = hipGetLastError();
      if (e == hipSuccess && ns > 1)
        hipLaunchKernelGGL(sigma_finish_kernel, finish_grid(items), dim3(256), 0, s, M, diag,
                           (int)ns, items, part, gsig);
      if (e == hipSuccess) e = hipGetLastError();
    }
    if (e == hipSuccess) e = timing_end(s);
  }
  return e;
}

}  // namespace gbs
