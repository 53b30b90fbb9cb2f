// B-tiled kernel for one colex rank range of one order (3..5) from Q alone.
//
// The subsets S = {a} + B with a < b_0 = min B are consecutive colex ranks,
// rank(S) = a + sum_j C(b_j, j + 2), so a rank range is a run of B's, partial
// at its two ends.  A workgroup takes up to kShardB consecutive B's and splits
// the principal-minor work of each subset into what depends on B alone and what
// involves a (App. D.1, Eq. vacuum_gaussian_prob: p(T) = det(Q_T)^(-1/2)):
//   phase 1, one lane per B: the principal-minor recursion on the 2x2 blocks of
//     Q_B (each block in turn is eliminated -- Schur complement -- or dropped);
//     every node keeps its pivot's inverse P^{-1} and u = P^{-1} A_{P,rest},
//     every leaf U gives p(U); then m(W) for every W subset of B (subset zeta
//     transform) and the coefficients c_B(V) of the cumulant as a linear form in
//     the p({a} + V) (cumulant_coefficients, gbs_subset.h);
//   phase 2, one lane per subset: the same recursion carried on a's block.  With
//     C the coupling of the remaining B blocks to a and S_a a's 2x2 block (both
//     reduced by the eliminated blocks), eliminating block b gives
//       S_a' = S_a - C_b^T P^{-1} C_b,    C_rest' = C_rest - u^T C_b,
//     dropping it leaves both unchanged, and at the leaf U
//       det(Q_{U+a}) = det(Q_U) det(S_a),  so  p({a} + U) = p(U) det(S_a)^(-1/2)
//     (block elimination of the bordered matrix).  Then m(S) = m(B) - nu(B)
//     with nu(B) = sum_V s(V) p({a} + V) (parity: -m(B) + 2 (-1)^|B| nu(B);
//     Eq. corre_cov_main split by whether the subset contains a), and
//     k(S) = sum_V c_B(V) p({a} + V) (Eq. cumulant_corr_main with the block
//     that contains a singled out).
// A subset thus costs 2^(d-1) 2x2 determinants and the a-block updates, where
// the all-minors kernel pays all 2^d - 1 minors of Q_S; its reads of Q are the
// a columns of B's rows (consecutive a across a wavefront) and a's diagonal
// block.  No lower-order tables are read, so every rank range is independent.
#include <hip/hip_runtime.h>

#include "gbs_internal.h"
#include "gbs_subset.h"

namespace gbs {

namespace {

constexpr int kShardB = 32;         // B's per tile
constexpr int kShardThreads = 256;  // threads per workgroup

// Node (k, mask) of the B recursion (blocks 0..k-1 decided, mask = the
// eliminated ones): P^{-1} (packed lower, 3 doubles), then u = P^{-1} A_{P,rest}
// (row 0, then row 1; 2 (NB - 1 - k) columns each).
template <int NB>
__host__ __device__ constexpr int node_size(int k) {
  return 3 + 4 * (NB - 1 - k);
}
template <int NB>
__host__ __device__ constexpr int node_offset(int k, unsigned mask) {
  int off = 0;
  for (int j = 0; j < k; ++j) off += (1 << j) * node_size<NB>(j);
  return off + (int)mask * node_size<NB>(k);
}

// Per-B record in LDS, doubles.
template <int NB>
struct ShardRec {
  static constexpr int oP = node_offset<NB>(NB, 0u);  // p(U), U subset of B (bit i <-> b_i)
  static constexpr int oC = oP + (1 << NB);           // c_B(V), V subset of B
  static constexpr int oMB = oC + (1 << NB);          // m(B)
  static constexpr int n = oMB + 1;
  static constexpr int stride = (n + 1) & ~1;
};

// Phase 1: A over the blocks K..NB-1 (reduced by the eliminated blocks of
// MASK), pT = p(MASK).  Writes the node data to rec and p(U) to p.
template <int NB, int K, unsigned MASK>
__device__ __forceinline__ void b_tree(const Tri<2 * (NB - K)>& A, double pT, double* rec,
                                       double (&p)[1 << NB], bool& bad) {
  constexpr int n = 2 * (NB - K);
  const double a00 = A.a[0], a10 = A.a[1], a11 = A.a[2];
  const double det = fma(a00, a11, -a10 * a10);
  bad |= !(a00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
  const double y = rsqrt_f64(det);
  const double id = y * y;
  const double i00 = a11 * id, i10 = -a10 * id, i11 = a00 * id;
  double* nd = rec + node_offset<NB>(K, MASK);
  nd[0] = i00;
  nd[1] = i10;
  nd[2] = i11;
  if constexpr (n == 2) {
    p[MASK | (1u << K)] = pT * y;
    p[MASK] = pT;
  } else {
#pragma unroll
    for (int j = 0; j < n - 2; ++j) {
      const double c0 = A.a[tri(2 + j, 0)], c1 = A.a[tri(2 + j, 1)];
      nd[3 + j] = fma(i00, c0, i10 * c1);
      nd[3 + (n - 2) + j] = fma(i10, c0, i11 * c1);
    }
    Tri<n - 2> S;
    schur_leading_block<n>(A, id, S);
    b_tree<NB, K + 1, MASK | (1u << K)>(S, pT * y, rec, p, bad);
    Tri<n - 2> R;
#pragma unroll
    for (int i = 2; i < n; ++i)
#pragma unroll
      for (int j = 2; j <= i; ++j) R.a[tri(i - 2, j - 2)] = A.a[tri(i, j)];
    b_tree<NB, K + 1, MASK>(R, pT, rec, p, bad);
  }
}

// p({a} + U) = p(U) det(S_a)^(-1/2) at the leaf U.
template <int NB, unsigned U>
__device__ __forceinline__ void a_leaf(const double* rec, double s00, double s10, double s11,
                                       double (&pa)[1 << NB], bool& bad) {
  const double det = fma(s00, s11, -s10 * s10);
  bad |= !(s00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
  pa[U] = rec[ShardRec<NB>::oP + U] * rsqrt_f64(det);
}

// Phase 2: C[j][c] couples remaining B row j (2 (NB - K) rows) with a's column
// c; (s00, s10, s11) is a's block; both reduced by the eliminated blocks of MASK.
template <int NB, int K, unsigned MASK>
__device__ __forceinline__ void a_tree(const double* rec, const double (&C)[2 * (NB - K)][2],
                                       double s00, double s10, double s11,
                                       double (&pa)[1 << NB], bool& bad) {
  constexpr int n = 2 * (NB - K);
  const double* nd = rec + node_offset<NB>(K, MASK);
  const double i00 = nd[0], i10 = nd[1], i11 = nd[2];
  // w = P^{-1} C_b; S_a' = S_a - C_b^T w
  const double w00 = fma(i00, C[0][0], i10 * C[1][0]);
  const double w01 = fma(i00, C[0][1], i10 * C[1][1]);
  const double w10 = fma(i10, C[0][0], i11 * C[1][0]);
  const double w11 = fma(i10, C[0][1], i11 * C[1][1]);
  const double t00 = fma(-C[0][0], w00, fma(-C[1][0], w10, s00));
  const double t10 = fma(-C[0][1], w00, fma(-C[1][1], w10, s10));
  const double t11 = fma(-C[0][1], w01, fma(-C[1][1], w11, s11));
  if constexpr (n == 2) {
    a_leaf<NB, MASK | (1u << K)>(rec, t00, t10, t11, pa, bad);
    a_leaf<NB, MASK>(rec, s00, s10, s11, pa, bad);
  } else {
    double Ce[n - 2][2];
#pragma unroll
    for (int j = 0; j < n - 2; ++j) {
      const double u0 = nd[3 + j], u1 = nd[3 + (n - 2) + j];
#pragma unroll
      for (int c = 0; c < 2; ++c) Ce[j][c] = fma(-u0, C[0][c], fma(-u1, C[1][c], C[2 + j][c]));
    }
    a_tree<NB, K + 1, MASK | (1u << K)>(rec, Ce, t00, t10, t11, pa, bad);
    double Cr[n - 2][2];
#pragma unroll
    for (int j = 0; j < n - 2; ++j) {
      Cr[j][0] = C[2 + j][0];
      Cr[j][1] = C[2 + j][1];
    }
    a_tree<NB, K + 1, MASK>(rec, Cr, s00, s10, s11, pa, bad);
  }
}

// Three waves per SIMD (168 VGPRs, no spills): with its updates written as
// fused multiply-add chains the per-subset recursion issues 581 instead of 670
// VALU instructions, and a cap of 128 registers for a fourth wave now fails in
// the compiler's spill code (the earlier form ran four waves with four
// registers spilled, about 1% slower than this).
template <int D, int CONV, bool WC, bool WK>
__global__ __launch_bounds__(kShardThreads) __attribute__((amdgpu_waves_per_eu(3)))
void forward_shard_kernel(
    const double* __restrict__ Qi, int M, uint64_t rank0, uint64_t count, uint64_t beta0,
    uint64_t nbeta, uint64_t ntiles, const uint64_t* __restrict__ binom,
    double* __restrict__ corr, double* __restrict__ cum, DeviceStatus* __restrict__ st) {
  constexpr int NB = D - 1;
  constexpr int NU = 1 << NB;               // subsets of B
  constexpr int FULL = NU - 1;
  using R = ShardRec<NB>;
  __shared__ double s_rec[kShardB * R::stride];
  __shared__ int s_b[kShardB][NB];
  __shared__ int s_alo[kShardB];
  __shared__ uint64_t s_out[kShardB];
  __shared__ uint32_t s_pre[kShardB + 1];
  const size_t ldq = 2 * (size_t)M;

  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();  // the previous tile's readers are done
    const uint64_t bt0 = tile * kShardB;
    const int nbt = (int)((nbeta - bt0) < (uint64_t)kShardB ? (nbeta - bt0) : (uint64_t)kShardB);

    // ---------------- phase 1: lane = B ----------------
    if (threadIdx.x < kShardB) {
      const int c = threadIdx.x;
      uint32_t cnt = 0;
      if (c < nbt) {
        int b[NB];
        colex_unrank<NB>(beta0 + bt0 + (uint64_t)c, M, binom, kBinLd, b);
        uint64_t base = 0;
#pragma unroll
        for (int j = 0; j < NB; ++j) base += binom[(j + 2) * kBinLd + b[j]];
        // ranks base + a, a in [0, b_0), inside [rank0, rank0 + count)
        const uint64_t lo = rank0 > base ? rank0 - base : 0;
        const uint64_t end = rank0 + count;
        const uint64_t hi = end > base ? ((uint64_t)b[0] < end - base ? (uint64_t)b[0] : end - base)
                                       : 0;
        cnt = hi > lo ? (uint32_t)(hi - lo) : 0u;
        s_alo[c] = (int)(cnt ? lo : 0);
        s_out[c] = cnt ? base + lo - rank0 : 0;
#pragma unroll
        for (int j = 0; j < NB; ++j) s_b[c][j] = b[j];
        if (cnt) {
          double* rec = s_rec + c * R::stride;
          Tri<2 * NB> A;
          gather_q<NB>(Qi, M, b, A);
          double p[NU];
          bool bad = false;
          b_tree<NB, 0, 0u>(A, 1.0, rec, p, bad);
          if (bad) latch_failure(st, D, (int64_t)(base + lo));
          double m[NU];
          correlators_from_vacuum<NB, CONV>(p, m);
#pragma unroll
          for (int u = 0; u < NU; ++u) rec[R::oP + u] = p[u];
          rec[R::oMB] = m[FULL];
          if constexpr (WK) {
            double cq[NU];
            cumulant_coefficients<NB, CONV>(m, cq);
#pragma unroll
            for (int v = 0; v < NU; ++v) rec[R::oC + v] = cq[v];
          }
        }
      }
      s_pre[c + 1] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_pre[0] = 0;
      for (int c = 1; c <= kShardB; ++c) s_pre[c] += s_pre[c - 1];
    }
    __syncthreads();

    // ---------------- phase 2: lane = subset ----------------
    const uint32_t total = s_pre[kShardB];
    for (uint32_t q = threadIdx.x; q < total; q += kShardThreads) {
      // the B of this subset: the last c with s_pre[c] <= q
      int lo = 0, hi = kShardB - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= q) lo = mid;
        else hi = mid - 1;
      }
      const int c = lo;
      const uint32_t off = q - s_pre[c];
      const int a = s_alo[c] + (int)off;
      const uint64_t out = s_out[c] + off;
      const double* rec = s_rec + c * R::stride;
      double C[2 * NB][2];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const double* row = Qi + (size_t)(2 * s_b[c][j]) * ldq + 2 * (size_t)a;
        const double2 q0 = *reinterpret_cast<const double2*>(row);
        const double2 q1 = *reinterpret_cast<const double2*>(row + ldq);
        C[2 * j][0] = q0.x;
        C[2 * j][1] = q0.y;
        C[2 * j + 1][0] = q1.x;
        C[2 * j + 1][1] = q1.y;
      }
      const double* qa = Qi + (size_t)(2 * a) * ldq + 2 * (size_t)a;
      const double2 qa0 = *reinterpret_cast<const double2*>(qa);
      const double qa11 = qa[ldq + 1];
      double pa[NU];
      bool bad = false;
      a_tree<NB, 0, 0u>(rec, C, qa0.x, qa0.y, qa11, pa, bad);
      if (bad) latch_failure(st, D, (int64_t)(rank0 + out));

      // m(S) = m(B) - nu(B) (click) or -m(B) + 2 (-1)^|B| nu(B) (parity)
      double nuB = 0.0;
#pragma unroll
      for (int u = 0; u < NU; ++u) nuB = fma(vacuum_sign<CONV>(u), pa[u], nuB);
      if constexpr (WC) {
        const double mB = rec[R::oMB];
        corr[out] = (CONV == GBS_CLICK) ? mB - nuB : fma((NB & 1) ? -2.0 : 2.0, nuB, -mB);
      }
      if constexpr (WK) {
        double kS = 0.0;
#pragma unroll
        for (int u = 0; u < NU; ++u) kS = fma(rec[R::oC + u], pa[u], kS);
        cum[out] = kS;
      }
    }
  }
}

template <int D, int CONV>
hipError_t launch_shard_t(int M, const double* Qi, const uint64_t* binom, uint64_t rank0,
                          uint64_t count, uint64_t beta0, uint64_t nbeta, double* corr,
                          double* cum, DeviceStatus* st, hipStream_t s) {
  const uint64_t ntiles = (nbeta + kShardB - 1) / kShardB;
  const unsigned grid = (unsigned)std::min<uint64_t>(ntiles, 1u << 20);
  if (corr && cum)
    hipLaunchKernelGGL((forward_shard_kernel<D, CONV, true, true>), dim3(grid), dim3(kShardThreads),
                       0, s, Qi, M, rank0, count, beta0, nbeta, ntiles, binom, corr, cum, st);
  else if (corr)
    hipLaunchKernelGGL((forward_shard_kernel<D, CONV, true, false>), dim3(grid),
                       dim3(kShardThreads), 0, s, Qi, M, rank0, count, beta0, nbeta, ntiles, binom,
                       corr, cum, st);
  else
    hipLaunchKernelGGL((forward_shard_kernel<D, CONV, false, true>), dim3(grid),
                       dim3(kShardThreads), 0, s, Qi, M, rank0, count, beta0, nbeta, ntiles, binom,
                       corr, cum, st);
  return hipGetLastError();
}

// Colex rank, among the (d-1)-subsets, of the top d-1 elements of the
// order-d subset of rank r.
uint64_t top_rank(int d, uint64_t r) {
  int32_t S[kMaxOrder];
  (void)gbs_colex_unrank(d, (int64_t)r, S);
  uint64_t beta = 0;
  for (int j = 1; j < d; ++j) beta += host_binom(S[j], j);
  return beta;
}

}  // namespace

hipError_t launch_forward_shard(int d, int M, int flags, const double* Qi, const uint64_t* binom,
                                uint64_t rank0, uint64_t count, double* corr, double* cum,
                                DeviceStatus* st, hipStream_t s) {
  if (count == 0 || (!corr && !cum)) return hipSuccess;
  if (d < 3 || d > kMaxOrder) return hipErrorInvalidValue;
  const uint64_t beta0 = top_rank(d, rank0);
  const uint64_t nbeta = top_rank(d, rank0 + count - 1) - beta0 + 1;
  using Launch = hipError_t (*)(int, const double*, const uint64_t*, uint64_t, uint64_t,
                                 uint64_t, uint64_t, double*, double*, DeviceStatus*, hipStream_t);
  const bool par = (flags & GBS_PARITY) != 0;
  Launch fn;
  switch (d) {
    case 3: fn = par ? launch_shard_t<3, GBS_PARITY> : launch_shard_t<3, GBS_CLICK>; break;
    case 4: fn = par ? launch_shard_t<4, GBS_PARITY> : launch_shard_t<4, GBS_CLICK>; break;
    default: fn = par ? launch_shard_t<5, GBS_PARITY> : launch_shard_t<5, GBS_CLICK>; break;
  }
  return fn(M, Qi, binom, rank0, count, beta0, nbeta, corr, cum, st, s);
}

}  // namespace gbs
