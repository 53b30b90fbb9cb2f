// T-shared kernel for one colex rank range of one order (3..5) from Q alone.
//
// With S = {a} + B, B = {b_0} + T, a < b_0 < min T = t_1, the subsets of one T
// form the triangle 0 <= a < b_0 < t_1 at colex ranks base(T) + C(b_0, 2) + a,
// base(T) = sum_j C(t_j, j + 3), so a rank range is a run of T's, partial at its
// two ends.  A workgroup (one wavefront) takes one T, kTsA consecutive a (one
// per lane) and up to kTsB consecutive b_0, and orders the blocks of every Q_S
// as [T, b_0, a] (App. D.1, Eq. vacuum_gaussian_prob: p(U) = det(Q_U)^(-1/2)):
//   phase A, one lane: the principal-minor recursion on the 2x2 blocks of Q_T
//     (each block in turn is eliminated -- Schur complement -- or dropped);
//     every node keeps its pivot's inverse P^{-1} and u = P^{-1} A_{P,rest},
//     every leaf V gives p(V);
//   phase B, lane = b_0: b_0's block carried through that recursion.  With C
//     the coupling of the remaining T blocks to b_0 and S b_0's 2x2 block (both
//     reduced by the eliminated blocks), eliminating block t gives
//       S' = S - C_t^T P^{-1} C_t,    C_rest' = C_rest - u^T C_t,
//     dropping it leaves both unchanged; each elimination edge keeps
//     w = P_t^{-1} C_t, each leaf V keeps the inverse Cholesky factor of S_b0|V and
//     p({b_0} + V) = p(V) det(S_b0|V)^(-1/2) (det(Q_{V+b}) = det(Q_V) det(S));
//     then m(W) for every W subset of B (subset zeta transform) and the
//     coefficients c_B(U) of the cumulant as a linear form in the p({a} + U)
//     (cumulant_coefficients, gbs_subset.h);
//   phase C, lane = a (registers): a's block through the same recursion, each
//     edge keeping a's coupling C_t^a, each leaf V the Schur complement S_a|V
//     and p({a} + V);
//   main loop, lane = a, over the b_0: the cross block G = Q_{b_0, a} goes
//     down the tree, G <- G - w^T C_t^a at every elimination edge, and at leaf V
//       S_a|{b_0}+V = S_a|V - G^T (S_b0|V)^{-1} G = S_a|V - H^T H, H = L^{-1} G,
//       p({a, b_0} + V) = p({b_0} + V) det(S_a|{b_0}+V)^(-1/2);
//     then m(S) = m(B) - nu(B) with nu(B) = sum_U s(U) p({a} + U) (parity:
//     -m(B) + 2 (-1)^|B| nu(B); Eq. corre_cov_main split by whether the subset
//     contains a), and k(S) = sum_U c_B(U) p({a} + U) (Eq. cumulant_corr_main
//     with the block that contains a singled out).
// Per subset that is 2^|T| - 1 cross-block updates and 2^|T| 2x2
// determinants; the half of the 2^|B| probabilities that does not contain b_0
// is shared by all the b_0 of a lane.  No lower-order tables are read, so
// every rank range is independent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <list>
#include <memory>
#include <mutex>
#include <vector>

#include "gbs_internal.h"
#include "gbs_subset.h"

namespace gbs {

namespace {

// Node (k, mask) of the principal-minor recursion over NB blocks (blocks
// 0..k-1 decided, mask = the eliminated ones): P^{-1} (packed lower, 3
// doubles), then u = P^{-1} A_{P,rest} (row 0, then row 1; 2 (NB - 1 - k)
// columns each).
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

// The recursion on A over the blocks K..NB-1 (reduced by the eliminated
// blocks of MASK), pT = p(MASK).  Writes the node data to rec and p(U) to p.
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

// a's per tile: one wavefront.  b_0's per tile: 30 records (19.1 KB of LDS at
// order 5) let the eight one-wavefront workgroups that the order-5 kernel's
// registers allow (over 168: two waves per SIMD) share a compute unit (M = 1152
// order-5 shard: 16 / 24 / 30 / 32 b_0's 8.3 / 8.1 / 7.8 / 7.8 ms; capping the
// registers for a third wave per SIMD spills and takes 25 ms).
constexpr int kTsA = 64;
constexpr int kTsB = 30;

// One T of the rank range (host-built list, in colex order of T).
struct ShardT {
  int64_t out0;          // output index of triangle offset 0: base(T) - rank0
  uint32_t lo, hi;       // the range's triangle offsets C(b_0, 2) + a: [lo, hi)
  uint32_t tile0;        // first tile of this T
  uint16_t t[3];         // T's modes, ascending (unused ones 0)
  uint16_t b0lo, b0hi;   // b_0 of the offsets lo and hi - 1
};
static_assert(sizeof(ShardT) == 32, "ShardT layout");

// Tiles of one T: a-blocks of kTsA from a = 0, each with the b_0 in
// [max(b0lo, a_first + 1), b0hi] in chunks of kTsB.  idx >= 0: decode tile idx
// into (al, bl, nb); idx < 0: return the tile count.
__host__ __device__ inline uint32_t ts_tiles(uint32_t b0lo, uint32_t b0hi, int64_t idx,
                                             uint32_t* al, uint32_t* bl, uint32_t* nb) {
  uint32_t n = 0;
  for (uint32_t a0 = 0; a0 < b0hi; a0 += kTsA) {
    const uint32_t bs = b0lo > a0 + 1 ? b0lo : a0 + 1;
    if (bs > b0hi) continue;
    const uint32_t nch = (b0hi - bs + kTsB) / kTsB;
    if (idx >= 0 && (uint64_t)idx < (uint64_t)n + nch) {
      const uint32_t j = (uint32_t)idx - n;
      *al = a0;
      *bl = bs + j * kTsB;
      *nb = (b0hi - *bl + 1) < (uint32_t)kTsB ? (b0hi - *bl + 1) : (uint32_t)kTsB;
      return n;
    }
    n += nch;
  }
  return n;
}

// Per-b_0 record in LDS, doubles: edges (w, 4 each), leaves (the inverse
// Cholesky factor of S_b0|V packed lower, then p({b_0} + V)), c_B(U) (bit 0 of
// U: b_0, bit k + 1: T block k), m(B), a failure flag.
template <int NT>
struct TsRec {
  static constexpr int NV = 1 << NT;
  static constexpr int NE = NV - 1;
  static constexpr int NU = 2 * NV;
  static constexpr int oW = 0;
  static constexpr int oL = 4 * NE;
  static constexpr int oC = oL + 4 * NV;
  static constexpr int oMB = oC + NU;
  static constexpr int oBad = oMB + 1;
  static constexpr int stride = (oBad + 2) & ~1;
};

// Leaf V of the bordered recursion: B0 keeps (L^{-1}, p) with S = L L^T
// (L^{-1} = [[r, 0], [-s10 r y, s00 r y]], r = s00^(-1/2), y = det(S)^(-1/2)),
// otherwise (S, p).
template <unsigned V, bool B0>
__device__ __forceinline__ void ts_leaf(const double* pT, double s00, double s10, double s11,
                                        double* lr, bool& bad) {
  const double det = fma(s00, s11, -s10 * s10);
  bad |= !(s00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
  const double y = rsqrt_f64(det);
  double* l = lr + 4 * V;
  if constexpr (B0) {
    const double r = rsqrt_f64(s00);
    const double ry = r * y;
    l[0] = r;
    l[1] = -s10 * ry;
    l[2] = s00 * ry;
  } else {
    l[0] = s00;
    l[1] = s10;
    l[2] = s11;
  }
  l[3] = pT[V] * y;
}

// A bordering block (b_0, or a) carried through the T recursion from node
// (K, MASK); C[j][c] couples remaining T row j with the block's column c, s its
// diagonal block, both reduced by the eliminated blocks of MASK.  Edge e of
// node (K, MASK) is (2^K - 1) + MASK; B0 records w = P^{-1} C_K there,
// otherwise C_K itself.
template <int NT, int K, unsigned MASK, bool B0>
__device__ __forceinline__ void ts_border(const double* tn, const double* pT,
                                          const double (&C)[2 * (NT - K)][2], double s00,
                                          double s10, double s11, double* er, double* lr,
                                          bool& bad) {
  constexpr int n = 2 * (NT - K);
  constexpr int e = (1 << K) - 1 + (int)MASK;
  const double* nd = tn + node_offset<NT>(K, MASK);
  const double i00 = nd[0], i10 = nd[1], i11 = nd[2];
  const double w00 = fma(i00, C[0][0], i10 * C[1][0]);
  const double w01 = fma(i00, C[0][1], i10 * C[1][1]);
  const double w10 = fma(i10, C[0][0], i11 * C[1][0]);
  const double w11 = fma(i10, C[0][1], i11 * C[1][1]);
  double* ed = er + 4 * e;
  if constexpr (B0) {
    ed[0] = w00;
    ed[1] = w01;
    ed[2] = w10;
    ed[3] = w11;
  } else {
    ed[0] = C[0][0];
    ed[1] = C[0][1];
    ed[2] = C[1][0];
    ed[3] = C[1][1];
  }
  const double t00 = fma(-C[0][0], w00, fma(-C[1][0], w10, s00));
  const double t10 = fma(-C[0][1], w00, fma(-C[1][1], w10, s10));
  const double t11 = fma(-C[0][1], w01, fma(-C[1][1], w11, s11));
  if constexpr (n == 2) {
    ts_leaf<MASK | (1u << K), B0>(pT, t00, t10, t11, lr, bad);
    ts_leaf<MASK, B0>(pT, s00, s10, s11, lr, bad);
  } else {
    double Ce[n - 2][2], Cr[n - 2][2];
#pragma unroll
    for (int j = 0; j < n - 2; ++j) {
      const double u0 = nd[3 + j], u1 = nd[3 + (n - 2) + j];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        Ce[j][c] = fma(-u0, C[0][c], fma(-u1, C[1][c], C[2 + j][c]));
        Cr[j][c] = C[2 + j][c];
      }
    }
    ts_border<NT, K + 1, MASK | (1u << K), B0>(tn, pT, Ce, t00, t10, t11, er, lr, bad);
    ts_border<NT, K + 1, MASK, B0>(tn, pT, Cr, s00, s10, s11, er, lr, bad);
  }
}

// Leaf V of the main loop: p({a, b_0} + V) from G, the b_0 record and S_a|V:
// with H = L^{-1} G, S_a|{b_0}+V = S_a|V - H^T H.  Its diagonal is at most that
// of S_a|V, which phase C found finite, so a finite determinant needs no check.
template <int NT, unsigned V>
__device__ __forceinline__ void ts_pair_leaf(const double* br, const double (&sa)[1 << NT][3],
                                             double g00, double g01, double g10, double g11,
                                             double (&pab)[1 << NT], bool& bad) {
  using R = TsRec<NT>;
  const double* l = br + R::oL + 4 * V;
  const double2 iv = *reinterpret_cast<const double2*>(l);
  const double2 lp = *reinterpret_cast<const double2*>(l + 2);
  const double r = iv.x, m = iv.y, q = lp.x;
  const double h00 = r * g00;
  const double h01 = r * g01;
  const double h10 = fma(m, g00, q * g10);
  const double h11 = fma(m, g01, q * g11);
  const double s00 = fma(-h00, h00, fma(-h10, h10, sa[V][0]));
  const double s10 = fma(-h00, h01, fma(-h10, h11, sa[V][1]));
  const double s11 = fma(-h01, h01, fma(-h11, h11, sa[V][2]));
  const double det = fma(s00, s11, -s10 * s10);
  bad |= !(s00 > 0.0) || !(det > 0.0);
  pab[V] = lp.y * rsqrt_f64(det);
}

// The cross block G (b_0 rows, a columns) down the tree from node (K, MASK).
template <int NT, int K, unsigned MASK>
__device__ __forceinline__ void ts_pair(const double* br, const double (&ca)[(1 << NT) - 1][4],
                                        const double (&sa)[1 << NT][3], double g00, double g01,
                                        double g10, double g11, double (&pab)[1 << NT],
                                        bool& bad) {
  constexpr int e = (1 << K) - 1 + (int)MASK;
  const double* w = br + TsRec<NT>::oW + 4 * e;
  const double2 wa = *reinterpret_cast<const double2*>(w);
  const double2 wb = *reinterpret_cast<const double2*>(w + 2);
  const double w00 = wa.x, w01 = wa.y, w10 = wb.x, w11 = wb.y;
  const double* c = ca[e];
  const double e00 = fma(-w00, c[0], fma(-w10, c[2], g00));
  const double e01 = fma(-w00, c[1], fma(-w10, c[3], g01));
  const double e10 = fma(-w01, c[0], fma(-w11, c[2], g10));
  const double e11 = fma(-w01, c[1], fma(-w11, c[3], g11));
  if constexpr (K == NT - 1) {
    ts_pair_leaf<NT, MASK | (1u << K)>(br, sa, e00, e01, e10, e11, pab, bad);
    ts_pair_leaf<NT, MASK>(br, sa, g00, g01, g10, g11, pab, bad);
  } else {
    ts_pair<NT, K + 1, MASK | (1u << K)>(br, ca, sa, e00, e01, e10, e11, pab, bad);
    ts_pair<NT, K + 1, MASK>(br, ca, sa, g00, g01, g10, g11, pab, bad);
  }
}

template <int D, int CONV, bool WC, bool WK>
__global__ __launch_bounds__(kTsA) void forward_tshard_kernel(
    const double* __restrict__ Qi, int M, uint64_t rank0, const ShardT* __restrict__ tl,
    uint32_t nT, uint32_t ntiles, double* __restrict__ corr, double* __restrict__ cum,
    DeviceStatus* __restrict__ st) {
  constexpr int NB = D - 1;
  constexpr int NT = D - 2;
  constexpr int NV = 1 << NT;
  constexpr int NE = NV - 1;
  constexpr int NU = 1 << NB;
  using R = TsRec<NT>;
  constexpr int nTnode = node_offset<NT>(NT, 0u);
  __shared__ __align__(16) double s_t[nTnode + NV + 1];  // T nodes, p(V), failure flag
  __shared__ __align__(16) double s_b[kTsB * R::stride];
  const uint32_t lane = threadIdx.x;
  const size_t ldq = 2 * (size_t)M;

  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    // this tile's T: the last with tile0 <= tile
    uint32_t lo = 0, hi = nT - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (tl[mid].tile0 <= tile) lo = mid;
      else hi = mid - 1;
    }
    const ShardT T = tl[lo];
    uint32_t al = 0, bl = 0, nb = 0;
    (void)ts_tiles(T.b0lo, T.b0hi, (int64_t)(tile - T.tile0), &al, &bl, &nb);
    int tm[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) tm[j] = (int)T.t[j];
    __syncthreads();  // the previous tile's readers are done

    // ---------------- phase A: the T recursion (lane 0) ----------------
    if (lane == 0) {
      Tri<2 * NT> A;
      gather_q<NT>(Qi, M, tm, A);
      double pT[NV];
      bool bad = false;
      b_tree<NT, 0, 0u>(A, 1.0, s_t, pT, bad);
#pragma unroll
      for (int v = 0; v < NV; ++v) s_t[nTnode + v] = pT[v];
      s_t[nTnode + NV] = bad ? 1.0 : 0.0;
    }
    __syncthreads();
    const double* pT = s_t + nTnode;

    // ---------------- phase B: lane = b_0 ----------------
    if (lane < nb) {
      const int b0 = (int)(bl + lane);
      double* br = s_b + lane * R::stride;
      double C[2 * NT][2];
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const double* row = Qi + (size_t)(2 * tm[k]) * ldq + 2 * (size_t)b0;
        const double2 q0 = *reinterpret_cast<const double2*>(row);
        const double2 q1 = *reinterpret_cast<const double2*>(row + ldq);
        C[2 * k][0] = q0.x;
        C[2 * k][1] = q0.y;
        C[2 * k + 1][0] = q1.x;
        C[2 * k + 1][1] = q1.y;
      }
      const double* qb = Qi + (size_t)(2 * b0) * ldq + 2 * (size_t)b0;
      const double2 qb0 = *reinterpret_cast<const double2*>(qb);
      const double qb11 = qb[ldq + 1];
      bool bad = false;
      ts_border<NT, 0, 0u, true>(s_t, pT, C, qb0.x, qb0.y, qb11, br + R::oW, br + R::oL, bad);
      double p[NU], m[NU];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        p[2 * v] = pT[v];
        p[2 * v + 1] = br[R::oL + 4 * v + 3];
      }
      correlators_from_vacuum<NB, CONV>(p, m);
      br[R::oMB] = m[NU - 1];
      if constexpr (WK) {
        double cq[NU];
        cumulant_coefficients<NB, CONV>(m, cq);
#pragma unroll
        for (int u = 0; u < NU; ++u) br[R::oC + u] = cq[u];
      }
      br[R::oBad] = bad ? 1.0 : 0.0;
    }

    // ---------------- phase C: lane = a (registers) ----------------
    const uint32_t a = al + lane;
    const uint32_t ac = a < (uint32_t)tm[0] ? a : (uint32_t)tm[0] - 1u;  // in-bounds column
    double ca[NE][4], sa[NV][3], pat[NV];
    bool bad_a = false;
    {
      double C[2 * NT][2];
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const double* row = Qi + (size_t)(2 * tm[k]) * ldq + 2 * (size_t)ac;
        const double2 q0 = *reinterpret_cast<const double2*>(row);
        const double2 q1 = *reinterpret_cast<const double2*>(row + ldq);
        C[2 * k][0] = q0.x;
        C[2 * k][1] = q0.y;
        C[2 * k + 1][0] = q1.x;
        C[2 * k + 1][1] = q1.y;
      }
      const double* qa = Qi + (size_t)(2 * ac) * ldq + 2 * (size_t)ac;
      const double2 qa0 = *reinterpret_cast<const double2*>(qa);
      const double qa11 = qa[ldq + 1];
      double er[4 * NE], lr[4 * NV];
      ts_border<NT, 0, 0u, false>(s_t, pT, C, qa0.x, qa0.y, qa11, er, lr, bad_a);
#pragma unroll
      for (int e = 0; e < NE; ++e)
#pragma unroll
        for (int i = 0; i < 4; ++i) ca[e][i] = er[4 * e + i];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        sa[v][0] = lr[4 * v];
        sa[v][1] = lr[4 * v + 1];
        sa[v][2] = lr[4 * v + 2];
        pat[v] = lr[4 * v + 3];
      }
    }
    double nuT = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) nuT = fma(vacuum_sign<CONV>(2 * v), pat[v], nuT);
    bad_a |= s_t[nTnode + NV] != 0.0;
    __syncthreads();  // b_0 records written

    // ---------------- main loop: lane = a, over the b_0 ----------------
    for (uint32_t j = 0; j < nb; ++j) {
      const uint32_t b0 = bl + j;
      const uint32_t off = b0 * (b0 - 1) / 2 + a;
      const bool valid = a < b0 && off >= T.lo && off < T.hi;
      const double* br = s_b + j * R::stride;
      const double* qg = Qi + (size_t)(2 * b0) * ldq + 2 * (size_t)ac;
      const double2 g0 = *reinterpret_cast<const double2*>(qg);
      const double2 g1 = *reinterpret_cast<const double2*>(qg + ldq);
      double pab[NV];
      bool bad = false;
      ts_pair<NT, 0, 0u>(br, ca, sa, g0.x, g0.y, g1.x, g1.y, pab, bad);
      double nuB = nuT;
#pragma unroll
      for (int v = 0; v < NV; ++v) nuB = fma(vacuum_sign<CONV>(2 * v + 1), pab[v], nuB);
      const int64_t out = T.out0 + (int64_t)off;
      if (valid && (bad || bad_a || br[R::oBad] != 0.0))
        latch_failure(st, D, (int64_t)rank0 + out);
      if constexpr (WC) {
        const double mB = br[R::oMB];
        const double mS = (CONV == GBS_CLICK) ? mB - nuB : fma((NB & 1) ? -2.0 : 2.0, nuB, -mB);
        if (valid) corr[out] = mS;
      }
      if constexpr (WK) {
        double kS = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          kS = fma(br[R::oC + 2 * v], pat[v], kS);
          kS = fma(br[R::oC + 2 * v + 1], pab[v], kS);
        }
        if (valid) cum[out] = kS;
      }
    }
  }
}

template <int D, int CONV>
hipError_t launch_tshard_t(int M, const double* Qi, uint64_t rank0, const ShardT* tl, uint32_t nT,
                           uint32_t ntiles, double* corr, double* cum, DeviceStatus* st,
                           hipStream_t s) {
  const unsigned grid = std::min<uint32_t>(ntiles, 1u << 20);
  if (corr && cum)
    hipLaunchKernelGGL((forward_tshard_kernel<D, CONV, true, true>), dim3(grid), dim3(kTsA), 0, s,
                       Qi, M, rank0, tl, nT, ntiles, corr, cum, st);
  else if (corr)
    hipLaunchKernelGGL((forward_tshard_kernel<D, CONV, true, false>), dim3(grid), dim3(kTsA), 0,
                       s, Qi, M, rank0, tl, nT, ntiles, corr, cum, st);
  else
    hipLaunchKernelGGL((forward_tshard_kernel<D, CONV, false, true>), dim3(grid), dim3(kTsA), 0,
                       s, Qi, M, rank0, tl, nT, ntiles, corr, cum, st);
  return hipGetLastError();
}

// Largest b with C(b, 2) <= x.
uint32_t tri_root(uint64_t x) {
  uint64_t b = (uint64_t)((1.0 + std::sqrt(1.0 + 8.0 * (double)x)) / 2.0);
  while (b > 0 && b * (b - 1) / 2 > x) --b;
  while ((b + 1) * b / 2 <= x) ++b;
  return (uint32_t)b;
}

// T list of the start of an order-d rank range (colex order of T, tile
// offsets), at most max_t T's: returns how many ranks from rank0 on the list
// covers (count when it covers the whole range), so that a range of more T's
// runs as consecutive chunks.
constexpr size_t kTsMaxT = size_t(1) << 16;
uint64_t ts_build(int d, int M, uint64_t rank0, uint64_t count, std::vector<ShardT>& out,
                  uint32_t* ntiles, size_t max_t = kTsMaxT) {
  const int NT = d - 2;
  int32_t S[kMaxOrder];
  int t[3] = {0, 0, 0}, tl[3] = {0, 0, 0};
  (void)gbs_colex_unrank(d, (int64_t)rank0, S);
  for (int j = 0; j < NT; ++j) t[j] = S[j + 2];
  (void)gbs_colex_unrank(d, (int64_t)(rank0 + count - 1), S);
  for (int j = 0; j < NT; ++j) tl[j] = S[j + 2];
  uint64_t tiles = 0;
  out.clear();
  for (;;) {
    uint64_t base = 0;
    for (int j = 0; j < NT; ++j) base += host_binom(t[j], j + 3);
    const uint64_t tri = host_binom(t[0], 2);
    const uint64_t lo = rank0 > base ? rank0 - base : 0;
    const uint64_t end = rank0 + count;
    const uint64_t hi = end < base + tri ? end - base : tri;
    if (hi > lo) {
      ShardT e{};
      e.out0 = (int64_t)base - (int64_t)rank0;
      e.lo = (uint32_t)lo;
      e.hi = (uint32_t)hi;
      e.tile0 = (uint32_t)tiles;
      for (int j = 0; j < NT; ++j) e.t[j] = (uint16_t)t[j];
      e.b0lo = (uint16_t)tri_root(lo);
      e.b0hi = (uint16_t)tri_root(hi - 1);
      uint32_t al, bl, nb;
      const uint32_t n = ts_tiles(e.b0lo, e.b0hi, -1, &al, &bl, &nb);
      if (out.size() == max_t || tiles + n >= (uint64_t(1) << 32)) {
        *ntiles = (uint32_t)tiles;
        return base + lo - rank0;  // this T starts the next chunk
      }
      tiles += n;
      out.push_back(e);
    }
    bool last = true;
    for (int j = 0; j < NT; ++j) last = last && t[j] == tl[j];
    if (last) break;
    // colex successor among the NT-subsets of [0, M)
    for (int i = 0; i < NT; ++i) {
      const int lim = (i + 1 < NT) ? t[i + 1] : M;
      if (t[i] + 1 < lim) {
        ++t[i];
        for (int j = 0; j < i; ++j) t[j] = j;
        break;
      }
    }
  }
  *ntiles = (uint32_t)tiles;
  return count;
}

// Device copies of recent T lists, most recent first.  A caller holds its list
// by shared pointer until its launch is enqueued, so a list evicted meanwhile
// by another thread is freed only after that (hipFree waits for the device).
// The cache itself is never destroyed (no frees at process exit).
struct TsKey {
  int device, d, M;
  uint64_t rank0, count;
  bool operator==(const TsKey& o) const {
    return device == o.device && d == o.d && M == o.M && rank0 == o.rank0 && count == o.count;
  }
};
struct TsPlan {
  ShardT* dev = nullptr;
  uint32_t nT = 0, ntiles = 0;
  uint64_t covered = 0;  // ranks from rank0 on that the list covers
  TsPlan() = default;
  TsPlan(const TsPlan&) = delete;
  TsPlan& operator=(const TsPlan&) = delete;
  ~TsPlan() {
    if (dev) (void)hipFree(dev);
  }
};
constexpr size_t kTsCache = 8;
std::mutex g_ts_mu;
auto& g_ts = *new std::list<std::pair<TsKey, std::shared_ptr<TsPlan>>>();

// The T list of the start of a range (cached).
hipError_t ts_plan(int d, int M, uint64_t rank0, uint64_t count, std::shared_ptr<TsPlan>* out) {
  out->reset();
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return e;
  const TsKey key{device, d, M, rank0, count};
  std::shared_ptr<TsPlan> evicted;  // released after the lock
  std::lock_guard<std::mutex> lock(g_ts_mu);
  for (auto it = g_ts.begin(); it != g_ts.end(); ++it) {
    if (it->first == key) {
      g_ts.splice(g_ts.begin(), g_ts, it);
      *out = g_ts.front().second;
      return hipSuccess;
    }
  }
  std::vector<ShardT> host;
  uint32_t ntiles = 0;
  const uint64_t covered = ts_build(d, M, rank0, count, host, &ntiles);
  if (host.empty()) return hipErrorInvalidValue;  // a nonempty range has a T
  auto p = std::make_shared<TsPlan>();
  p->nT = (uint32_t)host.size();
  p->ntiles = ntiles;
  p->covered = covered;
  e = hipMalloc(&p->dev, host.size() * sizeof(ShardT));
  if (e != hipSuccess) {
    p->dev = nullptr;
    return e;
  }
  e = hipMemcpy(p->dev, host.data(), host.size() * sizeof(ShardT), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  g_ts.emplace_front(key, p);
  if (g_ts.size() > kTsCache) {
    evicted = std::move(g_ts.back().second);
    g_ts.pop_back();
  }
  *out = p;
  return hipSuccess;
}

}  // namespace

hipError_t launch_forward_shard(int d, int M, int flags, const double* Qi, uint64_t rank0,
                                uint64_t count, double* corr, double* cum, DeviceStatus* st,
                                hipStream_t s) {
  if (count == 0 || (!corr && !cum)) return hipSuccess;
  if (d < 3 || d > kMaxOrder) return hipErrorInvalidValue;
  using TsLaunch = hipError_t (*)(int, const double*, uint64_t, const ShardT*, uint32_t, uint32_t,
                                  double*, double*, DeviceStatus*, hipStream_t);
  const bool par = (flags & GBS_PARITY) != 0;
  TsLaunch fn;
  switch (d) {
    case 3: fn = par ? launch_tshard_t<3, GBS_PARITY> : launch_tshard_t<3, GBS_CLICK>; break;
    case 4: fn = par ? launch_tshard_t<4, GBS_PARITY> : launch_tshard_t<4, GBS_CLICK>; break;
    default: fn = par ? launch_tshard_t<5, GBS_PARITY> : launch_tshard_t<5, GBS_CLICK>; break;
  }
  // consecutive chunks of at most kTsMaxT T's each
  uint64_t done = 0;
  while (done < count) {
    std::shared_ptr<TsPlan> tp;
    hipError_t e = ts_plan(d, M, rank0 + done, count - done, &tp);
    if (e != hipSuccess) return e;
    e = fn(M, Qi, rank0 + done, tp->dev, tp->nT, tp->ntiles, corr ? corr + done : nullptr,
           cum ? cum + done : nullptr, st, s);
    if (e != hipSuccess) return e;
    done += tp->covered;
  }
  return hipSuccess;
}

}  // namespace gbs
