// Tiled order-recursive forward kernel (FP64, orders 3..5): the work that
// depends only on B = S \ {a} is done once per B and shared, through LDS, by
// the lanes that handle the subsets {a} + B, a < min B.
//
// Colex ranks are B-major: the subsets {a} + B, a = 0 .. b_0 - 1, occupy the
// consecutive ranks base(B) + a with base(B) = sum_j C(b_j, j + 2), and the
// B-blocks follow the colex order of the (d-1)-subsets B.  A tile is kTileB
// consecutive B's (colex index beta, rank sum_j C(b_j, j + 1)) and so a
// contiguous range of output ranks.
//
// Phase 1 (lane = B; each wave fills one part of the per-B record in LDS):
//   wave 0: Q_B = L L^T (Cholesky in the interleaved mode order b_0, .., e),
//           L with 1/L_ii on its diagonal, and p(b_0 .. b_j) for every prefix;
//   wave 1: m(B), m(W) for the non-empty W subset of B' = B \ {e}, k(R + {e})
//           and m(R + {e}) for R subset of B' (lower-order tables);
//   wave 2: the rank parts of the per-subset table reads;
//   wave 3: the run-start bitmap and the first run of every 64-rank window.
// Phase 2 (lane = subset, consecutive ranks across a wavefront), S = {a} + B:
//   1. y = L^{-1} Q_{B,a} by forward substitution.  For every prefix
//      U = {b_0 .. b_j} of B, Q_aa - y_U^T y_U is the Schur complement of Q_U
//      in Q_{U + a}, so p({a} + U) = p(U) det(Q_aa - y_U^T y_U)^(-1/2)
//      (App. D.1, Eq. vacuum_gaussian_prob: p(T) = det(Q_T)^(-1/2)); with
//      U = empty this is p({a}), with U = B it is p(S);
//   2. the other p({a} + U), U subset of B, come from the lower-order tables;
//   3. nu(W) and nu(W + e), the signed sums of p({a} + U) over U subset of W
//      (resp. W + e), W subset of B', by subset zeta transforms; then
//      m({a} + W) = m(W) - nu(W) and m({a} + W + e) = m(W + e) - nu(W + e)
//      (the inclusion-exclusion of Eq. corre_cov_main split by whether T
//      contains a; parity: -c + 2 (-1)^|.| nu with weights (-2)^|U|);
//   4. the cumulants k(Y + e) of the subsets Y of {a} + B' that contain a, in
//      increasing order, by k(Y + e) = m(Y + e) - sum_{R proper subset of Y}
//      k(R + e) m(Y \ R) (the partition sum of Eq. cumulant_corr_main grouped
//      by the block containing e; App. B, Eq. correlators_expanded_2); the
//      B-only k(R + e) come from LDS; Y = {a} + B' gives k(S).
// Per order-5 subset: 11 table reads, 8 16-byte reads of Q, one 8 x 2 forward
// substitution and five 2x2 determinants; the Cholesky of Q_B is paid once per
// B (about 29 subsets on average at M = 144).
#include <hip/hip_runtime.h>

#include "gbs_internal.h"

namespace gbs {

namespace {

constexpr int kTileB = 64;        // B's per tile (one per lane of wave 0)
constexpr int kTileThreads = 256;  // threads per workgroup (4 waves)

// Per-B record in LDS.  Doubles first (16-byte aligned), then 32-bit words.
template <int NB>
struct TileLayout {
  static constexpr int N = 2 * NB;                 // rows of Q_B
  static constexpr int NU = 1 << NB;               // subsets of B
  static constexpr int NP = 1 << (NB - 1);         // subsets of B'
  static constexpr int FULL = NU - 1;
  static constexpr int FULLP = NP - 1;
  // doubles
  static constexpr int dL = 0;                     // tri(i, j): L_ij (j < i), tri(i, i): 1/L_ii
  static constexpr int dP = tri_size(N);           // p(b_0 .. b_j), j = 0 .. NB-1
  static constexpr int dMB = dP + NB;              // m(B)
  static constexpr int dMW = dMB + 1;              // m(W), W = 1 .. FULLP (index W - 1)
  static constexpr int dKB = dMW + (NP - 1);       // k(R + e), R = 0 .. FULLP
  static constexpr int dME = dKB + NP;             // m(R + e), R = 0 .. FULLP
  static constexpr int nD = dME + NP;
  static constexpr int nDpad = (nD + 1) & ~1;
  // 32-bit words
  static constexpr int wStart = 0;                 // first rank of the B-block, tile relative
  static constexpr int wRow = 1;                   // byte offset of row 2 b_j of Q (NB words)
  static constexpr int wOP = wRow + NB;            // rank parts of p({a} + U), U not a prefix
  static constexpr int nOP = NU - (NB + 1);
  static constexpr int nW = wOP + nOP;
  static constexpr int nWpad = (nW + 3) & ~3;
  static constexpr int bytes = nDpad * 8 + nWpad * 4;  // multiple of 16
};

// U = {b_0 .. b_j} (bit mask 2^(j+1) - 1, or 0) is a prefix of B in the
// elimination order: p({a} + U) comes from the factorisation, the other
// p({a} + U) are read from the tables.
__host__ __device__ constexpr bool is_prefix(int u) { return (u & (u + 1)) == 0; }

// Index of a non-prefix U among the table reads.
__host__ __device__ constexpr int op_index(int u) {
  int n = 0;
  for (int v = 0; v < u; ++v) n += is_prefix(v) ? 0 : 1;
  return n;
}

}  // namespace

template <int D, int CONV, bool WANT_CUM>
__global__ __launch_bounds__(kTileThreads) void forward_tile_kernel(
    const double* __restrict__ Qi, const double* __restrict__ Qd, int M, uint64_t nB,
    const uint64_t* __restrict__ binom, OrderTables tab, double* __restrict__ m_out,
    double* __restrict__ k_out, double* __restrict__ p_out, DeviceStatus* __restrict__ st,
    int nwin_max) {
  constexpr int NB = D - 1;
  using TL = TileLayout<NB>;
  constexpr int N = TL::N;
  constexpr int NP = TL::NP;
  constexpr int FULL = TL::FULL;
  constexpr int FULLP = TL::FULLP;
  constexpr int EBIT = 1 << (NB - 1);

  extern __shared__ __align__(16) unsigned char smem[];
  // [records kTileB x TL::bytes][binomials (D+1) x (M+1) u32][bitmap nwin u64][first slot nwin u8]
  unsigned char* rec = smem;
  uint32_t* bin = reinterpret_cast<uint32_t*>(smem + kTileB * TL::bytes);
  const int ld = M + 1;
  uint64_t* bits = reinterpret_cast<uint64_t*>(bin + (((D + 1) * ld + 1) & ~1));
  unsigned char* first = reinterpret_cast<unsigned char*>(bits + nwin_max);
  __shared__ uint32_t s_ntile;  // ranks in the tile
  __shared__ uint32_t s_r0;     // rank of the tile's first subset

  for (int i = threadIdx.x; i < (D + 1) * ld; i += blockDim.x) {
    const int kk = i / ld, nn = i - kk * ld;
    bin[i] = (uint32_t)binom[kk * kBinLd + nn];
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t ntiles = (nB + kTileB - 1) / kTileB;
  const uint32_t ldq8 = 2u * (uint32_t)M * (uint32_t)sizeof(double);
  const double* Qodd = Qi + 2 * (size_t)M;  // odd rows (p quadratures)

  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();  // previous tile's readers are done; binomials are visible
    for (int i = threadIdx.x; i < nwin_max; i += blockDim.x) bits[i] = 0;
    __syncthreads();

    // ---------------- phase 1: lane = B, wave = part of the record ----------------
    {
      const uint64_t beta = tile * kTileB + lane;
      const bool valid = beta < nB;
      int b[NB];
      colex_unrank_est<NB>(valid ? beta : 0, M, bin, ld, b);
      uint32_t base = 0;
#pragma unroll
      for (int j = 0; j < NB; ++j) base += bin[(j + 2) * ld + b[j]];
      const uint32_t r0 = __builtin_amdgcn_readfirstlane(base);
      const bool nonempty = valid && b[0] >= 1;
      const uint64_t mask = __ballot(nonempty);
      const int c = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
      const uint32_t start = base - r0;  // first rank of this B's run, tile relative
      const uint32_t end = nonempty ? start + (uint32_t)b[0] : 0u;
      double* rd = reinterpret_cast<double*>(rec + c * TL::bytes);
      uint32_t* rw = reinterpret_cast<uint32_t*>(rec + c * TL::bytes + TL::nDpad * 8);
      if (wave == 0) {
        if (nonempty) {
          // Cholesky of Q_B (modes b_0 .. b_{NB-1}, interleaved x, p)
          Tri<N> A;
          gather_q<NB>(Qi, M, b, A);
          bool bad = false;
          double dinv[N];
#pragma unroll
          for (int i = 0; i < N; ++i) {
#pragma unroll
            for (int j = 0; j < i; ++j) {
              double v = A.a[tri(i, j)];
#pragma unroll
              for (int k = 0; k < j; ++k) v = fma(-A.a[tri(i, k)], A.a[tri(j, k)], v);
              A.a[tri(i, j)] = v * dinv[j];
            }
            double dd = A.a[tri(i, i)];
#pragma unroll
            for (int k = 0; k < i; ++k) dd = fma(-A.a[tri(i, k)], A.a[tri(i, k)], dd);
            bad |= !(dd > 0.0) || !(dd < INFINITY);
            dinv[i] = rsqrt_f64(dd);
            A.a[tri(i, i)] = dinv[i];
          }
          if (bad) latch_failure(st, D, (int64_t)base);
#pragma unroll
          for (int i = 0; i < tri_size(N); ++i) rd[TL::dL + i] = A.a[i];
          double pj = 1.0;  // p(b_0 .. b_j) = product of 1 / L_ii over its rows
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            pj *= dinv[2 * j] * dinv[2 * j + 1];
            rd[TL::dP + j] = pj;
          }
        }
      } else if (wave == 1) {
        if (nonempty) {
          // B-only correlators and cumulants from the lower-order tables
          uint32_t cb[NB][NB + 1];
#pragma unroll
          for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int kk = 1; kk <= NB; ++kk) cb[j][kk] = bin[kk * ld + b[j]];
          rd[TL::dMB] = load_at(tab.m[NB], (uint32_t)beta);
#pragma unroll
          for (int w = 1; w < NP; ++w) {  // m(W), W non-empty subset of B'
            uint32_t rk = 0;
            int pos = 0;
#pragma unroll
            for (int j = 0; j < NB - 1; ++j)
              if (w & (1 << j)) rk += cb[j][(pos++) + 1];
            rd[TL::dMW + w - 1] = load_at(tab.m[popcount_c((unsigned)w)], rk);
          }
          if constexpr (WANT_CUM) {
#pragma unroll
            for (int R = 0; R < NP; ++R) {  // k(R + e)
              uint32_t rk = 0;
              int pos = 0;
#pragma unroll
              for (int j = 0; j < NB - 1; ++j)
                if (R & (1 << j)) rk += cb[j][(pos++) + 1];
              rk += cb[NB - 1][pos + 1];
              rd[TL::dKB + R] = load_at(tab.k[pos + 1], rk);
              rd[TL::dME + R] = load_at(tab.m[pos + 1], rk);
            }
          }
        }
      } else if (wave == 2) {
        if (nonempty) {
          // rank parts of the per-subset reads, less the run start: with p the
          // tile-relative rank of {a} + B, rank({a} + U) = part(U) + a = part(U) - start + p
          // (a comes first, so the i-th element u_i of U adds C(u_i, i + 2))
          uint32_t cb[NB][NB + 2];
#pragma unroll
          for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int kk = 2; kk <= NB + 1; ++kk) cb[j][kk] = bin[kk * ld + b[j]];
          rw[TL::wStart] = start;
#pragma unroll
          for (int j = 0; j < NB; ++j) rw[TL::wRow + j] = 2u * (uint32_t)b[j] * ldq8;
#pragma unroll
          for (int u = 0; u < FULL; ++u) {
            if (is_prefix(u)) continue;
            uint32_t rk = 0;
            int pos = 0;
#pragma unroll
            for (int j = 0; j < NB; ++j)
              if (u & (1 << j)) rk += cb[j][(pos++) + 2];
            rw[TL::wOP + op_index(u)] = rk - start;
          }
        }
      } else {
        // ranks in the tile (end of the last non-empty run), the run-start
        // bitmap and the first run of every 64-rank window
        uint32_t ntile = end;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
          ntile = max(ntile, (uint32_t)__shfl_xor((int)ntile, off));
        if (lane == 0) {
          s_ntile = ntile;
          s_r0 = r0;
        }
        if (nonempty) {
          atomicOr(reinterpret_cast<unsigned int*>(bits) + (start >> 5), 1u << (start & 31));
          for (uint32_t w = (start + 63) >> 6; (w << 6) < end; ++w) first[w] = (unsigned char)c;
        }
      }
    }
    __syncthreads();

    // ---------------- phase 2: one lane per subset ----------------
    const uint32_t ntile = s_ntile;
    const uint32_t r0 = s_r0;
    const uint64_t lane_mask = lane == 63 ? ~1ull : ((2ull << lane) - 2ull);  // bits 1 .. lane
    for (uint32_t w = wave; (w << 6) < ntile; w += kTileThreads / 64) {
      const uint32_t p = (w << 6) + lane;
      if (p >= ntile) continue;
      const int c = (int)first[w] + __popcll(bits[w] & lane_mask);
      const double* rd = reinterpret_cast<const double*>(rec + c * TL::bytes);
      const uint32_t* rw = reinterpret_cast<const uint32_t*>(rec + c * TL::bytes + TL::nDpad * 8);
      const uint32_t a = p - rw[TL::wStart];
      const uint32_t r = r0 + p;

      // table reads (issued first; the factorisation below hides their latency)
      double pu[1 << NB];
#pragma unroll
      for (int u = 0; u < FULL; ++u) {
        if (is_prefix(u)) continue;
        pu[u] = load_at(tab.p[popcount_c((unsigned)u) + 1], rw[TL::wOP + op_index(u)] + p);
      }

      // y = L^{-1} Q_{B,a}; the Schur complement of Q_U in Q_{U + a} is
      // Q_aa - y_U^T y_U for every prefix U = {b_0 .. b_j} of B, so
      // p({a} + U) = p(U) det(Q_aa - y_U^T y_U)^(-1/2) (p({a}) for U empty)
      const double2 qd0 = load2_at(Qd, a << 5);
      const double qd2 = load_at(Qd, 4 * a + 2);
      double s00 = qd0.x, s10 = qd0.y, s11 = qd2;
      double y0[N], y1[N];
      bool bad = false;
      {
        const double det = fma(s00, s11, -s10 * s10);
        bad |= !(s00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
        pu[0] = rsqrt_f64(det);
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int j = i >> 1;
        // rows 2 b_j (x) and 2 b_j + 1 (p) of Q, columns 2a, 2a + 1
        const double2 q = load2_at((i & 1) ? Qodd : Qi, rw[TL::wRow + j] + (a << 4));
        double v0 = q.x, v1 = q.y;
#pragma unroll
        for (int k = 0; k < i; ++k) {
          const double l = rd[TL::dL + tri(i, k)];
          v0 = fma(-l, y0[k], v0);
          v1 = fma(-l, y1[k], v1);
        }
        const double di = rd[TL::dL + tri(i, i)];
        y0[i] = v0 * di;
        y1[i] = v1 * di;
        s00 = fma(-y0[i], y0[i], s00);
        s10 = fma(-y0[i], y1[i], s10);
        s11 = fma(-y1[i], y1[i], s11);
        if (i & 1) {
          const double det = fma(s00, s11, -s10 * s10);
          bad |= !(s00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
          pu[(2 << j) - 1] = rd[TL::dP + j] * rsqrt_f64(det);
        }
      }
      if (bad) latch_failure(st, D, (int64_t)r);
      const double pS = pu[FULL];

      // nu(W) = sum over U subset of W of s_|U| p({a} + U) for W subset of B'
      // (subset zeta transform), then the correlators m({a} + W) = m(W) - nu(W)
      // (click) or -c(W) + 2 (-1)^|W| nu(W) (parity), m(empty) = 1
      double nu[NP];
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        const int t = popcount_c((unsigned)u);
        nu[u] = (CONV == GBS_CLICK) ? ((t & 1) ? -pu[u] : pu[u])
                                    : ((t & 1) ? -1.0 : 1.0) * (double)(1 << t) * pu[u];
      }
      double nue[NP];  // the same over the sets U + e
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        const int t = popcount_c((unsigned)u) + 1;
        nue[u] = ((CONV == GBS_CLICK) ? ((t & 1) ? -1.0 : 1.0)
                                      : ((t & 1) ? -1.0 : 1.0) * (double)(1 << t)) * pu[u | EBIT];
      }
#pragma unroll
      for (int bit = 0; bit < NB - 1; ++bit)
#pragma unroll
        for (int u = 0; u < NP; ++u)
          if (u & (1 << bit)) {
            nu[u] += nu[u ^ (1 << bit)];
            nue[u] += nue[u ^ (1 << bit)];
          }
      double mwa[NP];  // m({a} + W), W subset of B'
#pragma unroll
      for (int w = 0; w < NP; ++w) {
        const double mw = w ? rd[TL::dMW + w - 1] : 1.0;
        if constexpr (CONV == GBS_CLICK) mwa[w] = mw - nu[w];
        else mwa[w] = fma((popcount_c((unsigned)w) & 1) ? -2.0 : 2.0, nu[w], -mw);
      }
      const double nuB = nu[FULLP] + nue[FULLP];
      const double mB = rd[TL::dMB];
      double mS;
      if constexpr (CONV == GBS_CLICK) mS = mB - nuB;
      else mS = fma((NB & 1) ? -2.0 : 2.0, nuB, -mB);
      if (m_out) store_at(m_out, r, mS);
      if (p_out) store_at(p_out, r, pS);

      if constexpr (WANT_CUM) {
        // K(Y) = k(Y + e) for Y subset of X = {a} + B' (bit 0 of Y = a, bit
        // i + 1 = b_i): B-only ones from LDS, the ones containing a by the
        // fixed-element recursion K(Y) = m(Y + e) - sum_{R proper subset of Y} K(R) m(Y \ R)
        constexpr int NX = 2 * NP;
        double Kv[NX];
#pragma unroll
        for (int R = 0; R < NP; ++R) Kv[2 * R] = rd[TL::dKB + R];
        auto mu_x = [&](int Y) -> double {  // m(Y), Y non-empty subset of X
          return (Y & 1) ? mwa[Y >> 1] : rd[TL::dMW + (Y >> 1) - 1];
        };
#pragma unroll
        for (int Y = 1; Y < NX; Y += 2) {
          const int W = Y >> 1;  // Y = {a} + W
          double v;
          if constexpr (CONV == GBS_CLICK) v = rd[TL::dME + W] - (nu[W] + nue[W]);
          else v = fma((popcount_c((unsigned)W) & 1) ? 2.0 : -2.0, nu[W] + nue[W], -rd[TL::dME + W]);
#pragma unroll
          for (int R = 0; R < Y; ++R)
            if ((R & Y) == R) v = fma(-Kv[R], mu_x(Y ^ R), v);
          Kv[Y] = v;
        }
        store_at(k_out, r, Kv[NX - 1]);
      }
    }
  }
}

bool tile_supported(int d, int M, int flags) {
  if (d < 3 || d > kMaxOrder || (flags & GBS_MIXED)) return false;
  for (int q = 1; q <= d; ++q)
    if (host_binom(M, q) >= (1ull << 29)) return false;
  return true;
}

template <int D, int CONV, bool WC>
static hipError_t launch_tile_t(int M, const double* Qi, const double* Qd, const uint64_t* binom,
                                const OrderTables& tab, double* m_out, double* k_out,
                                double* p_out, DeviceStatus* st, hipStream_t s) {
  constexpr int NB = D - 1;
  const uint64_t nB = host_binom(M, NB);
  const uint64_t ntiles = (nB + kTileB - 1) / kTileB;
  if (ntiles == 0 || host_binom(M, D) == 0) return hipSuccess;
  // ranks per tile <= kTileB * (M - NB): the run of B has b_0 <= M - NB subsets
  const int nwin = (int)((kTileB * (uint64_t)(M - NB) + 63) / 64) + 1;
  const size_t lds = (size_t)kTileB * TileLayout<NB>::bytes +
                     (size_t)(((D + 1) * (M + 1) + 1) & ~1) * sizeof(uint32_t) +
                     (size_t)nwin * (sizeof(uint64_t) + 1);
  if (lds > 64 * 1024) return hipErrorInvalidConfiguration;
  const uint64_t grid = std::min<uint64_t>(ntiles, kMaxGrid);
  hipLaunchKernelGGL((forward_tile_kernel<D, CONV, WC>), dim3((unsigned)grid), dim3(kTileThreads),
                     lds, s, Qi, Qd, M, nB, binom, tab, m_out, k_out, p_out, st, nwin);
  return hipGetLastError();
}

template <int D>
static hipError_t launch_tile_c(int M, int flags, const double* Qi, const double* Qd,
                                const uint64_t* binom, const OrderTables& tab, double* m_out,
                                double* k_out, double* p_out, DeviceStatus* st, hipStream_t s) {
  if (flags & GBS_PARITY) {
    if (k_out) return launch_tile_t<D, GBS_PARITY, true>(M, Qi, Qd, binom, tab, m_out, k_out, p_out, st, s);
    return launch_tile_t<D, GBS_PARITY, false>(M, Qi, Qd, binom, tab, m_out, k_out, p_out, st, s);
  }
  if (k_out) return launch_tile_t<D, GBS_CLICK, true>(M, Qi, Qd, binom, tab, m_out, k_out, p_out, st, s);
  return launch_tile_t<D, GBS_CLICK, false>(M, Qi, Qd, binom, tab, m_out, k_out, p_out, st, s);
}

hipError_t launch_forward_tile(int d, int M, int flags, const double* Qi, const double* Qd,
                               const uint64_t* binom, const OrderTables& tab, double* m_out,
                               double* k_out, double* p_out, DeviceStatus* st, hipStream_t s) {
  switch (d) {
    case 3: return launch_tile_c<3>(M, flags, Qi, Qd, binom, tab, m_out, k_out, p_out, st, s);
    case 4: return launch_tile_c<4>(M, flags, Qi, Qd, binom, tab, m_out, k_out, p_out, st, s);
    case 5: return launch_tile_c<5>(M, flags, Qi, Qd, binom, tab, m_out, k_out, p_out, st, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gbs
