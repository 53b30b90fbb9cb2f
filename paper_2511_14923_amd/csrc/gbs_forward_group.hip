// Group-tiled forward kernel (FP64, orders 3..5).
//
// For S = {a} + B, B = {b_0 < b_1 < .. < e}, write B = {b_0} + T with
// T = P + {e}, P = B \ {b_0, e}.  The subsets that share T form a group: the
// pairs (a, b_0) with a < b_0 < min T, at consecutive colex ranks.  Q_S is
// factored in the block order [P, b_0, e, a], so the work splits by what it
// depends on:
//   (T)         the Cholesky rows of P and of e against P;
//   (T, a)      y_P = L_P^{-1} Q_{P,a}, the Schur complement Q_aa - y_P^T y_P of
//               Q_P in Q_{P + a}, t_e = Q_{e,a} - L_{e,P} y_P, and p({a} + U) for
//               every U subset of T;
//   (B)         the Cholesky rows of b_0 and e (against P and b_0);
//   (a, B)      y_{b_0}, y_e: two block rows of the forward substitution.
// With det(Q_{U + a}) = det(Q_U) det(Q_aa - y_U^T y_U) for every leading set U
// of the order (App. D.1, Eq. vacuum_gaussian_prob: p(T) = det(Q_T)^(-1/2)),
// the subset itself needs only p(B' + a) = p(S \ e) and p(S), from two 2x2
// determinants, plus the p({a} + U) with b_0 in U that are not leading sets,
// read from the tables of the lower orders.  Correlators and cumulants follow
// as in the tile kernel (gbs_forward_tile.hip): subset zeta transforms for
// nu(W) and nu(W + e), m({a} + W) = m(W) - nu(W) (Eq. corre_cov_main split by
// whether T contains a), and the fixed-element recursion on e for the
// cumulants (Eq. cumulant_corr_main grouped by the block containing e; App. B,
// Eq. correlators_expanded_2).
//
// Displaced states (first moments mu, Eq. vacuum_gaussian_prob): the same
// factorisation also gives z = L^{-1} mu in the order [P, b_0, e] (z_P and
// z_e(T) once per group, z_{b_0} and z_e(B) once per B), and for a leading set
// U of the order the quadratic form splits as
//   mu_{U+a}^T Q_{U+a}^{-1} mu_{U+a} = |z_U|^2 + r^T (Q_aa - y_U^T y_U)^{-1} r,
//   r = mu_a - y_U^T z_U,
// so every probability computed here gains exp(-q/2) from two more 2-vectors
// per block row; |z|^2 of the T, B' and B parts is folded into the per-group
// and per-B probabilities.
//
// A tile is a run of consecutive B's (at most GL::kB) whose groups need at
// most rmax (T, a) records; the host plans the tiles once per (M, d).  Per
// tile: phase 1 builds the per-B records (lane = B, one part per wave) and the
// group list; phase 1b builds the (T, a) records (one per thread); phase 2
// takes one subset per lane, consecutive ranks across a wavefront.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "gbs_internal.h"

namespace gbs {

namespace {

constexpr int kGroupB = 40;         // B's per tile at most
constexpr int kGroupG = 16;         // groups per tile at most
constexpr int kGroupThreads = 256;  // threads per workgroup (4 waves)
constexpr int kGroupRmax = 148;     // (T, a) records per tile at most (M - d + 1 needed)

template <int NB, bool DISP>
struct GroupLayout {
  // B's per tile: fewer for displaced states, whose larger records must still
  // let three workgroups share a compute unit's LDS
  static constexpr int kB = DISP ? 36 : kGroupB;
  static constexpr int NPm = NB - 2;       // |P|
  static constexpr int NT = NB - 1;        // |T|
  static constexpr int NTS = 1 << NT;      // subsets of T
  static constexpr int N = 2 * NB;         // rows of Q_B
  static constexpr int NU = 1 << NB;       // subsets of B (bit 0: b_0, bit i: b_i)
  static constexpr int NP = 1 << (NB - 1); // subsets of B' = B \ {e}
  static constexpr int FULL = NU - 1;
  static constexpr int FULLP = NP - 1;
  // per-B record, doubles
  static constexpr int dLb = 0;                 // b_0 rows: [r][k < 2|P|], then 1/L, L, 1/L of the b_0 block
  static constexpr int nLb = 4 * NPm + 3;
  static constexpr int dLe = dLb + nLb;         // e rows against b_0 ([r][2]), then the e block
  static constexpr int nLe = 7;
  static constexpr int dP = dLe + nLe;          // p(B'), p(B) (displaced: with exp(-|z|^2 / 2))
  static constexpr int dMB = dP + 2;            // m(B)
  static constexpr int dMW = dMB + 1;           // m(W), W = 1 .. FULLP (index W - 1)
  static constexpr int dKB = dMW + (NP - 1);    // k(R + e), R = 0 .. FULLP
  static constexpr int dME = dKB + NP;          // m(R + e), R = 0 .. FULLP
  static constexpr int dZ = dME + NP;           // displaced: z_{b_0} [2], z_e(B) [2]
  static constexpr int nD = dZ + (DISP ? 4 : 0);
  static constexpr int nDpad = (nD + 1) & ~1;
  // per-B record, 32-bit words
  static constexpr int wStart = 0;              // first rank of the B-block, tile relative
  static constexpr int wRow = 1;                // byte offset of row 2 b_0 of Q
  static constexpr int wRbase = 2;              // (T, a) record of a = 0 for this B's group
  static constexpr int wOP = 3;                 // rank parts (less start) of p({a} + U), b_0 in U
  static constexpr int nOP = NP - 2;            // all U containing b_0 except B' and B
  static constexpr int wG = wOP + nOP;          // this B's group (displaced states)
  static constexpr int nW = wG + (DISP ? 1 : 0);
  static constexpr int nWpad = (nW + 3) & ~3;
  static constexpr int bytes = nDpad * 8 + nWpad * 4;
  // (T, a) record, doubles; stored as 16-byte units, unit q of record i at
  // [q][i], so that consecutive records (consecutive a across a wavefront) fall
  // in consecutive LDS banks
  static constexpr int rY = 0;                  // y_P [k < 2|P|][2]
  static constexpr int rT = rY + 4 * NPm;       // t_e [r][2]
  static constexpr int rS = rT + 4;             // Schur complement of Q_P in Q_{P + a}: s00, s10, s11
  static constexpr int rPT = rS + 4;            // p({a} + U), U subset of T (T bit i <-> B bit i + 1)
  static constexpr int rN = rPT + NTS;
  static constexpr int rUnits = (rN + 1) / 2;
  static constexpr int rbytes = rUnits * 16;    // per record
  // per-group record (Cholesky of Q_T in the order P, e), doubles
  static constexpr int I0 = 2 * NPm;            // rows of P
  static constexpr int gP = 0;                  // L_P: tri(i, j), 1/L_ii on the diagonal
  static constexpr int gE = gP + tri_size(I0);  // e rows against P: [r][k < I0]
  static constexpr int gS = gE + 2 * I0;        // Q_ee - L_eP L_eP^T: s00, s10, s11
  static constexpr int gEd = gS + 3;            // e block of Q_T: 1/L, L, 1/L
  static constexpr int gpP = gEd + 3;           // p(P) (displaced: with exp(-|z_P|^2 / 2))
  static constexpr int gpT = gpP + 1;           // p(T) (displaced: with exp(-|z_T|^2 / 2))
  static constexpr int gZ = gpT + 1;            // displaced: z_P [2|P|], z_e(T) [2]
  static constexpr int gN = ((gZ + (DISP ? I0 + 2 : 0)) + 1) & ~1;
  static constexpr int gbytes = gN * 8;
};

// Index among the per-subset table reads of a B-subset U that contains b_0.
template <int NB>
__host__ __device__ constexpr int gop_index(int u) {
  int n = 0;
  for (int v = 0; v < u; ++v)
    n += ((v & 1) && v != (1 << (NB - 1)) - 1 && v != (1 << NB) - 1) ? 1 : 0;
  return n;
}

// Leading sets of T in the order [P, e]: empty, {P_0}, .., P, T.
template <int NT>
__host__ __device__ constexpr bool t_leading(int t) {
  return t == (1 << NT) - 1 || ((t & (t + 1)) == 0 && t < (1 << (NT - 1)));
}

}  // namespace

template <int D, int CONV, bool WANT_CUM, bool DISP>
__global__ __launch_bounds__(kGroupThreads) void forward_group_kernel(
    const double* __restrict__ Qi, const double* __restrict__ Qd,
    const double* __restrict__ mi, int M,
    const uint64_t* __restrict__ plan, uint32_t ntiles, const uint64_t* __restrict__ binom,
    OrderTables tab, double* __restrict__ m_out, double* __restrict__ k_out,
    double* __restrict__ p_out, DeviceStatus* __restrict__ st, int nwin_max) {
  constexpr int rmax = kGroupRmax;
  constexpr int NB = D - 1;
  using GL = GroupLayout<NB, DISP>;
  constexpr int NPm = GL::NPm;
  constexpr int NT = GL::NT;
  constexpr int NTS = GL::NTS;
  constexpr int N = GL::N;
  constexpr int NP = GL::NP;
  constexpr int FULL = GL::FULL;
  constexpr int FULLP = GL::FULLP;
  constexpr int EBIT = 1 << (NB - 1);

  extern __shared__ __align__(16) unsigned char smem[];
  // [B records][(T, a) records][group records][binomials][bitmap][first run per window]
  unsigned char* brec = smem;
  unsigned char* rrec = smem + GL::kB * GL::bytes;
  double* grec = reinterpret_cast<double*>(rrec + (size_t)rmax * GL::rbytes);
  uint32_t* bin = reinterpret_cast<uint32_t*>(grec + kGroupG * GL::gN);
  const int ld = M + 1;
  uint64_t* bits = reinterpret_cast<uint64_t*>(bin + (((D + 1) * ld + 1) & ~1));
  unsigned char* first = reinterpret_cast<unsigned char*>(bits + nwin_max);
  __shared__ uint32_t s_ntile, s_r0, s_ngroups, s_nrec;
  __shared__ uint32_t s_gbase[kGroupG];      // first (T, a) record of each group
  __shared__ int s_gT[kGroupG][NB - 1];       // modes of T, in the order P, e

  for (int i = threadIdx.x; i < (D + 1) * ld; i += blockDim.x) {
    const int kk = i / ld, nn = i - kk * ld;
    bin[i] = (uint32_t)binom[kk * kBinLd + nn];
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint32_t ldq8 = 2u * (uint32_t)M * (uint32_t)sizeof(double);
  const double* Qodd = Qi + 2 * (size_t)M;  // odd rows (p quadratures)

  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t desc = plan[tile];
    const uint32_t beta0 = (uint32_t)desc;
    const int nBt = (int)(desc >> 32);
    __syncthreads();  // the previous tile's readers are done; binomials are visible
    for (int i = threadIdx.x; i < nwin_max; i += blockDim.x) bits[i] = 0;
    __syncthreads();

    // ---------------- phase 1: lane = B, wave = part of the record ----------------
    {
      const bool valid = lane < nBt;
      const uint32_t beta = beta0 + (valid ? lane : 0);
      int b[NB];
      colex_unrank_est<NB>(beta, M, bin, ld, b);
      uint32_t base = 0;
#pragma unroll
      for (int j = 0; j < NB; ++j) base += bin[(j + 2) * ld + b[j]];
      const uint32_t r0 = __builtin_amdgcn_readfirstlane(base);
      const bool nonempty = valid && b[0] >= 1;
      const uint64_t mask = __ballot(nonempty);
      const int c = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
      const uint32_t start = base - r0;
      const uint32_t end = nonempty ? start + (uint32_t)b[0] : 0u;
      // groups: runs of equal T = B \ {b_0}; (T, a) records a < max b_0 of the group in the tile
      uint64_t key = 0;  // T's modes, 11 bits each
#pragma unroll
      for (int j = 1; j < NB; ++j) key = (key << 11) | (uint64_t)b[j];
      const uint64_t key_prev = __shfl_up(key, 1);
      const uint64_t key_next = __shfl_down(key, 1);
      const bool gstart = valid && (lane == 0 || key != key_prev);
      const bool glast = valid && (lane == nBt - 1 || key != key_next);
      const uint64_t gmask = __ballot(gstart);
      const int g = __builtin_amdgcn_mbcnt_hi((uint32_t)(gmask >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)gmask, 0u)) +
                    (gstart ? 0 : -1);
      const uint32_t contrib = glast ? (uint32_t)b[0] : 0u;
      uint32_t incl = contrib;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
      }
      const uint32_t gbase = incl - contrib;  // records before this lane's group
      double* rd = reinterpret_cast<double*>(brec + c * GL::bytes);
      uint32_t* rw = reinterpret_cast<uint32_t*>(brec + c * GL::bytes + GL::nDpad * 8);
      constexpr int I0 = GL::I0;
      if (wave == 0) {
        if (gstart) {
          // Cholesky of Q_T in the order P, e (interleaved x, p), once per group
          int tm[NT];
#pragma unroll
          for (int j = 0; j < NT; ++j) tm[j] = b[j + 1];
          constexpr int NTT = 2 * NT;
          Tri<NTT> A;
#pragma unroll
          for (int jb = 0; jb < NT; ++jb) {
#pragma unroll
            for (int kb = 0; kb <= jb; ++kb) {
              const uint32_t off = 2u * (uint32_t)tm[jb] * ldq8 + 16u * (uint32_t)tm[kb];
              const double2 q0 = load2_at(Qi, off);
              const double2 q1 = load2_at(Qodd, off);
              A.a[tri(2 * jb, 2 * kb)] = q0.x;
              A.a[tri(2 * jb + 1, 2 * kb)] = q1.x;
              A.a[tri(2 * jb + 1, 2 * kb + 1)] = q1.y;
              if (kb != jb) A.a[tri(2 * jb, 2 * kb + 1)] = q0.y;
            }
          }
          const double qe00 = A.a[tri(I0, I0)], qe10 = A.a[tri(I0 + 1, I0)];
          const double qe11 = A.a[tri(I0 + 1, I0 + 1)];
          bool bad = false;
          double dinv[NTT];
#pragma unroll
          for (int i = 0; i < NTT; ++i) {
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
          }
          if (bad) {  // T is an order d-2 subset with a non-positive pivot
            uint32_t rk = 0;
#pragma unroll
            for (int j = 0; j < NT; ++j) rk += bin[(j + 1) * ld + tm[j]];
            latch_failure(st, D - 2, (int64_t)rk);
          }
          double* gr = grec + g * GL::gN;
          double se00 = qe00, se10 = qe10, se11 = qe11;
          double pP = 1.0;
#pragma unroll
          for (int i = 0; i < I0; ++i) {
#pragma unroll
            for (int j = 0; j < i; ++j) gr[GL::gP + tri(i, j)] = A.a[tri(i, j)];
            gr[GL::gP + tri(i, i)] = dinv[i];
            pP *= dinv[i];
          }
#pragma unroll
          for (int k = 0; k < I0; ++k) {
            const double l0 = A.a[tri(I0, k)], l1 = A.a[tri(I0 + 1, k)];
            gr[GL::gE + k] = l0;
            gr[GL::gE + I0 + k] = l1;
            se00 = fma(-l0, l0, se00);
            se10 = fma(-l1, l0, se10);
            se11 = fma(-l1, l1, se11);
          }
          gr[GL::gS + 0] = se00;
          gr[GL::gS + 1] = se10;
          gr[GL::gS + 2] = se11;
          gr[GL::gEd + 0] = dinv[I0];
          gr[GL::gEd + 1] = A.a[tri(I0 + 1, I0)];
          gr[GL::gEd + 2] = dinv[I0 + 1];
          double eP = 1.0, eT = 1.0;
          if constexpr (DISP) {
            // z_T = L_T^{-1} mu_T (order P, e); |z_P|^2 and |z_T|^2
            double z[NTT];
            double qP = 0.0, qT = 0.0;
#pragma unroll
            for (int i = 0; i < NTT; ++i) {
              double v = mi[2 * tm[i >> 1] + (i & 1)];
#pragma unroll
              for (int k = 0; k < i; ++k) v = fma(-A.a[tri(i, k)], z[k], v);
              z[i] = v * dinv[i];
              gr[GL::gZ + i] = z[i];
              if (i < I0) qP = fma(z[i], z[i], qP);
              qT = fma(z[i], z[i], qT);
            }
            eP = exp(-0.5 * qP);
            eT = exp(-0.5 * qT);
          }
          gr[GL::gpP] = pP * eP;
          gr[GL::gpT] = pP * dinv[I0] * dinv[I0 + 1] * eT;
        }
      } else if (wave == 1) {
        if (nonempty) {
          // B-only correlators and cumulants from the lower-order tables
          uint32_t cb[NB][NB + 1];
#pragma unroll
          for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int kk = 1; kk <= NB; ++kk) cb[j][kk] = bin[kk * ld + b[j]];
          rd[GL::dMB] = load_at(tab.m[NB], beta);
#pragma unroll
          for (int w = 1; w < NP; ++w) {  // m(W), W non-empty subset of B'
            uint32_t rk = 0;
            int pos = 0;
#pragma unroll
            for (int j = 0; j < NB - 1; ++j)
              if (w & (1 << j)) rk += cb[j][(pos++) + 1];
            rd[GL::dMW + w - 1] = load_at(tab.m[popcount_c((unsigned)w)], rk);
          }
          if constexpr (WANT_CUM) {
#pragma unroll
            for (int R = 0; R < NP; ++R) {  // k(R + e), m(R + e)
              uint32_t rk = 0;
              int pos = 0;
#pragma unroll
              for (int j = 0; j < NB - 1; ++j)
                if (R & (1 << j)) rk += cb[j][(pos++) + 1];
              rk += cb[NB - 1][pos + 1];
              rd[GL::dKB + R] = load_at(tab.k[pos + 1], rk);
              rd[GL::dME + R] = load_at(tab.m[pos + 1], rk);
            }
          }
        }
      } else if (wave == 2) {
        if (nonempty) {
          // rank parts of the per-subset reads, less the run start: with p the
          // tile-relative rank of {a} + B, rank({a} + U) = part(U) - start + p
          // (a comes first, so the i-th element u_i of U adds C(u_i, i + 2))
          uint32_t cb[NB][NB + 2];
#pragma unroll
          for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int kk = 2; kk <= NB + 1; ++kk) cb[j][kk] = bin[kk * ld + b[j]];
          rw[GL::wStart] = start;
          rw[GL::wRow] = 2u * (uint32_t)b[0] * ldq8;
          rw[GL::wRbase] = gbase;
          if constexpr (DISP) rw[GL::wG] = (uint32_t)g;
#pragma unroll
          for (int u = 1; u < FULL; u += 2) {
            if (u == FULLP) continue;
            uint32_t rk = 0;
            int pos = 0;
#pragma unroll
            for (int j = 0; j < NB; ++j)
              if (u & (1 << j)) rk += cb[j][(pos++) + 2];
            rw[GL::wOP + gop_index<NB>(u)] = rk - start;
          }
        }
      } else {
        // tile size, run bitmap, first run of every 64-rank window, group list
        uint32_t ntile = end;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
          ntile = max(ntile, (uint32_t)__shfl_xor((int)ntile, off));
        if (lane == 0) {
          s_ntile = ntile;
          s_r0 = r0;
          s_ngroups = (uint32_t)__popcll(gmask);
        }
        if (lane == nBt - 1) s_nrec = incl;
        if (gstart) {
          s_gbase[g] = gbase;
#pragma unroll
          for (int j = 0; j < NB - 1; ++j) s_gT[g][j] = b[j + 1];
        }
        if (nonempty) {
          atomicOr(reinterpret_cast<unsigned int*>(bits) + (start >> 5), 1u << (start & 31));
          for (uint32_t w = (start + 63) >> 6; (w << 6) < end; ++w) first[w] = (unsigned char)c;
        }
      }
    }
    __syncthreads();

    // ---------------- phase 1b: B rows (wave 0), (T, a) records (waves 1-3) ----------------
    if (wave == 0) {
      const bool valid = lane < nBt;
      const uint32_t beta = beta0 + (valid ? lane : 0);
      int b[NB];
      colex_unrank_est<NB>(beta, M, bin, ld, b);
      const bool nonempty = valid && b[0] >= 1;
      const uint64_t mask = __ballot(nonempty);
      const int c = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
      uint64_t key = 0;
#pragma unroll
      for (int j = 1; j < NB; ++j) key = (key << 11) | (uint64_t)b[j];
      const uint64_t key_prev = __shfl_up(key, 1);
      const bool gstart = valid && (lane == 0 || key != key_prev);
      const uint64_t gmask = __ballot(gstart);
      const int g = __builtin_amdgcn_mbcnt_hi((uint32_t)(gmask >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)gmask, 0u)) +
                    (gstart ? 0 : -1);
      if (nonempty) {
        // rows of b_0 and e of the Cholesky factor of Q_B in the order P, b_0, e,
        // from the group's factor of Q_T
        constexpr int I0 = GL::I0;
        const double* gr = grec + g * GL::gN;
        double* rd = reinterpret_cast<double*>(brec + c * GL::bytes);
        const int b0 = b[0], e = b[NB - 1];
        double lb[2][I0 > 0 ? I0 : 1];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
#pragma unroll
          for (int k = 0; k < I0; ++k) {
            const double2 q = load2_at(r ? Qodd : Qi, 2u * (uint32_t)b0 * ldq8 + 16u * (uint32_t)b[1 + (k >> 1)]);
            double v = (k & 1) ? q.y : q.x;
#pragma unroll
            for (int j = 0; j < k; ++j) v = fma(-lb[r][j], gr[GL::gP + tri(k, j)], v);
            lb[r][k] = v * gr[GL::gP + tri(k, k)];
          }
        }
        const double2 qd0 = load2_at(Qd, (uint32_t)b0 << 5);
        const double qd2 = load_at(Qd, 4u * (uint32_t)b0 + 2u);
        double d0 = qd0.x, l10 = qd0.y, d1 = qd2;
#pragma unroll
        for (int k = 0; k < I0; ++k) {
          d0 = fma(-lb[0][k], lb[0][k], d0);
          l10 = fma(-lb[1][k], lb[0][k], l10);
          d1 = fma(-lb[1][k], lb[1][k], d1);
        }
        bool bad = !(d0 > 0.0) || !(d0 < INFINITY);
        const double ib0 = rsqrt_f64(d0);
        l10 *= ib0;
        d1 = fma(-l10, l10, d1);
        bad |= !(d1 > 0.0) || !(d1 < INFINITY);
        const double ib1 = rsqrt_f64(d1);
        // e rows against b_0, then the e block
        const double2 qe0 = load2_at(Qi, 2u * (uint32_t)e * ldq8 + 16u * (uint32_t)b0);
        const double2 qe1 = load2_at(Qodd, 2u * (uint32_t)e * ldq8 + 16u * (uint32_t)b0);
        double le[2][2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          double v0 = r ? qe1.x : qe0.x, v1 = r ? qe1.y : qe0.y;
#pragma unroll
          for (int k = 0; k < I0; ++k) {
            const double l = gr[GL::gE + r * I0 + k];
            v0 = fma(-l, lb[0][k], v0);
            v1 = fma(-l, lb[1][k], v1);
          }
          le[r][0] = v0 * ib0;
          le[r][1] = fma(-le[r][0], l10, v1) * ib1;
        }
        const double e00 = gr[GL::gS + 0] - le[0][0] * le[0][0] - le[0][1] * le[0][1];
        const double e10 = gr[GL::gS + 1] - le[1][0] * le[0][0] - le[1][1] * le[0][1];
        double e11 = gr[GL::gS + 2] - le[1][0] * le[1][0] - le[1][1] * le[1][1];
        bad |= !(e00 > 0.0) || !(e00 < INFINITY);
        const double iex = rsqrt_f64(e00);
        const double lpx = e10 * iex;
        e11 = fma(-lpx, lpx, e11);
        bad |= !(e11 > 0.0) || !(e11 < INFINITY);
        const double iep = rsqrt_f64(e11);
        if (bad) {
          uint32_t base = 0;
#pragma unroll
          for (int j = 0; j < NB; ++j) base += bin[(j + 2) * ld + b[j]];
          latch_failure(st, D, (int64_t)base);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int k = 0; k < I0; ++k) rd[GL::dLb + r * I0 + k] = lb[r][k];
        rd[GL::dLb + 2 * I0 + 0] = ib0;
        rd[GL::dLb + 2 * I0 + 1] = l10;
        rd[GL::dLb + 2 * I0 + 2] = ib1;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          rd[GL::dLe + 2 * r + 0] = le[r][0];
          rd[GL::dLe + 2 * r + 1] = le[r][1];
        }
        rd[GL::dLe + 4] = iex;
        rd[GL::dLe + 5] = lpx;
        rd[GL::dLe + 6] = iep;
        double eb = 1.0, ee = 1.0;
        if constexpr (DISP) {
          // z_{b_0} and z_e(B): the b_0 and e rows of L_B^{-1} mu_B (order P, b_0, e)
          double zb[2], ze[2];
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            double v = mi[2 * b0 + r];
#pragma unroll
            for (int k = 0; k < I0; ++k) v = fma(-lb[r][k], gr[GL::gZ + k], v);
            if (r == 1) v = fma(-l10, zb[0], v);
            zb[r] = v * (r ? ib1 : ib0);
          }
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            double v = mi[2 * e + r];
#pragma unroll
            for (int k = 0; k < I0; ++k) v = fma(-gr[GL::gE + r * I0 + k], gr[GL::gZ + k], v);
            v = fma(-le[r][0], zb[0], v);
            v = fma(-le[r][1], zb[1], v);
            if (r == 1) v = fma(-lpx, ze[0], v);
            ze[r] = v * (r ? iep : iex);
          }
          rd[GL::dZ + 0] = zb[0];
          rd[GL::dZ + 1] = zb[1];
          rd[GL::dZ + 2] = ze[0];
          rd[GL::dZ + 3] = ze[1];
          eb = exp(-0.5 * fma(zb[0], zb[0], zb[1] * zb[1]));
          ee = exp(-0.5 * fma(ze[0], ze[0], ze[1] * ze[1]));
        }
        const double pBp = gr[GL::gpP] * ib0 * ib1 * eb;
        rd[GL::dP] = pBp;
        rd[GL::dP + 1] = pBp * iex * iep * ee;
      }
    } else {
      const uint32_t nrec = s_nrec;
      const int ngroups = (int)s_ngroups;
      constexpr int I0 = GL::I0;
      for (uint32_t rix = threadIdx.x - 64; rix < nrec; rix += blockDim.x - 64) {
        int g = 0;
        for (int step = kGroupG / 2; step >= 1; step >>= 1)
          if (g + step < ngroups && s_gbase[g + step] <= rix) g += step;
        const uint32_t a = rix - s_gbase[g];
        int tm[NT];  // modes of T in the order P, e
#pragma unroll
        for (int j = 0; j < NT; ++j) tm[j] = s_gT[g][j];
        const double* gr = grec + g * GL::gN;
        double2* ru = reinterpret_cast<double2*>(rrec) + rix;  // unit q at ru[q * rmax]
        auto rset = [&](int i, double v) {
          reinterpret_cast<double*>(ru + (i >> 1) * rmax)[i & 1] = v;
        };
        // forward substitution of Q_{T,a} through the group's factor; Schur
        // complements at the leading sets give p({a} + U)
        const double2 qd0 = load2_at(Qd, a << 5);
        const double qd2 = load_at(Qd, 4 * a + 2);
        double s00 = qd0.x, s10 = qd0.y, s11 = qd2;
        double pt[NTS];
        bool bad = false;
        // displaced: r = mu_a - y_U^T z_U and |z_U|^2 along the leading sets U
        double r0 = 0.0, r1 = 0.0, qz = 0.0;
        if constexpr (DISP) {
          const double2 m = *reinterpret_cast<const double2*>(mi + 2 * (size_t)a);
          r0 = m.x;
          r1 = m.y;
        }
        // exp(-(|z_U|^2 + r^T S^{-1} r) / 2) with y = det(S)^(-1/2)
        auto mean_factor = [&](double y) -> double {
          if constexpr (!DISP) return 1.0;
          const double t = fma(s11 * r0, r0, fma(-2.0 * s10 * r0, r1, s00 * r1 * r1));
          return exp(-0.5 * fma(t, y * y, qz));
        };
        {
          const double det = fma(s00, s11, -s10 * s10);
          bad |= !(s00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
          const double y = rsqrt_f64(det);
          pt[0] = y * mean_factor(y);
        }
        double y0[I0 > 0 ? I0 : 1], y1[I0 > 0 ? I0 : 1];
        double pl = 1.0;
#pragma unroll
        for (int i = 0; i < I0; ++i) {
          const double2 q = load2_at((i & 1) ? Qodd : Qi, 2u * (uint32_t)tm[i >> 1] * ldq8 + (a << 4));
          double v0 = q.x, v1 = q.y;
#pragma unroll
          for (int k = 0; k < i; ++k) {
            const double l = gr[GL::gP + tri(i, k)];
            v0 = fma(-l, y0[k], v0);
            v1 = fma(-l, y1[k], v1);
          }
          const double di = gr[GL::gP + tri(i, i)];
          y0[i] = v0 * di;
          y1[i] = v1 * di;
          s00 = fma(-y0[i], y0[i], s00);
          s10 = fma(-y0[i], y1[i], s10);
          s11 = fma(-y1[i], y1[i], s11);
          pl *= di;
          if constexpr (DISP) {
            const double z = gr[GL::gZ + i];
            r0 = fma(-y0[i], z, r0);
            r1 = fma(-y1[i], z, r1);
            qz = fma(z, z, qz);
          }
          if (i & 1) {
            const double det = fma(s00, s11, -s10 * s10);
            bad |= !(s00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
            const double y = rsqrt_f64(det);
            pt[(2 << (i >> 1)) - 1] = pl * y * mean_factor(y);
          }
        }
#pragma unroll
        for (int k = 0; k < I0; ++k) ru[(GL::rY / 2 + k) * rmax] = make_double2(y0[k], y1[k]);
        ru[(GL::rS / 2) * rmax] = make_double2(s00, s10);
        rset(GL::rS + 2, s11);
        // e rows: t_e = Q_{e,a} - L_eP y_P, then the e block of Q_T for p({a} + T)
        double te0[2], te1[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const double2 q = load2_at(r ? Qodd : Qi, 2u * (uint32_t)tm[NT - 1] * ldq8 + (a << 4));
          double v0 = q.x, v1 = q.y;
#pragma unroll
          for (int k = 0; k < I0; ++k) {
            const double l = gr[GL::gE + r * I0 + k];
            v0 = fma(-l, y0[k], v0);
            v1 = fma(-l, y1[k], v1);
          }
          te0[r] = v0;
          te1[r] = v1;
          ru[(GL::rT / 2 + r) * rmax] = make_double2(v0, v1);
        }
        {
          const double ex0 = te0[0] * gr[GL::gEd + 0], ex1 = te1[0] * gr[GL::gEd + 0];
          const double ep0 = fma(-gr[GL::gEd + 1], ex0, te0[1]) * gr[GL::gEd + 2];
          const double ep1 = fma(-gr[GL::gEd + 1], ex1, te1[1]) * gr[GL::gEd + 2];
          s00 = fma(-ex0, ex0, s00);
          s10 = fma(-ex0, ex1, s10);
          s11 = fma(-ex1, ex1, s11);
          s00 = fma(-ep0, ep0, s00);
          s10 = fma(-ep0, ep1, s10);
          s11 = fma(-ep1, ep1, s11);
          if constexpr (DISP) {
            // |z_T|^2 is already in p(T); only the a block's share remains
            const double zx = gr[GL::gZ + I0], zp = gr[GL::gZ + I0 + 1];
            r0 = fma(-ex0, zx, fma(-ep0, zp, r0));
            r1 = fma(-ex1, zx, fma(-ep1, zp, r1));
            qz = 0.0;
          }
          const double det = fma(s00, s11, -s10 * s10);
          bad |= !(s00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
          const double y = rsqrt_f64(det);
          pt[NTS - 1] = gr[GL::gpT] * y * mean_factor(y);
        }
        if (bad) {  // {a} + T is an order d-1 subset with a non-positive pivot
          uint32_t rk = a;
#pragma unroll
          for (int j = 0; j < NT; ++j) rk += bin[(j + 2) * ld + tm[j]];
          latch_failure(st, D - 1, (int64_t)rk);
        }
        // the other p({a} + U), U subset of T, from the tables
#pragma unroll
        for (int t = 1; t < NTS; ++t) {
          if (t_leading<NT>(t)) continue;
          uint32_t rk = a;
          int pos = 0;
#pragma unroll
          for (int j = 0; j < NT; ++j)
            if (t & (1 << j)) rk += bin[(pos++ + 2) * ld + tm[j]];
          pt[t] = load_at(tab.p[popcount_c((unsigned)t) + 1], rk);
        }
#pragma unroll
        for (int t = 0; t < NTS; t += 2) ru[((GL::rPT + t) / 2) * rmax] = make_double2(pt[t], pt[t + 1]);
      }
    }
    __syncthreads();

    // ---------------- phase 2: one lane per subset ----------------
    const uint32_t ntile = s_ntile;
    const uint32_t r0 = s_r0;
    const uint64_t lane_mask = lane == 63 ? ~1ull : ((2ull << lane) - 2ull);  // bits 1 .. lane
    for (uint32_t w = wave; (w << 6) < ntile; w += kGroupThreads / 64) {
      const uint32_t p = (w << 6) + lane;
      if (p >= ntile) continue;
      const int c = (int)first[w] + __popcll(bits[w] & lane_mask);
      const double* rd = reinterpret_cast<const double*>(brec + c * GL::bytes);
      const uint32_t* rw = reinterpret_cast<const uint32_t*>(brec + c * GL::bytes + GL::nDpad * 8);
      const uint32_t a = p - rw[GL::wStart];
      const uint32_t r = r0 + p;
      const double2* ru = reinterpret_cast<const double2*>(rrec) + (rw[GL::wRbase] + a);

      // table reads of p({a} + U), b_0 in U, U not B' or B
      double pu[1 << NB];
#pragma unroll
      for (int u = 1; u < FULL; u += 2) {
        if (u == FULLP) continue;
        pu[u] = load_at(tab.p[popcount_c((unsigned)u) + 1], rw[GL::wOP + gop_index<NB>(u)] + p);
      }
      const double2 qb0 = load2_at(Qi, rw[GL::wRow] + (a << 4));
      const double2 qb1 = load2_at(Qodd, rw[GL::wRow] + (a << 4));

      // block rows of b_0 and e of the forward substitution
      constexpr int I0 = 2 * NPm;
      const double2 sPa = ru[(GL::rS / 2) * rmax];
      double s00 = sPa.x, s10 = sPa.y, s11 = ru[(GL::rS / 2 + 1) * rmax].x;
      double yb0[2], yb1[2];
      bool bad = false;
      // displaced: r = mu_a - y^T z over the rows eliminated so far (|z|^2 of
      // B' and B is already in p(B') and p(B))
      double r0 = 0.0, r1 = 0.0;
      if constexpr (DISP) {
        const double* gz = grec + rw[GL::wG] * GL::gN + GL::gZ;
        const double2 m = *reinterpret_cast<const double2*>(mi + 2 * (size_t)a);
        r0 = m.x;
        r1 = m.y;
#pragma unroll
        for (int k = 0; k < I0; ++k) {
          const double2 yk = ru[(GL::rY / 2 + k) * rmax];
          r0 = fma(-yk.x, gz[k], r0);
          r1 = fma(-yk.y, gz[k], r1);
        }
      }
      auto mean_factor = [&](double y) -> double {  // exp(-r^T S^{-1} r / 2), y = det(S)^(-1/2)
        if constexpr (!DISP) return 1.0;
        const double t = fma(s11 * r0, r0, fma(-2.0 * s10 * r0, r1, s00 * r1 * r1));
        return exp(-0.5 * t * (y * y));
      };
#pragma unroll
      for (int rrow = 0; rrow < 2; ++rrow) {
        double v0 = rrow ? qb1.x : qb0.x, v1 = rrow ? qb1.y : qb0.y;
#pragma unroll
        for (int k = 0; k < I0; ++k) {
          const double l = rd[GL::dLb + rrow * I0 + k];
          const double2 yk = ru[(GL::rY / 2 + k) * rmax];
          v0 = fma(-l, yk.x, v0);
          v1 = fma(-l, yk.y, v1);
        }
        if (rrow == 1) {
          const double l = rd[GL::dLb + 2 * I0 + 1];
          v0 = fma(-l, yb0[0], v0);
          v1 = fma(-l, yb1[0], v1);
        }
        const double di = rd[GL::dLb + 2 * I0 + 2 * rrow];
        yb0[rrow] = v0 * di;
        yb1[rrow] = v1 * di;
        s00 = fma(-yb0[rrow], yb0[rrow], s00);
        s10 = fma(-yb0[rrow], yb1[rrow], s10);
        s11 = fma(-yb1[rrow], yb1[rrow], s11);
      }
      double pA, pS;
      if constexpr (DISP) {
#pragma unroll
        for (int rrow = 0; rrow < 2; ++rrow) {
          const double z = rd[GL::dZ + rrow];
          r0 = fma(-yb0[rrow], z, r0);
          r1 = fma(-yb1[rrow], z, r1);
        }
      }
      {
        const double det = fma(s00, s11, -s10 * s10);
        bad |= !(s00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
        const double y = rsqrt_f64(det);
        pA = rd[GL::dP] * y * mean_factor(y);
      }
      double ye0[2], ye1[2];
#pragma unroll
      for (int rrow = 0; rrow < 2; ++rrow) {
        const double2 te = ru[(GL::rT / 2 + rrow) * rmax];
        double v0 = te.x, v1 = te.y;
        v0 = fma(-rd[GL::dLe + 2 * rrow + 0], yb0[0], v0);
        v1 = fma(-rd[GL::dLe + 2 * rrow + 0], yb1[0], v1);
        v0 = fma(-rd[GL::dLe + 2 * rrow + 1], yb0[1], v0);
        v1 = fma(-rd[GL::dLe + 2 * rrow + 1], yb1[1], v1);
        if (rrow == 1) {
          v0 = fma(-rd[GL::dLe + 5], ye0[0], v0);
          v1 = fma(-rd[GL::dLe + 5], ye1[0], v1);
        }
        const double di = rd[GL::dLe + 4 + 2 * rrow];
        ye0[rrow] = v0 * di;
        ye1[rrow] = v1 * di;
        s00 = fma(-ye0[rrow], ye0[rrow], s00);
        s10 = fma(-ye0[rrow], ye1[rrow], s10);
        s11 = fma(-ye1[rrow], ye1[rrow], s11);
      }
      if constexpr (DISP) {
#pragma unroll
        for (int rrow = 0; rrow < 2; ++rrow) {
          const double z = rd[GL::dZ + 2 + rrow];
          r0 = fma(-ye0[rrow], z, r0);
          r1 = fma(-ye1[rrow], z, r1);
        }
      }
      {
        const double det = fma(s00, s11, -s10 * s10);
        bad |= !(s00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
        const double y = rsqrt_f64(det);
        pS = rd[GL::dP + 1] * y * mean_factor(y);
      }
      if (bad) latch_failure(st, D, (int64_t)r);
#pragma unroll
      for (int t = 0; t < NTS; t += 2) {
        const double2 pp = ru[((GL::rPT + t) / 2) * rmax];
        pu[t << 1] = pp.x;
        pu[(t + 1) << 1] = pp.y;
      }
      pu[FULLP] = pA;
      pu[FULL] = pS;

      // nu(W), nu(W + e) for W subset of B' by subset zeta transforms, then
      // m({a} + W) = m(W) - nu(W) (click) or -c(W) + 2 (-1)^|W| nu(W) (parity)
      double nu[NP], nue[NP];
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        const int t = popcount_c((unsigned)u);
        const double sw = (CONV == GBS_CLICK) ? ((t & 1) ? -1.0 : 1.0)
                                              : ((t & 1) ? -1.0 : 1.0) * (double)(1 << t);
        nu[u] = sw * pu[u];
        nue[u] = ((CONV == GBS_CLICK) ? -sw : -2.0 * sw) * pu[u | EBIT];
      }
#pragma unroll
      for (int bit = 0; bit < NB - 1; ++bit)
#pragma unroll
        for (int u = 0; u < NP; ++u)
          if (u & (1 << bit)) {
            nu[u] += nu[u ^ (1 << bit)];
            nue[u] += nue[u ^ (1 << bit)];
          }
      double mwa[NP];
#pragma unroll
      for (int w = 0; w < NP; ++w) {
        const double mw = w ? rd[GL::dMW + w - 1] : 1.0;
        if constexpr (CONV == GBS_CLICK) mwa[w] = mw - nu[w];
        else mwa[w] = fma((popcount_c((unsigned)w) & 1) ? -2.0 : 2.0, nu[w], -mw);
      }
      const double nuB = nu[FULLP] + nue[FULLP];
      const double mB = rd[GL::dMB];
      double mS;
      if constexpr (CONV == GBS_CLICK) mS = mB - nuB;
      else mS = fma((NB & 1) ? -2.0 : 2.0, nuB, -mB);
      if (m_out) store_at(m_out, r, mS);
      if (p_out) store_at(p_out, r, pS);

      if constexpr (WANT_CUM) {
        // K(Y) = k(Y + e) for Y subset of X = {a} + B' (bit 0 of Y = a, bit
        // i + 1 = b_i): B-only ones from LDS, the ones containing a by
        // K(Y) = m(Y + e) - sum_{R proper subset of Y} K(R) m(Y \ R)
        constexpr int NX = 2 * NP;
        double Kv[NX];
#pragma unroll
        for (int R = 0; R < NP; ++R) Kv[2 * R] = rd[GL::dKB + R];
        auto mu_x = [&](int Y) -> double {  // m(Y), Y non-empty subset of X
          return (Y & 1) ? mwa[Y >> 1] : rd[GL::dMW + (Y >> 1) - 1];
        };
#pragma unroll
        for (int Y = 1; Y < NX; Y += 2) {
          const int W = Y >> 1;  // Y = {a} + W
          double v;
          if constexpr (CONV == GBS_CLICK) v = rd[GL::dME + W] - (nu[W] + nue[W]);
          else v = fma((popcount_c((unsigned)W) & 1) ? 2.0 : -2.0, nu[W] + nue[W], -rd[GL::dME + W]);
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

// ---------------- host: tile plans ----------------

namespace {

// Tiles of consecutive B's (colex order of the (d-1)-subsets) such that each
// holds at most kB B's of at most kGroupG groups, which need at most rmax
// (T, a) records.  A group is all B = {b_0} + T with b_0 < min T; within a tile
// it needs the records a < (largest b_0 of the group in the tile).
std::vector<uint64_t> plan_tiles(int M, int NB, int rmax, int kB) {
  std::vector<uint64_t> tiles;
  uint32_t beta = 0, tstart = 0;
  int nB = 0, rec = 0, ng = 0;
  auto close = [&]() {
    if (nB > 0) tiles.push_back((uint64_t)tstart | ((uint64_t)nB << 32));
    tstart = beta;
    nB = 0;
    rec = 0;
    ng = 0;
  };
  // T runs over the (NB-1)-subsets of [0, M) in colex order; its group has min T B's
  const int nt = NB - 1;
  std::vector<int> t(nt);
  for (int i = 0; i < nt; ++i) t[i] = i;
  while (true) {
    const int gsize = t[0];  // b_0 = 0 .. t_0 - 1
    int k = 0;
    while (k < gsize) {
      int n = std::min(gsize - k, kB - nB);
      int need = k + n - 1;  // records a < max b_0 = k + n - 1
      if (rec + need > rmax || ng == kGroupG) {
        close();
        n = std::min(gsize - k, kB);
        need = k + n - 1;
      }
      nB += n;
      rec += need;
      ++ng;
      beta += (uint32_t)n;
      k += n;
      if (nB == kB) close();
    }
    // next T in colex order
    int i = 0;
    while (i < nt && t[i] + 1 == (i + 1 < nt ? t[i + 1] : M)) ++i;
    if (i == nt) break;
    ++t[i];
    for (int j = 0; j < i; ++j) t[j] = j;
  }
  close();
  return tiles;
}

struct PlanKey {
  int device, M, NB, kB;
  bool operator<(const PlanKey& o) const {
    return std::tie(device, M, NB, kB) < std::tie(o.device, o.M, o.NB, o.kB);
  }
};
struct Plan {
  uint64_t* dev = nullptr;
  uint32_t ntiles = 0;
};
std::mutex g_plan_mu;
std::map<PlanKey, Plan> g_plans;

int group_rmax(int M, int NB) { return M - NB <= kGroupRmax ? M - NB : -1; }

hipError_t get_plan(int M, int NB, int kB, Plan* out) {
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_plan_mu);
  auto it = g_plans.find(PlanKey{device, M, NB, kB});
  if (it != g_plans.end()) {
    *out = it->second;
    return hipSuccess;
  }
  const std::vector<uint64_t> tiles = plan_tiles(M, NB, group_rmax(M, NB), kB);
  Plan p;
  p.ntiles = (uint32_t)tiles.size();
  if (!tiles.empty()) {
    e = hipMalloc(&p.dev, tiles.size() * sizeof(uint64_t));
    if (e != hipSuccess) return e;
    e = hipMemcpy(p.dev, tiles.data(), tiles.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p.dev);
      return e;
    }
  }
  g_plans[PlanKey{device, M, NB, kB}] = p;
  *out = p;
  return hipSuccess;
}

template <int NB, bool DISP>
int group_windows(int M) {
  return (GroupLayout<NB, DISP>::kB * (M - NB) + 63) / 64 + 1;
}

template <int NB, bool DISP>
size_t group_lds(int M) {
  using GL = GroupLayout<NB, DISP>;
  const int D = NB + 1;
  return (size_t)GL::kB * GL::bytes + (size_t)kGroupRmax * GL::rbytes +
         (size_t)kGroupG * GL::gbytes +
         (size_t)(((D + 1) * (M + 1) + 1) & ~1) * sizeof(uint32_t) +
         (size_t)group_windows<NB, DISP>(M) * (sizeof(uint64_t) + 1);
}

template <bool DISP>
size_t group_lds_d(int d, int M) {
  switch (d) {
    case 3: return group_lds<2, DISP>(M);
    case 4: return group_lds<3, DISP>(M);
    default: return group_lds<4, DISP>(M);
  }
}

}  // namespace

bool group_supported(int d, int M, int flags, bool displaced) {
  if (d < 3 || d > kMaxOrder || (flags & GBS_MIXED)) return false;
  for (int q = 1; q <= d; ++q)
    if (host_binom(M, q) >= (1ull << 29)) return false;
  if (group_rmax(M, d - 1) < 0) return false;
  const size_t lds = displaced ? group_lds_d<true>(d, M) : group_lds_d<false>(d, M);
  return lds <= 64 * 1024;
}

template <int D, int CONV, bool WC, bool DISP>
static hipError_t launch_group_t(int M, const double* Qi, const double* Qd, const double* mi,
                                 const uint64_t* binom, const OrderTables& tab, double* m_out,
                                 double* k_out, double* p_out, DeviceStatus* st, hipStream_t s) {
  constexpr int NB = D - 1;
  if (host_binom(M, D) == 0) return hipSuccess;
  Plan plan;
  hipError_t e = get_plan(M, NB, GroupLayout<NB, DISP>::kB, &plan);
  if (e != hipSuccess) return e;
  if (plan.ntiles == 0) return hipSuccess;
  const int nwin = group_windows<NB, DISP>(M);
  const size_t lds = group_lds<NB, DISP>(M);
  hipLaunchKernelGGL((forward_group_kernel<D, CONV, WC, DISP>), dim3(plan.ntiles),
                     dim3(kGroupThreads), lds, s, Qi, Qd, mi, M, plan.dev, plan.ntiles, binom, tab,
                     m_out, k_out, p_out, st, nwin);
  return hipGetLastError();
}

template <int D, int CONV, bool DISP>
static hipError_t launch_group_w(int M, const double* Qi, const double* Qd, const double* mi,
                                 const uint64_t* binom, const OrderTables& tab, double* m_out,
                                 double* k_out, double* p_out, DeviceStatus* st, hipStream_t s) {
  if (k_out)
    return launch_group_t<D, CONV, true, DISP>(M, Qi, Qd, mi, binom, tab, m_out, k_out, p_out, st,
                                               s);
  return launch_group_t<D, CONV, false, DISP>(M, Qi, Qd, mi, binom, tab, m_out, k_out, p_out, st,
                                              s);
}

template <int D>
static hipError_t launch_group_c(int M, int flags, const double* Qi, const double* Qd,
                                 const double* mi, const uint64_t* binom, const OrderTables& tab,
                                 double* m_out, double* k_out, double* p_out, DeviceStatus* st,
                                 hipStream_t s) {
  if (flags & GBS_PARITY) {
    if (mi)
      return launch_group_w<D, GBS_PARITY, true>(M, Qi, Qd, mi, binom, tab, m_out, k_out, p_out,
                                                 st, s);
    return launch_group_w<D, GBS_PARITY, false>(M, Qi, Qd, mi, binom, tab, m_out, k_out, p_out,
                                                st, s);
  }
  if (mi)
    return launch_group_w<D, GBS_CLICK, true>(M, Qi, Qd, mi, binom, tab, m_out, k_out, p_out, st,
                                              s);
  return launch_group_w<D, GBS_CLICK, false>(M, Qi, Qd, mi, binom, tab, m_out, k_out, p_out, st, s);
}

hipError_t launch_forward_group(int d, int M, int flags, const double* Qi, const double* Qd,
                                const double* mi, const uint64_t* binom, const OrderTables& tab,
                                double* m_out, double* k_out, double* p_out, DeviceStatus* st,
                                hipStream_t s) {
  switch (d) {
    case 3: return launch_group_c<3>(M, flags, Qi, Qd, mi, binom, tab, m_out, k_out, p_out, st, s);
    case 4: return launch_group_c<4>(M, flags, Qi, Qd, mi, binom, tab, m_out, k_out, p_out, st, s);
    case 5: return launch_group_c<5>(M, flags, Qi, Qd, mi, binom, tab, m_out, k_out, p_out, st, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gbs
