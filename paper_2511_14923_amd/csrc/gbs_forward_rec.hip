// Order-recursive forward kernel: one new determinant per subset, everything
// else read from the tables of the lower orders.
//
// Orders run in sequence (1, 2, ..., K); order d reads the vacuum
// probabilities p, correlators m and cumulants k that orders 1..d-1 stored.
// For a subset S = {a} + B with a its smallest mode, e its largest, d its
// second largest and B' = B \ {e}, the thread
//   1. reads p({a} + U) for the subsets U of B that the factorisation below
//      does not give, m(W) for the subsets W of B, and k(Y + {e}) for the
//      subsets Y of B' (all issued first, so that the factorisation hides
//      their latency);
//   2. factors Q_S in block order [B' \ {d}, a, d, e] (2x2 pivots, one
//      reciprocal square root each; p(T) = det(Q_T)^(-1/2), App. D.1, Eq.
//      vacuum_gaussian_prob): its leading minors give p(S \ {d, e}),
//      p(S \ {e}) and p(S), and the e block of the Schur complement taken after
//      S \ {d, e} gives p(S \ {d}) with one more 2x2 determinant (the mixed
//      form factors the normalised FP32 deviation in order [B', a, e]);
//   3. forms nu(W) = sum_{U subset W} s_|U| p({a} + U) for every W subset of B by a
//      subset zeta transform (s_t = (-1)^t click, (-2)^t parity), then
//        click   mu(W + a) = mu(W) - nu(W)
//        parity  c(W + a)  = -c(W) + 2 (-1)^|W| nu(W)
//      (both split the inclusion-exclusion of App. D.1 / Eq. corre_cov_main
//      into the terms without and with mode a; m(empty) = 1);
//   4. forms the cumulants k(Y + {e}) of the subsets Y of {a} + B' that contain
//      a, in increasing order, by the fixed-element recursion on e
//        k(Y + {e}) = m(Y + {e}) - sum_{R proper subset of Y} k(R + {e}) m(Y \ R)
//      (the partition sum of Eq. cumulant_corr_main grouped by the block that
//      contains e; App. B, Eq. correlators_expanded_2); Y = {a} + B' gives k(S);
//   5. stores m(S), k(S) and, below the last order, p(S).
// For a displaced state (first moments mu) the factorisation also carries the
// mean reduced by the eliminated blocks: each pivot adds its share of
// mu_T^T Q_T^{-1} mu_T (pivot_mean), and the four probabilities of step 2 gain
// exp(-mu_T^T Q_T^{-1} mu_T / 2) (Eq. vacuum_gaussian_prob); the tables of the
// lower orders already hold displaced values, so steps 3-5 are unchanged.
// Every output thus costs one 2d x 2d factorisation plus O(2^d) additions --
// the work count of the method's cost model.  A capped grid of workgroups
// strides over the ranks, so each workgroup fills its LDS binomial table once.
#include <hip/hip_runtime.h>

#include "gbs_internal.h"

namespace gbs {

// Workgroups of a launch; each strides over many subsets.  Order 5 (the
// mixed form at M = 144, 4.8e8 subsets) runs faster on the larger grid
// (16.3 -> 15.7 ms), order 4 on the smaller one (0.30 against 0.32 ms).
constexpr uint64_t kRecGrid = 4096;
constexpr uint64_t kRecGridTop = 65536;  // orders 5 and above

// Quadratic-form shares of a displaced state, accumulated beside the
// determinant products of the chains below (unused, and removed by the
// compiler, for a zero-mean state).
struct MeanForms {
  double de = 0.0, d = 0.0, a = 0.0, s = 0.0;  // mu_T^T Q_T^{-1} mu_T for the four T
};

// Leading-block elimination chain for the block order [.., a, d, e]: multiplies
// P by det(pivot)^(-1/2) for each block; pDE receives the product before d
// (p(S \ {d, e})), pD the product times the e block of the Schur complement
// at that point (p(S \ {d})), pA the product before e (p(S \ {e})), pS the
// full product.  With DISP, v is the mean over A's rows, q the quadratic form
// of the blocks eliminated so far, and qf receives the same four quantities
// for mu_T^T Q_T^{-1} mu_T.
template <int n, bool DISP>
__device__ __forceinline__ void chain2(const Tri<n>& A, const double (&v)[n], double P, double q,
                                       double& pDE, double& pD, double& pA, double& pS,
                                       MeanForms& qf, bool& bad) {
  if constexpr (n == 4) {
    pDE = P;
    // e block of the 4x4 Schur complement
    const double e00 = A.a[tri(2, 2)], e10 = A.a[tri(3, 2)], e11 = A.a[tri(3, 3)];
    const double dete = fma(e00, e11, -e10 * e10);
    bad |= !(dete > 0.0);
    const double ye = rsqrt_f64(dete);
    pD = P * ye;
    if constexpr (DISP) {
      qf.de = q;
      // v_e^T E^{-1} v_e with E^{-1} = adj(E) / det(E)
      const double t = fma(e11 * v[2], v[2], fma(-2.0 * e10 * v[2], v[3], e00 * v[3] * v[3]));
      qf.d = fma(t, ye * ye, q);
    }
  }
  const double a00 = A.a[0], a10 = A.a[1], a11 = A.a[2];
  const double det = fma(a00, a11, -a10 * a10);
  bad |= !(a00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
  const double y = rsqrt_f64(det);
  const double Pn = P * y;
  double vr[n > 2 ? n - 2 : 1];
  double qn = q;
  if constexpr (DISP) qn += pivot_mean<n>(A, y * y, v, vr);
  if constexpr (n == 2) {
    pS = Pn;
    if constexpr (DISP) qf.s = qn;
  } else {
    if constexpr (n == 4) {
      pA = Pn;
      if constexpr (DISP) qf.a = qn;
    }
    Tri<n - 2> S;
    schur_leading_block<n>(A, y * y, S);
    double vs[n - 2];
#pragma unroll
    for (int i = 0; i < n - 2; ++i) vs[i] = DISP ? vr[i] : 0.0;
    chain2<n - 2, DISP>(S, vs, Pn, qn, pDE, pD, pA, pS, qf, bad);
  }
}

// The same for the block order [.., a, e]: pA = p(S \ {e}), pS = p(S).
template <int n, int NB, bool DISP>
__device__ __forceinline__ void chain(const Tri<n>& A, const double (&v)[n], double P, double q,
                                      double& pA, double& pS, MeanForms& qf, bool& bad) {
  const double a00 = A.a[0], a10 = A.a[1], a11 = A.a[2];
  const double det = fma(a00, a11, -a10 * a10);
  bad |= !(a00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
  const double y = rsqrt_f64(det);
  const double Pn = P * y;
  double vr[n > 2 ? n - 2 : 1];
  double qn = q;
  if constexpr (DISP) qn += pivot_mean<n>(A, y * y, v, vr);
  if constexpr (n == 2) {
    pS = Pn;
    if constexpr (DISP) qf.s = qn;
  } else {
    if constexpr (n == 4) {
      pA = Pn;
      if constexpr (DISP) qf.a = qn;
    }
    Tri<n - 2> S;
    schur_leading_block<n>(A, y * y, S);
    double vs[n - 2];
#pragma unroll
    for (int i = 0; i < n - 2; ++i) vs[i] = DISP ? vr[i] : 0.0;
    chain<n - 2, NB, DISP>(S, vs, Pn, qn, pA, pS, qf, bad);
  }
}

// FP32 chain on the deviation F = A - I of the normalised matrix (unit
// diagonal blocks): every pivot contributes delta = det(I + F00) - 1 and the
// factor (1 + delta)^(-1/2) = 1 + eta with eta = -delta y^2 / (1 + y); the
// deviations compose as rho' = rho + eta + rho eta.  rhoA is the deviation
// after all but the last block, rhoS after all blocks.
template <int n>
__device__ __forceinline__ void chain_dev(const TriF<n>& F, float rho, float& rhoA, float& rhoS,
                                          bool& bad) {
  const float f00 = F.a[0], f10 = F.a[1], f11 = F.a[2];
  const float delta = f00 + f11 + fmaf(f00, f11, -f10 * f10);
  const float onep = 1.0f + delta;
  bad |= !(onep > 0.0f) || !(1.0f + f00 > 0.0f) || !(onep < INFINITY);
  const float y = __builtin_amdgcn_rsqf(onep);
  const float inv = y * y;
  const float eta = -delta * inv * __builtin_amdgcn_rcpf(1.0f + y);
  const float rn = rho + fmaf(rho, eta, eta);
  if constexpr (n == 2) {
    rhoS = rn;
  } else {
    if constexpr (n == 4) rhoA = rn;
    const float g00 = 1.0f + f00, g11 = 1.0f + f11;
    float u0[n], u1[n];
#pragma unroll
    for (int i = 2; i < n; ++i) {
      const float c0 = F.a[tri(i, 0)], c1 = F.a[tri(i, 1)];
      u0[i] = fmaf(g11, c0, -f10 * c1) * inv;
      u1[i] = fmaf(g00, c1, -f10 * c0) * inv;
    }
    TriF<n - 2> S;
#pragma unroll
    for (int i = 2; i < n; ++i)
#pragma unroll
      for (int j = 2; j <= i; ++j)
        S.a[tri(i - 2, j - 2)] =
            fmaf(-F.a[tri(i, 1)], u1[j], fmaf(-F.a[tri(i, 0)], u0[j], F.a[tri(i, j)]));
    chain_dev<n - 2>(S, rn, rhoA, rhoS, bad);
  }
}

template <int D, int CONV, bool WANT_CUM, bool LDS_BIN, typename Idx, bool MIXED, bool DISP>
__global__ __launch_bounds__(256) void forward_rec_kernel(const double* __restrict__ Qi,
                                                          const double* __restrict__ Qd,
                                                          const double* __restrict__ mi,
                                                          const double* __restrict__ pk,
                                                          const float* __restrict__ E, int M,
                                                          uint64_t count,
                                                          const uint64_t* __restrict__ binom,
                                                          OrderTables tab,
                                                          double* __restrict__ m_out,
                                                          double* __restrict__ k_out,
                                                          double* __restrict__ p_out,
                                                          DeviceStatus* __restrict__ st) {
  static_assert(D >= 2 && D <= kMaxOrder, "orders 2..5");
  static_assert(!(MIXED && DISP), "displaced states are FP64 only");
  constexpr int NB = D - 1;          // |B|
  constexpr int NU = 1 << NB;        // subsets of B
  constexpr int FULL = NU - 1;       // B
  constexpr int FULLP = (1 << (NB - 1)) - 1;  // B' = B \ {e}
  // binomial table C(n, k), k <= D, n <= M: in LDS (as Idx) when it fits
  extern __shared__ uint64_t sbin_raw[];
  const Idx* bin;
  const uint64_t* gbin = binom;
  int ld;
  if constexpr (LDS_BIN) {
    Idx* sb = reinterpret_cast<Idx*>(sbin_raw);
    ld = M + 1;
    for (int i = threadIdx.x; i < (D + 1) * ld; i += blockDim.x) {
      const int kk = i / ld, nn = i - kk * ld;
      sb[i] = (Idx)binom[kk * kBinLd + nn];
    }
    __syncthreads();
    bin = sb;
  } else {
    ld = kBinLd;
    bin = nullptr;
  }
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < count; r += stride) {
    int s[D];
    if constexpr (LDS_BIN) colex_unrank_est<D>(r, M, bin, ld, s);
    else colex_unrank_est<D>(r, M, gbin, ld, s);
    const int a = s[0], e = s[D - 1];
    constexpr bool PDROP = D >= 3 && !MIXED;
    // binomials C(s_i, k) for the rank arithmetic, read where they are used (a
    // per-thread array of them would live in scratch memory)
    auto cb = [&](int i, int kk) -> Idx {
      return LDS_BIN ? (Idx)bin[kk * ld + s[i]] : (Idx)gbin[kk * ld + s[i]];
    };
    constexpr int UDROP_D = (D >= 3) ? (FULL ^ (1 << (D - 3))) : -1;           // B minus d
    constexpr int UDROP_DE = (D >= 3) ? (FULL ^ (1 << (D - 3)) ^ (1 << (D - 2))) : -1;  // B minus d, e
    double pu[NU];
    double mw[NU];
    auto load_lookups = [&]() {
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        if (u == FULL || u == FULLP) continue;
        if (PDROP && (u == UDROP_D || u == UDROP_DE)) continue;
        Idx rk = (Idx)a;
        int j = 0;
#pragma unroll
        for (int i = 0; i < NB; ++i)
          if (u & (1 << i)) rk += cb(i + 1, (j++) + 2);
        pu[u] = load_at(tab.p[popcount_c((unsigned)u) + 1], rk);
      }
      mw[0] = 1.0;
#pragma unroll
      for (int w = 1; w < NU; ++w) {
        Idx rk = 0;
        int j = 0;
#pragma unroll
        for (int i = 0; i < NB; ++i)
          if (w & (1 << i)) rk += cb(i + 1, (j++) + 1);
        mw[w] = load_at(tab.m[popcount_c((unsigned)w)], rk);
      }
    };
    load_lookups();  // issued before the factorisation, which hides their latency

    double pA = 1.0, pS = 1.0;
    bool bad = false;
    if constexpr (MIXED) {
      int ch[D];
#pragma unroll
      for (int i = 0; i < D - 2; ++i) ch[i] = s[i + 1];
      ch[D - 2] = a;
      ch[D - 1] = e;
      TriF<2 * D> F;
      gather_e_coalesced<D, D - 2>(E, M, ch, F);
      float rhoA = 0.0f, rhoS = 0.0f;
      chain_dev<2 * D>(F, 0.0f, rhoA, rhoS, bad);
      double PA = pk[a];
#pragma unroll
      for (int i = 1; i < D - 1; ++i) PA *= pk[s[i]];
      const double PS = PA * pk[e];
      pA = fma(PA, (double)rhoA, PA);
      pS = fma(PS, (double)rhoS, PS);
    } else if constexpr (PDROP) {
      int ch[D];
#pragma unroll
      for (int i = 0; i < D - 3; ++i) ch[i] = s[i + 1];
      ch[D - 3] = a;
      ch[D - 2] = s[D - 2];
      ch[D - 1] = e;
      Tri<2 * D> A;
      gather_q_coalesced<D, D - 3>(Qi, Qd, M, ch, A);
      double v[2 * D] = {};
      if constexpr (DISP) gather_mean<D>(mi, ch, v);
      double pDE = 1.0, pD = 1.0;
      MeanForms qf;
      chain2<2 * D, DISP>(A, v, 1.0, 0.0, pDE, pD, pA, pS, qf, bad);
      if constexpr (DISP) {
        pDE *= exp(-0.5 * qf.de);
        pD *= exp(-0.5 * qf.d);
        pA *= exp(-0.5 * qf.a);
        pS *= exp(-0.5 * qf.s);
      }
      if constexpr (UDROP_D >= 0) {
        pu[UDROP_D] = pD;
        pu[UDROP_DE] = pDE;
      }
    } else {
      int ch[D];
#pragma unroll
      for (int i = 0; i < D - 2; ++i) ch[i] = s[i + 1];
      ch[D - 2] = a;
      ch[D - 1] = e;
      Tri<2 * D> A;
      gather_q_coalesced<D, D - 2>(Qi, Qd, M, ch, A);
      double v[2 * D] = {};
      if constexpr (DISP) gather_mean<D>(mi, ch, v);
      MeanForms qf;
      chain<2 * D, D, DISP>(A, v, 1.0, 0.0, pA, pS, qf, bad);
      if constexpr (DISP) {
        pA *= exp(-0.5 * qf.a);
        pS *= exp(-0.5 * qf.s);
      }
    }
    if (bad) latch_failure(st, D, (int64_t)r);
    pu[FULL] = pS;
    pu[FULLP] = pA;

    // 3. nu(W) by the zeta transform, then m(W + a)
    double nu[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int t = popcount_c((unsigned)u);
      if (CONV == GBS_CLICK) nu[u] = (t & 1) ? -pu[u] : pu[u];
      else nu[u] = ((t & 1) ? -1.0 : 1.0) * (double)(1 << t) * pu[u];
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int u = 0; u < NU; ++u)
        if (u & (1 << b)) nu[u] += nu[u ^ (1 << b)];
    double ma[NU];
#pragma unroll
    for (int w = 0; w < NU; ++w) {
      if (CONV == GBS_CLICK) ma[w] = mw[w] - nu[w];
      else ma[w] = fma((popcount_c((unsigned)w) & 1) ? -2.0 : 2.0, nu[w], -mw[w]);
    }
    const double mS = ma[FULL];
    const Idx ri = (Idx)r;
    if (m_out) store_at(m_out, ri, mS);
    if (p_out) store_at(p_out, ri, pS);

    if constexpr (WANT_CUM) {
      constexpr int NX = 1 << (D - 1);
      constexpr int FULLX = NX - 1;
      constexpr int EBIT = 1 << (D - 2);  // e as a B bit
      // K(Y) = k(Y + {e}) for Y subset of X = {a} + B' (X bit 0 <-> a, bit i <-> s[i])
      double Kv[NX];
#pragma unroll
      for (int Y = 0; Y < NX; ++Y) {
        const bool has_a = Y & 1;
        if (!has_a) {
          if (Y == FULLX) continue;
          Idx rk = 0;
          int j = 0;
#pragma unroll
          for (int i = 0; i < D - 1; ++i)
            if (Y & (1 << i)) rk += cb(i, (j++) + 1);
          rk += cb(D - 1, j + 1);
          Kv[Y] = load_at(tab.k[j + 1], rk);
        }
      }
      auto mu_of = [&](int Y) -> double {  // m(Y), Y subset of X
        return (Y & 1) ? ma[Y >> 1] : mw[Y >> 1];
      };
      auto mu_e = [&](int Y) -> double {   // m(Y + {e})
        const int W = (Y >> 1) | EBIT;
        return (Y & 1) ? ma[W] : mw[W];
      };
      double kS = 0.0;
#pragma unroll
      for (int Y = 1; Y < NX; Y += 2) {  // Y contains a
        double v = mu_e(Y);
        double c = 0.0;
#pragma unroll
        for (int R = 0; R < Y; ++R) {
          if ((R & Y) != R) continue;
          if constexpr (MIXED) {
            const double term = -Kv[R] * mu_of(Y ^ R);
            const double t = v + term;
            c += (fabs(v) >= fabs(term)) ? ((v - t) + term) : ((term - t) + v);
            v = t;
          } else {
            v = fma(-Kv[R], mu_of(Y ^ R), v);
          }
        }
        Kv[Y] = v + c;
        if (Y == FULLX) kS = v + c;
      }
      store_at(k_out, ri, kS);
    }
  }
}

// Order 1: p({a}) = det(Q_aa)^(-1/2) (times exp(-v^T Q_aa^{-1} v / 2) for a
// displaced state with mean v on mode a), mu = 1 - p (click) or c = 2p - 1
// (parity), and the cumulant of a single mode is its correlator.
template <int CONV, bool DISP>
__global__ void forward_order1_kernel(const double* __restrict__ Qi, const double* __restrict__ mi,
                                      int M, double* __restrict__ m_out,
                                      double* __restrict__ k_out, double* __restrict__ p_out,
                                      DeviceStatus* __restrict__ st) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= M) return;
  const size_t ldq = 2 * (size_t)M;
  const double* q = Qi + (size_t)(2 * a) * ldq + 2 * a;
  const double a00 = q[0], a10 = q[ldq], a11 = q[ldq + 1];
  const double det = fma(a00, a11, -a10 * a10);
  if (!(a00 > 0.0) || !(det > 0.0) || !(det < INFINITY)) latch_failure(st, 1, a);
  const double y = rsqrt_f64(det);
  double p = y;
  if constexpr (DISP) {
    const double v0 = mi[2 * (size_t)a], v1 = mi[2 * (size_t)a + 1];
    const double t = fma(a11 * v0, v0, fma(-2.0 * a10 * v0, v1, a00 * v1 * v1));
    p *= exp(-0.5 * t * (y * y));
  }
  const double m = (CONV == GBS_CLICK) ? 1.0 - p : fma(2.0, p, -1.0);
  if (m_out) m_out[a] = m;
  if (k_out) k_out[a] = m;
  if (p_out) p_out[a] = p;
}

template <int D, int CONV, bool WC, typename Idx, bool MX, bool DP>
static hipError_t launch_rec_t(int M, const double* Qi, const double* Qd, const double* mi,
                               const double* pk, const float* E,
                               const uint64_t* binom, const OrderTables& tab, double* m_out,
                               double* k_out, double* p_out, DeviceStatus* st, hipStream_t s) {
  const uint64_t count = host_binom(M, D);
  if (count == 0) return hipSuccess;
  const int block = 256;
  const uint64_t grid =
      std::min<uint64_t>((count + block - 1) / block, D >= 5 ? kRecGridTop : kRecGrid);
  const size_t lds = (size_t)(D + 1) * (M + 1) * sizeof(Idx);
  if (lds <= 48 * 1024) {
    hipLaunchKernelGGL((forward_rec_kernel<D, CONV, WC, true, Idx, MX, DP>), dim3((unsigned)grid),
                       dim3(block), lds, s, Qi, Qd, mi, pk, E, M, count, binom, tab, m_out, k_out,
                       p_out, st);
  } else {
    hipLaunchKernelGGL((forward_rec_kernel<D, CONV, WC, false, Idx, MX, DP>), dim3((unsigned)grid),
                       dim3(block), 0, s, Qi, Qd, mi, pk, E, M, count, binom, tab, m_out, k_out,
                       p_out, st);
  }
  return hipGetLastError();
}

template <int D, int CONV, bool MX, bool DP>
static hipError_t launch_rec_w(int M, const double* Qi, const double* Qd, const double* mi,
                               const double* pk, const float* E,
                               const uint64_t* binom, const OrderTables& tab, double* m_out,
                               double* k_out, double* p_out, DeviceStatus* st, hipStream_t s) {
  // 32-bit rank and byte-offset arithmetic when every table of orders <= D
  // has fewer than 2^29 entries
  bool small = true;
  for (int d = 1; d <= D; ++d) small = small && host_binom(M, d) < (1ull << 29);
  if (k_out) {
    if (small)
      return launch_rec_t<D, CONV, true, uint32_t, MX, DP>(M, Qi, Qd, mi, pk, E, binom, tab, m_out,
                                                           k_out, p_out, st, s);
    return launch_rec_t<D, CONV, true, uint64_t, MX, DP>(M, Qi, Qd, mi, pk, E, binom, tab, m_out,
                                                         k_out, p_out, st, s);
  }
  if (small)
    return launch_rec_t<D, CONV, false, uint32_t, MX, DP>(M, Qi, Qd, mi, pk, E, binom, tab, m_out,
                                                          k_out, p_out, st, s);
  return launch_rec_t<D, CONV, false, uint64_t, MX, DP>(M, Qi, Qd, mi, pk, E, binom, tab, m_out,
                                                        k_out, p_out, st, s);
}

template <int D, int CONV>
static hipError_t launch_rec_v(int M, int flags, const double* Qi, const double* Qd,
                               const double* mi, const double* pk, const float* E,
                               const uint64_t* binom, const OrderTables& tab, double* m_out,
                               double* k_out, double* p_out, DeviceStatus* st, hipStream_t s) {
  if (flags & GBS_MIXED)
    return launch_rec_w<D, CONV, true, false>(M, Qi, Qd, mi, pk, E, binom, tab, m_out, k_out, p_out,
                                              st, s);
  if (mi)
    return launch_rec_w<D, CONV, false, true>(M, Qi, Qd, mi, pk, E, binom, tab, m_out, k_out, p_out,
                                              st, s);
  return launch_rec_w<D, CONV, false, false>(M, Qi, Qd, mi, pk, E, binom, tab, m_out, k_out, p_out,
                                             st, s);
}

template <int D>
static hipError_t launch_rec_c(int M, int flags, const double* Qi, const double* Qd,
                               const double* mi, const double* pk, const float* E,
                               const uint64_t* binom, const OrderTables& tab, double* m_out,
                               double* k_out, double* p_out, DeviceStatus* st, hipStream_t s) {
  if (flags & GBS_PARITY)
    return launch_rec_v<D, GBS_PARITY>(M, flags, Qi, Qd, mi, pk, E, binom, tab, m_out, k_out,
                                       p_out, st, s);
  return launch_rec_v<D, GBS_CLICK>(M, flags, Qi, Qd, mi, pk, E, binom, tab, m_out, k_out, p_out,
                                    st, s);
}

hipError_t launch_forward_rec(int d, int M, int flags, const double* Qi, const double* Qd,
                              const double* mi, const double* pk,
                              const float* E, const uint64_t* binom, const double* const* p_tab,
                              const double* const* m_tab, const double* const* k_tab,
                              double* m_out, double* k_out, double* p_out, DeviceStatus* st,
                              hipStream_t s, const GroupPlanRef* plans) {
  if (mi && (flags & GBS_MIXED)) return hipErrorInvalidValue;
  OrderTables tab{};
  for (int q = 1; q <= kMaxOrder; ++q) {
    tab.p[q] = p_tab[q];
    tab.m[q] = m_tab[q];
    tab.k[q] = k_tab[q];
  }
  if (d == 1) {
    const int block = 256;
    const int grid = (M + block - 1) / block;
    if (flags & GBS_PARITY) {
      if (mi)
        hipLaunchKernelGGL((forward_order1_kernel<GBS_PARITY, true>), dim3(grid), dim3(block), 0, s,
                           Qi, mi, M, m_out, k_out, p_out, st);
      else
        hipLaunchKernelGGL((forward_order1_kernel<GBS_PARITY, false>), dim3(grid), dim3(block), 0,
                           s, Qi, mi, M, m_out, k_out, p_out, st);
    } else {
      if (mi)
        hipLaunchKernelGGL((forward_order1_kernel<GBS_CLICK, true>), dim3(grid), dim3(block), 0, s,
                           Qi, mi, M, m_out, k_out, p_out, st);
      else
        hipLaunchKernelGGL((forward_order1_kernel<GBS_CLICK, false>), dim3(grid), dim3(block), 0, s,
                           Qi, mi, M, m_out, k_out, p_out, st);
    }
    return hipGetLastError();
  }
  // the tile kernel takes zero-mean states only
  if (group_supported(d, M, flags, mi != nullptr))
    return launch_forward_group(d, M, flags, Qi, Qd, mi, pk, E, binom, tab, m_out, k_out, p_out, st,
                                s, (plans && !mi) ? &plans[d] : nullptr);
  if (!mi && tile_supported(d, M, flags))
    return launch_forward_tile(d, M, flags, Qi, Qd, binom, tab, m_out, k_out, p_out, st, s);
  switch (d) {
    case 2: return launch_rec_c<2>(M, flags, Qi, Qd, mi, pk, E, binom, tab, m_out, k_out, p_out, st, s);
    case 3: return launch_rec_c<3>(M, flags, Qi, Qd, mi, pk, E, binom, tab, m_out, k_out, p_out, st, s);
    case 4: return launch_rec_c<4>(M, flags, Qi, Qd, mi, pk, E, binom, tab, m_out, k_out, p_out, st, s);
    case 5: return launch_rec_c<5>(M, flags, Qi, Qd, mi, pk, E, binom, tab, m_out, k_out, p_out, st, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gbs
