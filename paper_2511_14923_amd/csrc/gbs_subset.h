// Per-subset arithmetic of the one-subset-per-thread kernels (FP64 and mixed),
// shared by the single-instance and the batched launches.
#pragma once

#include "gbs_device.h"

namespace gbs {

// p[MASK | ...] for every subset of the remaining blocks K..D-1, given the
// matrix A over those blocks (Schur complement with respect to the blocks in
// MASK, restriction with respect to the others) and pT = p(MASK).
template <int D, int K, unsigned MASK>
__device__ __forceinline__ void principal_minors(const Tri<2 * (D - K)>& A, double pT,
                                                 double (&p)[1 << D], bool& bad) {
  constexpr int n = 2 * (D - K);
  const double a00 = A.a[0], a10 = A.a[1], a11 = A.a[2];
  const double det = fma(a00, a11, -a10 * a10);
  bad |= !(a00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
  const double y = rsqrt_f64(det);  // det(Q_b | eliminated)^(-1/2)
  if constexpr (n == 2) {
    p[MASK | (1u << K)] = pT * y;
    p[MASK] = pT;
  } else {
    Tri<n - 2> S;
    schur_leading_block<n>(A, y * y, S);
    principal_minors<D, K + 1, MASK | (1u << K)>(S, pT * y, p, bad);
    Tri<n - 2> R;
#pragma unroll
    for (int i = 2; i < n; ++i) {
#pragma unroll
      for (int j = 2; j <= i; ++j) R.a[tri(i - 2, j - 2)] = A.a[tri(i, j)];
    }
    principal_minors<D, K + 1, MASK>(R, pT, p, bad);
  }
}

// Displaced states: as principal_minors, also carrying the mean v over the
// remaining blocks (reduced by every eliminated block, see pivot_mean) and the
// quadratic form qT = mu_MASK^T Q_MASK^{-1} mu_MASK accumulated so far; writes
// det(Q_T)^(-1/2) to p[T] and mu_T^T Q_T^{-1} mu_T to q[T].
template <int D, int K, unsigned MASK>
__device__ __forceinline__ void principal_minors_disp(const Tri<2 * (D - K)>& A,
                                                      const double (&v)[2 * (D - K)], double pT,
                                                      double qT, double (&p)[1 << D],
                                                      double (&q)[1 << D], bool& bad) {
  constexpr int n = 2 * (D - K);
  const double a00 = A.a[0], a10 = A.a[1], a11 = A.a[2];
  const double det = fma(a00, a11, -a10 * a10);
  bad |= !(a00 > 0.0) || !(det > 0.0) || !(det < INFINITY);
  const double y = rsqrt_f64(det);
  double vr[n > 2 ? n - 2 : 1];
  const double qb = pivot_mean<n>(A, y * y, v, vr);
  if constexpr (n == 2) {
    p[MASK | (1u << K)] = pT * y;
    q[MASK | (1u << K)] = qT + qb;
    p[MASK] = pT;
    q[MASK] = qT;
  } else {
    Tri<n - 2> S;
    schur_leading_block<n>(A, y * y, S);
    double vs[n - 2];
#pragma unroll
    for (int i = 0; i < n - 2; ++i) vs[i] = vr[i];
    principal_minors_disp<D, K + 1, MASK | (1u << K)>(S, vs, pT * y, qT + qb, p, q, bad);
    Tri<n - 2> R;
#pragma unroll
    for (int i = 2; i < n; ++i) {
#pragma unroll
      for (int j = 2; j <= i; ++j) R.a[tri(i - 2, j - 2)] = A.a[tri(i, j)];
    }
    double vk[n - 2];
#pragma unroll
    for (int i = 2; i < n; ++i) vk[i - 2] = v[i];
    principal_minors_disp<D, K + 1, MASK>(R, vk, pT, qT, p, q, bad);
  }
}

// m[B] for every B subset S from the vacuum probabilities (subset zeta transform).
template <int D, int CONV>
__device__ __forceinline__ void correlators_from_vacuum(const double (&p)[1 << D],
                                                        double (&m)[1 << D]) {
  constexpr int NS = 1 << D;
#pragma unroll
  for (int T = 0; T < NS; ++T) {
    const int t = popcount_c((unsigned)T);
    if (CONV == GBS_CLICK) {
      m[T] = (t & 1) ? -p[T] : p[T];
    } else {
      m[T] = ((t & 1) ? -1.0 : 1.0) * (double)(1 << t) * p[T];
    }
  }
#pragma unroll
  for (int b = 0; b < D; ++b) {
#pragma unroll
    for (int T = 0; T < NS; ++T) {
      if (T & (1 << b)) m[T] += m[T ^ (1 << b)];
    }
  }
  if (CONV == GBS_PARITY) {
#pragma unroll
    for (int T = 0; T < NS; ++T)
      if (popcount_c((unsigned)T) & 1) m[T] = -m[T];
  }
}

// Cumulant of the full set from all sub-correlators (m[0] = 1).
template <int D>
__device__ __forceinline__ double cumulant_from_correlators(const double (&m)[1 << D]) {
  constexpr unsigned top = 1u << (D - 1);
  constexpr int NR = 1 << (D - 1);
  double k[NR];
#pragma unroll
  for (int B = 0; B < NR; ++B) {
    double v = m[B | top];
#pragma unroll
    for (int R = 0; R < NR; ++R) {
      if (R != B && (R & B) == R) v = fma(-k[R], m[B ^ R], v);
    }
    k[B] = v;
  }
  return k[NR - 1];
}

// Coefficients c(V), V subset of B (NB modes, bit i <-> b_i), of the cumulant of
// {a} + B as a linear form in the vacuum probabilities p({a} + V):
//   k({a} + B) = sum_V c(V) p({a} + V),
// from the B-only correlators m (m[0] = 1).  Eq. cumulant_corr_main with the
// block that contains a singled out reads k({a} + B) = sum_U m({a} + U) g(B \ U),
// where g(Z), the sum over the set partitions rho of Z of
// (-1)^|rho| |rho|! prod m(blocks), is the inverse of m under subset convolution
// (sum_{Y subset Z} m(Y) g(Z \ Y) = 0 for non-empty Z).  With m({a} + U) =
// m(U) - nu(U) (click; parity -m(U) + 2 (-1)^|U| nu(U)) and nu(U) =
// sum_{V subset U} s(V) p({a} + V) (Eq. corre_cov_main), the m(U) terms cancel
// for non-empty B, leaving
//   click:  c(V) = -s(V) G(B \ V),             G(Z) = sum_{W subset Z} g(W),
//   parity: c(V) = 2 s(V) (-1)^|B| G'(B \ V),  G'(Z) = sum_{W subset Z} (-1)^|W| g(W),
// s(V) = (-1)^|V| (click) or (-2)^|V| (parity).
template <int NB, int CONV>
__host__ __device__ __forceinline__ void cumulant_coefficients(const double (&m)[1 << NB],
                                                               double (&c)[1 << NB]) {
  constexpr int NU = 1 << NB;
  constexpr int FULL = NU - 1;
  double g[NU];
  g[0] = 1.0;
#pragma unroll
  for (int z = 1; z < NU; ++z) {
    double acc = 0.0;
#pragma unroll
    for (int y = 1; y <= z; ++y)
      if ((y & z) == y) acc = fma(m[y], g[z ^ y], acc);
    g[z] = -acc;
  }
  if constexpr (CONV != GBS_CLICK) {
#pragma unroll
    for (int w = 0; w < NU; ++w)
      if (popcount_c((unsigned)w) & 1) g[w] = -g[w];
  }
#pragma unroll
  for (int bit = 0; bit < NB; ++bit)
#pragma unroll
    for (int w = 0; w < NU; ++w)
      if (w & (1 << bit)) g[w] += g[w ^ (1 << bit)];
#pragma unroll
  for (int v = 0; v < NU; ++v) {
    const int cv = popcount_c((unsigned)v);
    const double coef = (CONV == GBS_CLICK) ? ((cv & 1) ? 1.0 : -1.0)
                                            : (((cv + NB) & 1) ? -2.0 : 2.0) * (double)(1 << cv);
    c[v] = coef * g[FULL ^ v];
  }
}

// The sign s(V) of a vacuum probability p({a} + V) in nu (Eq. corre_cov_main):
// (-1)^|V| for click, (-2)^|V| for parity.
template <int CONV>
__host__ __device__ constexpr double vacuum_sign(int v) {
  return (CONV == GBS_CLICK) ? ((popcount_c((unsigned)v) & 1) ? -1.0 : 1.0)
                             : ((popcount_c((unsigned)v) & 1) ? -1.0 : 1.0) *
                                   (double)(1 << popcount_c((unsigned)v));
}

// Correlator, cumulant and vacuum probability of the subset s[0] < ... < s[D-1].
template <int D, int CONV, bool WANT_CUM>
__device__ __forceinline__ void subset_fp64(const double* __restrict__ Qi, int M, const int (&s)[D],
                                            double& corr, double& cum, double& pS, bool& bad) {
  Tri<2 * D> A;
  gather_q<D>(Qi, M, s, A);
  double p[1 << D];
  principal_minors<D, 0, 0u>(A, 1.0, p, bad);
  pS = p[(1 << D) - 1];
  double m[1 << D];
  correlators_from_vacuum<D, CONV>(p, m);
  corr = m[(1 << D) - 1];
  if constexpr (WANT_CUM) cum = cumulant_from_correlators<D>(m);
  else cum = 0.0;
}

// Displaced states (first moments in mi, interleaved): every vacuum
// probability gains exp(-mu_T^T Q_T^{-1} mu_T / 2) (Eq. vacuum_gaussian_prob).
template <int D, int CONV, bool WANT_CUM>
__device__ __forceinline__ void subset_fp64_disp(const double* __restrict__ Qi,
                                                 const double* __restrict__ mi, int M,
                                                 const int (&s)[D], double& corr, double& cum,
                                                 double& pS, bool& bad) {
  Tri<2 * D> A;
  gather_q<D>(Qi, M, s, A);
  double v[2 * D];
  gather_mean<D>(mi, s, v);
  double p[1 << D], q[1 << D];
  principal_minors_disp<D, 0, 0u>(A, v, 1.0, 0.0, p, q, bad);
#pragma unroll
  for (int T = 1; T < (1 << D); ++T) p[T] *= exp(-0.5 * q[T]);
  pS = p[(1 << D) - 1];
  double m[1 << D];
  correlators_from_vacuum<D, CONV>(p, m);
  corr = m[(1 << D) - 1];
  if constexpr (WANT_CUM) cum = cumulant_from_correlators<D>(m);
  else cum = 0.0;
}

struct Neumaier {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
  }
  __device__ __forceinline__ double value() const { return s + c; }
};

template <int D, int K, unsigned MASK>
__device__ __forceinline__ void minors_mixed(const TriF<2 * (D - K)>& F, float rho,
                                             float (&rhoT)[1 << D], bool& bad) {
  constexpr int n = 2 * (D - K);
  const float f00 = F.a[0], f10 = F.a[1], f11 = F.a[2];
  const float delta = f00 + f11 + fmaf(f00, f11, -f10 * f10);
  const float onep = 1.0f + delta;
  bad |= !(onep > 0.0f) || !(1.0f + f00 > 0.0f) || !(onep < INFINITY);
  const float y = __builtin_amdgcn_rsqf(onep);
  const float inv = y * y;
  const float eta = -delta * inv * __builtin_amdgcn_rcpf(1.0f + y);
  const float rho_c = rho + fmaf(rho, eta, eta);
  if constexpr (n == 2) {
    rhoT[MASK | (1u << K)] = rho_c;
    rhoT[MASK] = rho;
  } else {
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
    for (int i = 2; i < n; ++i) {
#pragma unroll
      for (int j = 2; j <= i; ++j)
        S.a[tri(i - 2, j - 2)] =
            fmaf(-F.a[tri(i, 1)], u1[j], fmaf(-F.a[tri(i, 0)], u0[j], F.a[tri(i, j)]));
    }
    minors_mixed<D, K + 1, MASK | (1u << K)>(S, rho_c, rhoT, bad);
    TriF<n - 2> R;
#pragma unroll
    for (int i = 2; i < n; ++i) {
#pragma unroll
      for (int j = 2; j <= i; ++j) R.a[tri(i - 2, j - 2)] = F.a[tri(i, j)];
    }
    minors_mixed<D, K + 1, MASK>(R, rho, rhoT, bad);
  }
}

// Mixed precision: FP32 deviation-form minors of the normalised Q, FP64 assembly.
// pS is the full set's vacuum probability P_S (1 + rho_S).
template <int D, int CONV, bool WANT_CUM>
__device__ __forceinline__ void subset_mixed(const double* __restrict__ pk, const float* __restrict__ E,
                                             int M, const int (&s)[D], double& corr, double& cum,
                                             double& pS, bool& bad) {
  constexpr int NS = 1 << D;
  double p1[D];
#pragma unroll
  for (int i = 0; i < D; ++i) p1[i] = pk[s[i]];

  float rhoT[NS];
  if constexpr (D == 1) {
    rhoT[0] = 0.0f;
    rhoT[1] = 0.0f;
  } else {
    TriF<2 * D> F;
    const size_t lde = 2 * (size_t)M;
#pragma unroll
    for (int i = 0; i < D; ++i) {
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
    minors_mixed<D, 0, 0u>(F, 0.0f, rhoT, bad);
  }

  // FP64 assembly.  P_T by subset products; corrections c_T = P_T rho_T.
  double P[NS];
  P[0] = 1.0;
#pragma unroll
  for (int T = 1; T < NS; ++T) {
    const int low = __builtin_ctz((unsigned)T);
    P[T] = P[T & (T - 1)] * p1[low];
  }
  pS = fma(P[NS - 1], (double)rhoT[NS - 1], P[NS - 1]);
  double g[NS];
#pragma unroll
  for (int T = 0; T < NS; ++T) {
    const int t = popcount_c((unsigned)T);
    const double c = P[T] * (double)rhoT[T];
    g[T] = (CONV == GBS_CLICK) ? ((t & 1) ? -c : c) : ((t & 1) ? -1.0 : 1.0) * (double)(1 << t) * c;
  }
  // zeta transform of the corrections for every proper subset; the full set's
  // correlator is accumulated term by term with compensation
  Neumaier top;
#pragma unroll
  for (int T = 0; T < NS; ++T) top.add(g[T]);
#pragma unroll
  for (int b = 0; b < D; ++b) {
#pragma unroll
    for (int T = 0; T < NS; ++T)
      if (T & (1 << b)) g[T] += g[T ^ (1 << b)];
  }
  // product parts
  double base[NS];
  base[0] = 1.0;
#pragma unroll
  for (int T = 1; T < NS; ++T) {
    const int low = __builtin_ctz((unsigned)T);
    const double f = (CONV == GBS_CLICK) ? (1.0 - p1[low]) : (2.0 * p1[low] - 1.0);
    base[T] = base[T & (T - 1)] * f;
  }
  double m[NS];
#pragma unroll
  for (int T = 0; T < NS; ++T) {
    const double corrT = (CONV == GBS_CLICK || !(popcount_c((unsigned)T) & 1)) ? g[T] : -g[T];
    m[T] = base[T] + corrT;
  }
  {
    const double corrS = (CONV == GBS_CLICK || !(D & 1)) ? top.value() : -top.value();
    Neumaier full;
    full.add(base[NS - 1]);
    full.add(corrS);
    m[NS - 1] = full.value();
  }
  corr = m[NS - 1];
  if constexpr (WANT_CUM) {
    constexpr unsigned topbit = 1u << (D - 1);
    constexpr int NR = 1 << (D - 1);
    double k[NR];
#pragma unroll
    for (int B = 0; B < NR; ++B) {
      if (B == NR - 1) {
        Neumaier acc;
        acc.add(m[B | topbit]);
#pragma unroll
        for (int R = 0; R < NR; ++R)
          if (R != B && (R & B) == R) acc.add(-k[R] * m[B ^ R]);
        k[B] = acc.value();
      } else {
        double v = m[B | topbit];
#pragma unroll
        for (int R = 0; R < NR; ++R)
          if (R != B && (R & B) == R) v = fma(-k[R], m[B ^ R], v);
        k[B] = v;
      }
    }
    cum = k[NR - 1];
  }
  if constexpr (!WANT_CUM) cum = 0.0;
}

}  // namespace gbs
