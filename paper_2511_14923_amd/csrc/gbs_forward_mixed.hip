// Mixed-precision all-minors kernel: FP32 determinant work, FP64 sums.  It
// runs for GBS_MIXED | GBS_ALL_MINORS (evaluating all 2^d minors of every
// subset, no lower-order tables); the default mixed path is the group kernel
// (gbs_forward_group.hip) with the same normalisation and deviation form in
// its shared factors and plain FP64 sums, and the order-recursive kernel's
// mixed branch for orders 1 and 2.
//
// Normalisation (per mode, FP64): Q_kk = L_k L_k^T (2x2 Cholesky), the
// single-mode vacuum probability p_k = det(Q_kk)^(-1/2), and the normalised
// couplings E_kl = L_k^{-1} Q_kl L_l^{-T} (k != l, stored FP32; E_kk = 0).  Then
//     det Q_T = prod_{k in T} det Q_kk * det(I + E_T)
// so that p(T) = P_T (1 + rho_T) with P_T = prod_{k in T} p_k (FP64, exact
// product) and rho_T = det(I + E_T)^(-1/2) - 1, a small deviation computed in
// FP32 with relative accuracy: the principal-minor recursion runs on the
// deviation F = A - I of every Schur complement, each 2x2 pivot contributes
// delta = det(I + F_00) - 1 = tr F_00 + det F_00 and
//     (1 + delta)^(-1/2) - 1 = -delta y^2 / (1 + y),  y = (1 + delta)^(-1/2),
// and deviations compose as rho' = rho + eta + rho eta.  No step subtracts
// two numbers close to one in FP32.
//
// FP64 assembly: the inclusion-exclusion splits into the product part,
// which has no cancellation at all,
//     sum_{T subset B} (-1)^|T| P_T = prod_{k in B} (1 - p_k)       (click),
//     (-1)^|B| sum_{T subset B} (-2)^|T| P_T = prod_{k in B} (2 p_k - 1)  (parity),
// plus the zeta transform of the signed corrections P_T rho_T.  The correlator
// and the cumulant of S (the two stored values) are accumulated with Neumaier
// compensation; sub-correlators used inside the cumulant recursion are plain
// FP64 sums, whose rounding is nine orders below the FP32 input error.
#include <hip/hip_runtime.h>

#include "gbs_internal.h"
#include "gbs_subset.h"

namespace gbs {

template <int D, int CONV, bool WRITE_CORR, bool WRITE_CUM, bool LDS_BIN>
__global__ __launch_bounds__(256) void forward_mixed_kernel(const double* __restrict__ pk,
                                                            const float* __restrict__ E, int M,
                                                            uint64_t count,
                                                            const uint64_t* __restrict__ binom,
                                                            double* __restrict__ corr,
                                                            double* __restrict__ cum,
                                                            DeviceStatus* __restrict__ st) {
  extern __shared__ uint64_t sbin[];
  const uint64_t* bin;
  int ld;
  if constexpr (LDS_BIN) {
    ld = M + 1;
    for (int i = threadIdx.x; i < (D + 1) * ld; i += blockDim.x) {
      const int k = i / ld, nn = i - k * ld;
      sbin[i] = binom[k * kBinLd + nn];
    }
    __syncthreads();
    bin = sbin;
  } else {
    ld = kBinLd;
    bin = binom;
  }
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < count; r += stride) {

  int s[D];
  colex_unrank<D>(r, M, bin, ld, s);

  double mS, kS, pS;
  bool bad = false;
  subset_mixed<D, CONV, WRITE_CUM>(pk, E, M, s, mS, kS, pS, bad);
  if (bad) latch_failure(st, D, (int64_t)r);
  if constexpr (WRITE_CORR) corr[r] = mS;
  if constexpr (WRITE_CUM) cum[r] = kS;
  }
}

// Per-mode 2x2 Cholesky factors, p_k, and E_kl = L_k^{-1} Q_kl L_l^{-T}.
__global__ void build_normalised_kernel(const double* __restrict__ Qi, int M,
                                        double* __restrict__ pk, float* __restrict__ E) {
  const size_t ldq = 2 * (size_t)M;
  const size_t total = (size_t)M * M;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / M), l = (int)(idx - (size_t)k * M);
    // L_k = [[a, 0], [b, c]]
    const double* qk = Qi + (size_t)(2 * k) * ldq + 2 * k;
    const double ak = sqrt(qk[0]);
    const double bk = qk[ldq] / ak;
    const double ck = sqrt(qk[ldq + 1] - bk * bk);
    if (l == k) {
      pk[k] = 1.0 / (ak * ck);
      E[(size_t)(2 * k) * ldq + 2 * k] = 0.0f;
      E[(size_t)(2 * k) * ldq + 2 * k + 1] = 0.0f;
      E[(size_t)(2 * k + 1) * ldq + 2 * k] = 0.0f;
      E[(size_t)(2 * k + 1) * ldq + 2 * k + 1] = 0.0f;
      continue;
    }
    const double* ql = Qi + (size_t)(2 * l) * ldq + 2 * l;
    const double al = sqrt(ql[0]);
    const double bl = ql[ldq] / al;
    const double cl = sqrt(ql[ldq + 1] - bl * bl);
    const double* q = Qi + (size_t)(2 * k) * ldq + 2 * l;
    const double q00 = q[0], q01 = q[1], q10 = q[ldq], q11 = q[ldq + 1];
    // X = L_k^{-1} Q_kl: forward substitution on the rows
    const double x00 = q00 / ak, x01 = q01 / ak;
    const double x10 = (q10 - bk * x00) / ck, x11 = (q11 - bk * x01) / ck;
    // E = X L_l^{-T}: forward substitution on the columns
    const double e00 = x00 / al, e10 = x10 / al;
    const double e01 = (x01 - bl * e00) / cl, e11 = (x11 - bl * e10) / cl;
    float* e = E + (size_t)(2 * k) * ldq + 2 * l;
    e[0] = (float)e00;
    e[1] = (float)e01;
    e[ldq] = (float)e10;
    e[ldq + 1] = (float)e11;
  }
}

hipError_t launch_build_normalised(const double* Qi, int M, double* pk, float* E, hipStream_t s) {
  const size_t total = (size_t)M * M;
  const int block = 256;
  const int grid = (int)((total + block - 1) / block < 4096 ? (total + block - 1) / block : 4096);
  hipLaunchKernelGGL(build_normalised_kernel, dim3(grid), dim3(block), 0, s, Qi, M, pk, E);
  return hipGetLastError();
}

template <int D, int CONV, bool WC, bool WK>
static hipError_t launch_mixed_t(int M, const double* pk, const float* E, const uint64_t* binom,
                                 double* corr, double* cum, DeviceStatus* st, hipStream_t s) {
  const uint64_t count = host_binom(M, D);
  if (count == 0) return hipSuccess;
  const int block = 256;
  const uint64_t grid = std::min<uint64_t>((count + block - 1) / block, kMaxGrid);
  const size_t lds = (size_t)(D + 1) * (M + 1) * sizeof(uint64_t);
  if (lds <= 48 * 1024) {
    hipLaunchKernelGGL((forward_mixed_kernel<D, CONV, WC, WK, true>), dim3((unsigned)grid),
                       dim3(block), lds, s, pk, E, M, count, binom, corr, cum, st);
  } else {
    hipLaunchKernelGGL((forward_mixed_kernel<D, CONV, WC, WK, false>), dim3((unsigned)grid),
                       dim3(block), 0, s, pk, E, M, count, binom, corr, cum, st);
  }
  return hipGetLastError();
}

template <int D, int CONV>
static hipError_t launch_mixed_w(int M, const double* pk, const float* E, const uint64_t* binom,
                                 double* corr, double* cum, DeviceStatus* st, hipStream_t s) {
  if (corr && cum) return launch_mixed_t<D, CONV, true, true>(M, pk, E, binom, corr, cum, st, s);
  if (corr) return launch_mixed_t<D, CONV, true, false>(M, pk, E, binom, corr, cum, st, s);
  return launch_mixed_t<D, CONV, false, true>(M, pk, E, binom, corr, cum, st, s);
}

template <int D>
static hipError_t launch_mixed_c(int M, int flags, const double* pk, const float* E,
                                 const uint64_t* binom, double* corr, double* cum,
                                 DeviceStatus* st, hipStream_t s) {
  if (flags & GBS_PARITY) return launch_mixed_w<D, GBS_PARITY>(M, pk, E, binom, corr, cum, st, s);
  return launch_mixed_w<D, GBS_CLICK>(M, pk, E, binom, corr, cum, st, s);
}

hipError_t launch_forward_mixed(int d, int M, int flags, const double* pk, const float* E,
                                const uint64_t* binom, double* corr, double* cum,
                                DeviceStatus* st, hipStream_t s) {
  switch (d) {
    case 1: return launch_mixed_c<1>(M, flags, pk, E, binom, corr, cum, st, s);
    case 2: return launch_mixed_c<2>(M, flags, pk, E, binom, corr, cum, st, s);
    case 3: return launch_mixed_c<3>(M, flags, pk, E, binom, corr, cum, st, s);
    case 4: return launch_mixed_c<4>(M, flags, pk, E, binom, corr, cum, st, s);
    case 5: return launch_mixed_c<5>(M, flags, pk, E, binom, corr, cum, st, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gbs
