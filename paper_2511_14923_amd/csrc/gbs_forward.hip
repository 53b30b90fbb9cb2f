// Forward kernels: vacuum probabilities -> correlators -> cumulants, one subset
// per thread.
//
// For a subset S = {s_0 < ... < s_{d-1}} the thread
//   1. unranks its colex rank into S;
//   2. gathers Q_S, the 2d x 2d principal block of Q = sigma + I/2 (App. D.1: the
//      reduced state keeps the rows/columns of the retained modes), from the
//      interleaved copy of Q so that each mode is one 2x2 block;
//   3. evaluates p(T) = det(Q_T)^(-1/2) for all 2^d subsets T of S at once with the
//      principal-minor recursion on 2x2 blocks: for the leading block b,
//        minors of T without b  = minors of Q_S with b's rows/columns deleted,
//        minors of T with b     = det(Q_b) * minors of the Schur complement Q_S / Q_b,
//      which reaches each of the 2^d - 1 non-empty T with one 2x2 pivot and one
//      reciprocal square root (p(T) = det(Q_T)^(-1/2), Eq. vacuum_gaussian_prob);
//   4. forms every sub-correlator of S by the subset zeta transform of the signed
//      p(T): click mu(B) = sum_{T subset B} (-1)^|T| p(T) (App. A.2), parity
//      c(B) = (-1)^|B| sum_{T subset B} (-2)^|T| p(T) (Eq. corre_cov_main);
//   5. forms the cumulant of S by the fixed-element recursion
//        k(B) = m(B) - sum_{R proper subset of B\{n}} k(R + {n}) m(B \ {n} \ R)
//      over the subsets B that contain the largest element n (App. B, Eq.
//      correlators_expanded_2; equivalent to the partition sum of Eq.
//      cumulant_corr_main / joint_cumulants_def);
//   6. stores the correlator and the cumulant of S at its colex rank.
// For a displaced state (first moments mu) the recursion also carries the mean
// reduced by the eliminated blocks, and every p(T) gains
// exp(-mu_T^T Q_T^{-1} mu_T / 2) (Eq. vacuum_gaussian_prob).
#include <hip/hip_runtime.h>

#include "gbs_internal.h"
#include "gbs_subset.h"

namespace gbs {

template <int D, int CONV, bool WRITE_CORR, bool WRITE_CUM, bool LDS_BIN, bool DISP>
__global__ __launch_bounds__(256) void forward_fp64_kernel(const double* __restrict__ Qi,
                                                           const double* __restrict__ mi, int M,
                                                           uint64_t rank0, uint64_t count,
                                                           const uint64_t* __restrict__ binom,
                                                           double* __restrict__ corr,
                                                           double* __restrict__ cum,
                                                           double* __restrict__ ptab,
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
  colex_unrank<D>(rank0 + r, M, bin, ld, s);
  double mS, kS, pS;
  bool bad = false;
  if constexpr (DISP) subset_fp64_disp<D, CONV, WRITE_CUM>(Qi, mi, M, s, mS, kS, pS, bad);
  else subset_fp64<D, CONV, WRITE_CUM>(Qi, M, s, mS, kS, pS, bad);
  if (bad) latch_failure(st, D, (int64_t)(rank0 + r));
  if (ptab) ptab[r] = pS;
  if constexpr (WRITE_CORR) corr[r] = mS;
  if constexpr (WRITE_CUM) cum[r] = kS;
  }
}

// ----------------------------------------------------------------------------

__global__ void build_q_kernel(const double* __restrict__ sigma, int M, double* __restrict__ Qi) {
  const int n = 2 * M;
  const size_t total = (size_t)n * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(idx / n), col = (int)(idx - (size_t)row * n);
    // interleaved index 2k + a  <->  xxpp index k + a M
    const int sr = (row >> 1) + (row & 1) * M;
    const int sc = (col >> 1) + (col & 1) * M;
    const double v = (sr >= sc) ? sigma[(size_t)sr * n + sc] : sigma[(size_t)sc * n + sr];
    Qi[idx] = v + (row == col ? 0.5 : 0.0);
  }
}

// Per-mode diagonal blocks of Q (x-x, p-x, p-p, 0) for coalesced access by mode.
__global__ void build_qdiag_kernel(const double* __restrict__ Qi, int M, double* __restrict__ Qd) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const size_t ldq = 2 * (size_t)M;
  const double* q = Qi + (size_t)(2 * k) * ldq + 2 * k;
  Qd[4 * (size_t)k + 0] = q[0];
  Qd[4 * (size_t)k + 1] = q[ldq];
  Qd[4 * (size_t)k + 2] = q[ldq + 1];
  Qd[4 * (size_t)k + 3] = 0.0;
}

hipError_t launch_build_qdiag(const double* Qi, int M, double* Qd, hipStream_t s) {
  hipLaunchKernelGGL(build_qdiag_kernel, dim3((M + 255) / 256), dim3(256), 0, s, Qi, M, Qd);
  return hipGetLastError();
}

__global__ void clear_status_kernel(DeviceStatus* st) {
  st->flag = 0;
  st->order = 0;
  st->rank = -1;
}

hipError_t launch_build_q(const double* sigma, int M, double* Qi, hipStream_t s) {
  const size_t total = 4 * (size_t)M * M;
  const int block = 256;
  const int grid = (int)((total + block - 1) / block < 4096 ? (total + block - 1) / block : 4096);
  hipLaunchKernelGGL(build_q_kernel, dim3(grid), dim3(block), 0, s, sigma, M, Qi);
  return hipGetLastError();
}

// First moments in interleaved order: mi[2k] = mu[k] (x_k), mi[2k+1] = mu[k+M] (p_k).
__global__ void build_mean_kernel(const double* __restrict__ mu, int M, double* __restrict__ mi) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  mi[2 * (size_t)k] = mu[k];
  mi[2 * (size_t)k + 1] = mu[(size_t)k + M];
}

hipError_t launch_build_mean(const double* mu, int M, double* mi, hipStream_t s) {
  hipLaunchKernelGGL(build_mean_kernel, dim3((M + 255) / 256), dim3(256), 0, s, mu, M, mi);
  return hipGetLastError();
}

hipError_t launch_clear_status(DeviceStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

template <int D, int CONV, bool WC, bool WK, bool DISP>
static hipError_t launch_fp64_t(int M, const double* Qi, const double* mi, const uint64_t* binom,
                                double* corr, double* cum, double* ptab, DeviceStatus* st,
                                hipStream_t s, uint64_t rank0 = 0, uint64_t count = ~0ull) {
  if (count == ~0ull) count = host_binom(M, D);
  if (count == 0) return hipSuccess;
  const int block = 256;
  const uint64_t grid = std::min<uint64_t>((count + block - 1) / block, kMaxGrid);
  const size_t lds = (size_t)(D + 1) * (M + 1) * sizeof(uint64_t);
  if (lds <= 48 * 1024) {
    hipLaunchKernelGGL((forward_fp64_kernel<D, CONV, WC, WK, true, DISP>), dim3((unsigned)grid),
                       dim3(block), lds, s, Qi, mi, M, rank0, count, binom, corr, cum, ptab, st);
  } else {
    hipLaunchKernelGGL((forward_fp64_kernel<D, CONV, WC, WK, false, DISP>), dim3((unsigned)grid),
                       dim3(block), 0, s, Qi, mi, M, rank0, count, binom, corr, cum, ptab, st);
  }
  return hipGetLastError();
}

template <int D, int CONV, bool DISP>
static hipError_t launch_fp64_w(int M, const double* Qi, const double* mi, const uint64_t* binom,
                                double* corr, double* cum, double* ptab, DeviceStatus* st,
                                hipStream_t s) {
  if (corr && cum)
    return launch_fp64_t<D, CONV, true, true, DISP>(M, Qi, mi, binom, corr, cum, ptab, st, s);
  if (corr)
    return launch_fp64_t<D, CONV, true, false, DISP>(M, Qi, mi, binom, corr, cum, ptab, st, s);
  return launch_fp64_t<D, CONV, false, true, DISP>(M, Qi, mi, binom, corr, cum, ptab, st, s);
}

template <int D>
static hipError_t launch_fp64_c(int M, int flags, const double* Qi, const double* mi,
                                const uint64_t* binom, double* corr, double* cum, double* ptab,
                                DeviceStatus* st, hipStream_t s) {
  if (mi) {
    if (flags & GBS_PARITY)
      return launch_fp64_w<D, GBS_PARITY, true>(M, Qi, mi, binom, corr, cum, ptab, st, s);
    return launch_fp64_w<D, GBS_CLICK, true>(M, Qi, mi, binom, corr, cum, ptab, st, s);
  }
  if (flags & GBS_PARITY)
    return launch_fp64_w<D, GBS_PARITY, false>(M, Qi, mi, binom, corr, cum, ptab, st, s);
  return launch_fp64_w<D, GBS_CLICK, false>(M, Qi, mi, binom, corr, cum, ptab, st, s);
}

hipError_t launch_forward_mixed(int d, int M, int flags, const double* pk, const float* E,
                                const uint64_t* binom, double* corr, double* cum,
                                DeviceStatus* st, hipStream_t s);

hipError_t launch_forward(int d, int M, int flags, const double* Qi, const double* mi,
                          const double* pk, const float* E, const uint64_t* binom, double* corr,
                          double* cum, double* ptab, DeviceStatus* st, hipStream_t s) {
  if (!corr && !cum) return hipSuccess;
  if (flags & GBS_MIXED) {
    if (mi) return hipErrorInvalidValue;
    return launch_forward_mixed(d, M, flags, pk, E, binom, corr, cum, st, s);
  }
  switch (d) {
    case 1: return launch_fp64_c<1>(M, flags, Qi, mi, binom, corr, cum, ptab, st, s);
    case 2: return launch_fp64_c<2>(M, flags, Qi, mi, binom, corr, cum, ptab, st, s);
    case 3: return launch_fp64_c<3>(M, flags, Qi, mi, binom, corr, cum, ptab, st, s);
    case 4: return launch_fp64_c<4>(M, flags, Qi, mi, binom, corr, cum, ptab, st, s);
    case 5: return launch_fp64_c<5>(M, flags, Qi, mi, binom, corr, cum, ptab, st, s);
    default: return hipErrorInvalidValue;
  }
}

// One order's outputs for the colex ranks rank0 .. rank0 + count - 1 by the
// tree kernel (no lower-order tables: every rank range is independent).
template <int D>
static hipError_t launch_range_d(int M, int flags, const double* Qi, const uint64_t* binom,
                                 uint64_t rank0, uint64_t count, double* corr, double* cum,
                                 DeviceStatus* st, hipStream_t s) {
  const bool par = (flags & GBS_PARITY) != 0;
  if (corr && cum)
    return par ? launch_fp64_t<D, GBS_PARITY, true, true, false>(M, Qi, nullptr, binom, corr, cum, nullptr, st, s, rank0, count)
               : launch_fp64_t<D, GBS_CLICK, true, true, false>(M, Qi, nullptr, binom, corr, cum, nullptr, st, s, rank0, count);
  if (corr)
    return par ? launch_fp64_t<D, GBS_PARITY, true, false, false>(M, Qi, nullptr, binom, corr, cum, nullptr, st, s, rank0, count)
               : launch_fp64_t<D, GBS_CLICK, true, false, false>(M, Qi, nullptr, binom, corr, cum, nullptr, st, s, rank0, count);
  return par ? launch_fp64_t<D, GBS_PARITY, false, true, false>(M, Qi, nullptr, binom, corr, cum, nullptr, st, s, rank0, count)
             : launch_fp64_t<D, GBS_CLICK, false, true, false>(M, Qi, nullptr, binom, corr, cum, nullptr, st, s, rank0, count);
}

hipError_t launch_forward_range(int d, int M, int flags, const double* Qi, const uint64_t* binom,
                                uint64_t rank0, uint64_t count, double* corr, double* cum,
                                DeviceStatus* st, hipStream_t s) {
  if (count == 0 || (!corr && !cum)) return hipSuccess;
  switch (d) {
    case 1: return launch_range_d<1>(M, flags, Qi, binom, rank0, count, corr, cum, st, s);
    case 2: return launch_range_d<2>(M, flags, Qi, binom, rank0, count, corr, cum, st, s);
    case 3: return launch_range_d<3>(M, flags, Qi, binom, rank0, count, corr, cum, st, s);
    case 4: return launch_range_d<4>(M, flags, Qi, binom, rank0, count, corr, cum, st, s);
    case 5: return launch_range_d<5>(M, flags, Qi, binom, rank0, count, corr, cum, st, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gbs
