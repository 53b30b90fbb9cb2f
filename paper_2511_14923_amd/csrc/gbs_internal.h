// Internal host-side interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "gbs_device.h"

namespace gbs {

// Binomial table C(n, k), k = 0..kMaxOrder+1, n = 0..GBS_MAX_MODES, laid out
// [k][n] with leading dimension kBinLd.
constexpr int kBinLd = GBS_MAX_MODES + 1;
constexpr int kBinRows = kMaxOrder + 2;

uint64_t host_binom(int n, int k);

// Per-device state created once per device and kept until the process ends.
struct DeviceContext {
  int device = -1;
  uint64_t* binom = nullptr;  // device copy of the binomial table
  int cu_count = 0;
};

// Context of the current device (created on first use); nullptr on failure.
DeviceContext* current_context(hipError_t* err);

// Q = sigma + I/2 in interleaved (x_0 p_0 x_1 p_1 ...) order, full symmetric
// 2M x 2M FP64, built from sigma's lower triangle.
hipError_t launch_build_q(const double* sigma, int M, double* Qi, hipStream_t s);

// First moments in interleaved order (mi[2k] = mu[k], mi[2k+1] = mu[k+M]).
hipError_t launch_build_mean(const double* mu, int M, double* mi, hipStream_t s);

// Per-mode diagonal blocks of Q, 4 doubles per mode (x-x, p-x, p-p, 0).
hipError_t launch_build_qdiag(const double* Qi, int M, double* Qd, hipStream_t s);

// Mixed-precision operands: per-mode block Cholesky factors of Q, the
// single-mode vacuum probabilities pk (FP64) and the normalised off-diagonal
// blocks E = L_k^{-1} Q_kl L_l^{-T} (FP32, interleaved 2M x 2M, zero diagonal blocks).
hipError_t launch_build_normalised(const double* Qi, int M, double* pk, float* E, hipStream_t s);

// Optional per-launch event timing (GBS_TIMING), per calling thread.
void timing_start_call(bool enabled);
hipError_t timing_begin(hipStream_t s, int stage, int order);
hipError_t timing_end(hipStream_t s);

// Status of a call: HIP error mapping, and the end of a call (copy the device
// status word back; synchronise and report unless GBS_ASYNC).
gbs_status to_status(hipError_t e);
gbs_status finish_status(DeviceStatus* dev_status, int32_t flags, hipStream_t s);
// The same without the pinned host slot (the allocation-free entry point): the
// status word is read back by a blocking copy, or by gbs_last_error after an
// asynchronous call.
gbs_status finish_status_device(const DeviceStatus* dev_status, int32_t flags, hipStream_t s);
// Argument check shared by the forward entry points (M, max_order, flag bits).
bool valid_problem(int32_t M, int32_t K, int32_t flags);

// Reset a status word (fill kernel, safe inside graph capture).
hipError_t launch_clear_status(DeviceStatus* st, hipStream_t s);

// Order-d forward pass over all C(M, d) subsets.
// FP64 reads Qi (and the interleaved first moments mi of a displaced state,
// or null for zero mean); MIXED reads pk and E (zero mean only).  corr and/or
// cum may be null (not written); ptab (FP64 only, may be null) receives p(S)
// of every subset.
hipError_t launch_forward(int d, int M, int flags, const double* Qi, const double* mi,
                          const double* pk, const float* E, const uint64_t* binom, double* corr,
                          double* cum, double* ptab, DeviceStatus* st, hipStream_t s);

// Order-d outputs for the colex ranks rank0 .. rank0 + count - 1 only (FP64
// tree kernel, no lower-order tables); corr / cum hold `count` values.
hipError_t launch_forward_range(int d, int M, int flags, const double* Qi, const uint64_t* binom,
                                uint64_t rank0, uint64_t count, double* corr, double* cum,
                                DeviceStatus* st, hipStream_t s);

// The same for orders 3..5 by the T-shared kernel (gbs_forward_shard.hip): the
// subsets {a, b_0} + T of one T share the factors of Q_T, of each b_0 and of
// each a against T.  The range runs as consecutive chunks of at most 2^16 T's.
hipError_t launch_forward_shard(int d, int M, int flags, const double* Qi, uint64_t rank0,
                                uint64_t count, double* corr, double* cum, DeviceStatus* st,
                                hipStream_t s);

// Lower-order tables read by the order-recursive kernels: p[q], m[q], k[q]
// point at the order-q blocks (q below the order being computed).
struct OrderTables {
  const double* p[kMaxOrder + 1];  // vacuum probabilities
  const double* m[kMaxOrder + 1];  // correlators
  const double* k[kMaxOrder + 1];  // cumulants
};

// Tiled FP64 kernel of order d (3..5) when every table of orders <= d has
// fewer than 2^29 entries (32-bit rank arithmetic); see gbs_forward_tile.hip.
bool tile_supported(int d, int M, int flags);
hipError_t launch_forward_tile(int d, int M, int flags, const double* Qi, const double* Qd,
                               const uint64_t* binom, const OrderTables& tab, double* m_out,
                               double* k_out, double* p_out, DeviceStatus* st, hipStream_t s);

// Group-tiled kernel of order d (3..5), FP64 or mixed, the default where it applies:
// 32-bit ranks and LDS for (M - d + 1) records per tile; see
// gbs_forward_group.hip.  Tile plans are built on the host once per (M, d,
// tile width) and kept on the device until the process ends.  mi: interleaved
// first moments of a displaced state, or null.
bool group_supported(int d, int M, int flags, bool displaced);
// A tile plan already on the device (caller-placed): ntiles descriptors at dev,
// launched on `grid` workgroups.  Passed to launch_forward_group to bypass the
// library's own cached plans (which it allocates once per (M, d)).
struct GroupPlanRef {
  const uint64_t* dev = nullptr;
  uint32_t ntiles = 0;
  uint32_t grid = 0;
};
// Host copy of the zero-mean tile plan of order d for M modes (built once,
// kept until the process ends) and the grid a single-instance launch uses
// on a device with cu_count compute units.
const std::vector<uint64_t>& group_plan_host(int d, int M, bool mixed);
uint32_t group_plan_grid(uint32_t ntiles, int cu_count);
hipError_t launch_forward_group(int d, int M, int flags, const double* Qi, const double* Qd,
                                const double* mi, const double* pk, const float* E,
                                const uint64_t* binom, const OrderTables& tab, double* m_out,
                                double* k_out, double* p_out, DeviceStatus* st, hipStream_t s,
                                const GroupPlanRef* plan = nullptr);

// The group kernel over many zero-mean instances: one persistent launch per
// order claims (instance, tile) items from a device work list.  Instance i of
// order d reads its lower-order tables through tab and writes the order-d
// blocks m_out (may be null), k_out and p_out (may be null).
struct GroupBatchInstance {
  const double* Qi;
  const double* Qd;
  const double* pk;  // mixed form: single-mode vacuum probabilities
  const float* E;    // mixed form: FP32 normalised couplings
  OrderTables tab;
  double* m_out;
  double* k_out;
  double* p_out;
  int M;
  int pad;
};
struct GroupBatchItem {
  uint32_t inst;
  uint32_t pad;
  uint64_t desc;  // tile descriptor of the instance's plan
};
// Tile descriptors of order d for M modes, appended to out (host).
void group_tiles(int d, int M, bool mixed, std::vector<uint64_t>* out);
// LDS bytes and bitmap windows of a batched launch of order d (FP64 or, with
// GBS_MIXED, the mixed form) whose largest M is max_M.
size_t group_batched_lds(int d, int flags, int max_M, int* nwin_max);
// Workgroups that fit on the device at once for that LDS size (before capture).
hipError_t group_batched_grid(int d, int flags, size_t lds, int cu_count, int* grid);
hipError_t launch_group_batched(int d, int flags, const GroupBatchInstance* inst,
                                const GroupBatchItem* items, uint32_t n_items, unsigned* counter,
                                int grid, int max_M, int nwin_max, size_t lds,
                                const uint64_t* binom, DeviceStatus* st, hipStream_t s);

// Order-recursive FP64 forward pass of order d (see gbs_forward_rec.hip):
// p_tab/m_tab/k_tab[q] point at the order-q blocks of the lower-order tables
// (q < d); m_out, k_out, p_out at the order-d blocks (each may be null).
// GBS_MIXED reads pk and E (normalised Q) instead of Qi.  mi (interleaved first
// moments, FP64 only) selects the displaced-state kernels; null for zero mean.
// plans (may be null): plans[d] is the device tile plan the group kernel of
// order d uses instead of the library's cached one (zero-mean states only).
hipError_t launch_forward_rec(int d, int M, int flags, const double* Qi, const double* Qd,
                              const double* mi, const double* pk,
                              const float* E, const uint64_t* binom, const double* const* p_tab,
                              const double* const* m_tab, const double* const* k_tab,
                              double* m_out, double* k_out, double* p_out, DeviceStatus* st,
                              hipStream_t s, const GroupPlanRef* plans = nullptr);

// Vector-Jacobian product given the forward correlators m and vacuum
// probabilities ptab of every subset (orders 1..K); d1, mbar, pbar are scratch
// of N(M, K) doubles, part scratch of kAdjointPartDoubles doubles (the partial
// sums of superset sums split over several workgroups); gsig (2M x 2M, xxpp)
// is overwritten.
constexpr int kAdjointSplitItems = 2048;  // a launch of fewer sums splits each one
constexpr int kAdjointMaxSplit = 16;
constexpr size_t kAdjointPartDoubles = 4 * 2 * (size_t)kAdjointSplitItems;
hipError_t launch_adjoint(int M, int K, int flags, const double* Qi, const uint64_t* binom,
                          const double* m, const double* ptab, const double* gm, const double* gk,
                          double* d1, double* mbar, double* pbar, double* gsig, DeviceStatus* st,
                          double* part, hipStream_t s);

// Stage-2 sampler (gbs_sampler.hip): nsamples patterns of M bits from the
// parity cumulants kap (orders 1..K, K = 3 or 5), uniforms u (M x nsamples),
// in launches of at most `batch` samples (0: a quarter of the free memory).
hipError_t run_sampler(int M, int K, const double* kap, int64_t nsamples, const double* u,
                       uint8_t* bits, double* prob, double* cond, int64_t batch, hipStream_t s);

// Sample statistics (gbs_estimator.hip): unbiased click cumulants of orders
// 1..K from N samples (bits N x M), written in the output layout; Pearson
// coefficient of two device arrays of length n, written to r (device).
hipError_t run_sample_cumulants(int M, int64_t N, const uint8_t* bits, int K,
                                const uint64_t* binom, double* out, hipStream_t s);
hipError_t run_pearson(uint64_t n, const double* x, const double* y, double* r, hipStream_t s);

}  // namespace gbs
