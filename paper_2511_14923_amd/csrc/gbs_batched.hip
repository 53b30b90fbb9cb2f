// Batched forward pass: many covariance instances of uneven M in persistent
// launches over device work lists.
//
// Orders 3..K, FP64 or mixed: the group kernel (gbs_forward_group.hip), one
// persistent launch per order whose work list holds the (instance, tile) items
// of every instance at that order; each instance reads the tables of its own
// lower orders, which the previous launches wrote.  Orders 1 and 2, instances
// the group kernel does not take (M too large) and GBS_ALL_MINORS:
// one persistent launch over (instance, order, rank range) items, longest
// first, each subset evaluated from all its minors (no tables needed), which
// also stores the tables the group launches read.  In every launch a fixed grid
// of workgroups claims items with one atomic counter until the list is
// exhausted, so large and small instances share the machine without
// per-instance launches or tail effects; every workgroup leaves its loop when
// the counter passes the end of the list, and no workgroup waits on another.
//
// The pipeline (counter and status reset, Q of every instance, diagonal blocks
// or normalisation, the persistent launches) is captured once into a HIP graph
// per instance list and replayed; the launch shapes come from the autotuner's
// cache (the group launches fill the device unless it caps their workgroups
// per compute unit).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <tuple>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "gbs_internal.h"
#include "gbs_subset.h"

namespace gbs {

struct BatchInstance {
  const double* sigma;
  double* Qi;
  double* Qd;    // diagonal blocks of Q (group kernel), or null
  double* pk;
  float* E;
  double* corr;
  double* cum;
  double* mtab;  // correlators of orders < K for the group kernel (corr, or scratch), or null
  double* ptab;  // vacuum probabilities of orders < K for the group kernel, or null
  int M;
  int K;
  int64_t off[kMaxOrder + 2];
};

struct WorkItem {
  int inst;
  int order;
  uint64_t begin;
  uint64_t end;
};

namespace {

// one counter per persistent launch: [0] all-minors items, [d] group items of order d
constexpr int kCounters = kMaxOrder + 1;

__global__ void reset_batch_kernel(unsigned* counter, DeviceStatus* st) {
  for (int i = 0; i < kCounters; ++i) counter[i] = 0u;
  st->flag = 0;
  st->order = 0;
  st->rank = -1;
}

__global__ void build_q_batched_kernel(const BatchInstance* __restrict__ inst) {
  const BatchInstance I = inst[blockIdx.y];
  const int n = 2 * I.M;
  const size_t total = (size_t)n * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(idx / n), col = (int)(idx - (size_t)row * n);
    const int sr = (row >> 1) + (row & 1) * I.M;
    const int sc = (col >> 1) + (col & 1) * I.M;
    const double v = (sr >= sc) ? I.sigma[(size_t)sr * n + sc] : I.sigma[(size_t)sc * n + sr];
    I.Qi[idx] = v + (row == col ? 0.5 : 0.0);
  }
}

__global__ void build_qdiag_batched_kernel(const BatchInstance* __restrict__ inst) {
  const BatchInstance I = inst[blockIdx.y];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (!I.Qd || k >= I.M) return;
  const size_t ldq = 2 * (size_t)I.M;
  const double* q = I.Qi + (size_t)(2 * k) * ldq + 2 * k;
  I.Qd[4 * (size_t)k + 0] = q[0];
  I.Qd[4 * (size_t)k + 1] = q[ldq];
  I.Qd[4 * (size_t)k + 2] = q[ldq + 1];
  I.Qd[4 * (size_t)k + 3] = 0.0;
}

__global__ void build_normalised_batched_kernel(const BatchInstance* __restrict__ inst) {
  const BatchInstance I = inst[blockIdx.y];
  const int M = I.M;
  const size_t ldq = 2 * (size_t)M;
  const size_t total = (size_t)M * M;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / M), l = (int)(idx - (size_t)k * M);
    const double* qk = I.Qi + (size_t)(2 * k) * ldq + 2 * k;
    const double ak = sqrt(qk[0]);
    const double bk = qk[ldq] / ak;
    const double ck = sqrt(qk[ldq + 1] - bk * bk);
    float* e = I.E + (size_t)(2 * k) * ldq + 2 * l;
    if (l == k) {
      I.pk[k] = 1.0 / (ak * ck);
      e[0] = e[1] = e[ldq] = e[ldq + 1] = 0.0f;
      continue;
    }
    const double* ql = I.Qi + (size_t)(2 * l) * ldq + 2 * l;
    const double al = sqrt(ql[0]);
    const double bl = ql[ldq] / al;
    const double cl = sqrt(ql[ldq + 1] - bl * bl);
    const double* q = I.Qi + (size_t)(2 * k) * ldq + 2 * l;
    const double x00 = q[0] / ak, x01 = q[1] / ak;
    const double x10 = (q[ldq] - bk * x00) / ck, x11 = (q[ldq + 1] - bk * x01) / ck;
    const double e00 = x00 / al, e10 = x10 / al;
    e[0] = (float)e00;
    e[1] = (float)((x01 - bl * e00) / cl);
    e[ldq] = (float)e10;
    e[ldq + 1] = (float)((x11 - bl * e10) / cl);
  }
}

template <int D, int UNROLL, int CONV, bool MIXED>
__device__ __forceinline__ void process_item(const BatchInstance& I, const WorkItem& w,
                                             const uint64_t* __restrict__ bin,
                                             DeviceStatus* __restrict__ st) {
  const uint64_t step = (uint64_t)blockDim.x * UNROLL;
  for (uint64_t base = w.begin + threadIdx.x; base < w.end; base += step) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const uint64_t r = base + (uint64_t)u * blockDim.x;
      if (r < w.end) {
        int s[D];
        colex_unrank<D>(r, I.M, bin, kBinLd, s);
        double mS, kS;
        bool bad = false;
        double pS = 0.0;
        if constexpr (MIXED) {
          subset_mixed<D, CONV, true>(I.pk, I.E, I.M, s, mS, kS, pS, bad);
        } else {
          subset_fp64<D, CONV, true>(I.Qi, I.M, s, mS, kS, pS, bad);
        }
        if (bad) latch_failure(st, D, (int64_t)r);
        const int64_t o = I.off[D] + (int64_t)r;
        if (I.corr) I.corr[o] = mS;
        else if (I.mtab && D < I.K) I.mtab[o] = mS;
        I.cum[o] = kS;
        if (I.ptab && D < I.K) I.ptab[o] = pS;
      }
    }
  }
}

template <int KMAX, int UNROLL, int CONV, bool MIXED>
__global__ __launch_bounds__(256) void batched_kernel(const BatchInstance* __restrict__ inst,
                                                      const WorkItem* __restrict__ items,
                                                      int n_items, unsigned* __restrict__ counter,
                                                      const uint64_t* __restrict__ bin,
                                                      DeviceStatus* __restrict__ st) {
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_items) break;  // every workgroup reaches this once the list is drained
    const WorkItem w = items[it];
    const BatchInstance I = inst[w.inst];
    switch (w.order) {
      case 1: process_item<1, UNROLL, CONV, MIXED>(I, w, bin, st); break;
      case 2: if constexpr (KMAX >= 2) process_item<2, UNROLL, CONV, MIXED>(I, w, bin, st); break;
      case 3: if constexpr (KMAX >= 3) process_item<3, UNROLL, CONV, MIXED>(I, w, bin, st); break;
      case 4: if constexpr (KMAX >= 4) process_item<4, UNROLL, CONV, MIXED>(I, w, bin, st); break;
      case 5: if constexpr (KMAX >= 5) process_item<5, UNROLL, CONV, MIXED>(I, w, bin, st); break;
      default: break;
    }
  }
}

using BatchedFn = void (*)(const BatchInstance*, const WorkItem*, int, unsigned*, const uint64_t*,
                           DeviceStatus*);

template <int KMAX, int UNROLL>
BatchedFn pick_conv(int flags) {
  const bool mixed = flags & GBS_MIXED;
  if (flags & GBS_PARITY)
    return mixed ? batched_kernel<KMAX, UNROLL, GBS_PARITY, true>
                 : batched_kernel<KMAX, UNROLL, GBS_PARITY, false>;
  return mixed ? batched_kernel<KMAX, UNROLL, GBS_CLICK, true>
               : batched_kernel<KMAX, UNROLL, GBS_CLICK, false>;
}

template <int KMAX>
BatchedFn pick_unroll(int unroll, int flags) {
  switch (unroll) {
    case 2: return pick_conv<KMAX, 2>(flags);
    case 4: return pick_conv<KMAX, 4>(flags);
    default: return pick_conv<KMAX, 1>(flags);
  }
}

BatchedFn pick_kernel(int K, int unroll, int flags) {
  if (K <= 3) return pick_unroll<3>(unroll, flags);
  if (K == 4) return pick_unroll<4>(unroll, flags);
  return pick_unroll<5>(unroll, flags);
}

// ---------------------------------------------------------------------------
// host side

struct TuneKey {
  int device, K, mode;
  bool operator<(const TuneKey& o) const {
    return std::tie(device, K, mode) < std::tie(o.device, o.K, o.mode);
  }
};
std::mutex g_tune_mutex;
std::map<TuneKey, gbs_tuning> g_tuning;

gbs_tuning default_tuning() { return gbs_tuning{256, 1, 65536, 2, 0}; }

bool valid_tuning(const gbs_tuning& t) {
  const bool blk = t.block == 64 || t.block == 128 || t.block == 256;
  const bool unr = t.unroll == 1 || t.unroll == 2 || t.unroll == 4;
  return blk && unr && t.tile >= t.block * t.unroll && t.tile % (t.block * t.unroll) == 0 &&
         t.waves_per_cu >= 1 && t.waves_per_cu <= 8 && t.group_wpc >= 0 && t.group_wpc <= 8;
}

gbs_tuning lookup_tuning(int device, int K, int flags) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  auto it = g_tuning.find(TuneKey{device, K, flags & (GBS_PARITY | GBS_MIXED)});
  return it == g_tuning.end() ? default_tuning() : it->second;
}

// Device-side state of one instance list: descriptors, work list, Q scratch,
// counter and status, plus the captured graph.
struct BatchPlan {
  int device = -1;
  std::vector<gbs_instance> key;
  int K = 0, flags = 0;
  gbs_tuning tuning{};
  void* mem = nullptr;
  BatchInstance* d_inst = nullptr;
  WorkItem* d_items = nullptr;
  unsigned* d_counter = nullptr;
  DeviceStatus* d_status = nullptr;
  int n_items = 0;
  int max_M = 0;
  int n = 0;
  bool any_group = false;
  // group launches, order d = 3..K
  GroupBatchInstance* d_ginst[kMaxOrder + 1] = {};
  GroupBatchItem* d_gitems[kMaxOrder + 1] = {};
  uint32_t n_gitems[kMaxOrder + 1] = {};
  int g_max_M[kMaxOrder + 1] = {};
  int g_nwin[kMaxOrder + 1] = {};
  size_t g_lds[kMaxOrder + 1] = {};
  int g_grid[kMaxOrder + 1] = {};
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the caller's stream: a plan serves one stream, whose order serialises the
  // calls that share its counter and status word
  hipStream_t stream = nullptr;
  // held while a call enqueues this plan's launches (threads sharing a stream)
  std::mutex launch_mu;

  ~BatchPlan() {
    if (mem) (void)hipDeviceSynchronize();  // the last holder frees it; its work may be queued
    release();
  }

  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (mem) (void)hipFree(mem);
    exec = nullptr;
    graph = nullptr;
    cap_stream = nullptr;
    mem = nullptr;
  }
};

std::mutex g_plan_mutex;
// most recent first; shared so that an evicted plan lives until the calls
// that hold it return
std::list<std::shared_ptr<BatchPlan>> g_plans;
constexpr size_t kMaxPlans = 8;

bool same_key(const BatchPlan* p, int dev, hipStream_t s, int n, const gbs_instance* inst, int K,
              int flags, const gbs_tuning& t) {
  if (p->device != dev || p->stream != s || p->K != K || p->flags != flags ||
      (int)p->key.size() != n)
    return false;
  if (p->tuning.block != t.block || p->tuning.unroll != t.unroll || p->tuning.tile != t.tile ||
      p->tuning.waves_per_cu != t.waves_per_cu || p->tuning.group_wpc != t.group_wpc)
    return false;
  return std::memcmp(p->key.data(), inst, sizeof(gbs_instance) * n) == 0;
}

// Order d of an instance of M modes runs on the group kernel (reading the
// tables of its lower orders) unless the call asks for all minors or the group
// kernel does not take that (d, M, form).
bool group_order(int d, int M, int flags) {
  return d >= 3 && !(flags & GBS_ALL_MINORS) && group_supported(d, M, flags, false);
}

double item_cost(const WorkItem& w) {
  // per-subset work grows like 2^d d^2 (2^d minors of a 2d x 2d matrix)
  return (double)(w.end - w.begin) * (double)(1 << w.order) * w.order * w.order;
}

hipError_t launch_pipeline(const BatchPlan& p, hipStream_t s, bool timed) {
  hipError_t e = hipSuccess;
  hipLaunchKernelGGL(reset_batch_kernel, dim3(1), dim3(1), 0, s, p.d_counter, p.d_status);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int bx = std::min(4096, (4 * p.max_M * p.max_M + 255) / 256);
  if (timed) e = timing_begin(s, GBS_STAGE_BUILD_Q, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(build_q_batched_kernel, dim3(bx, p.n), dim3(256), 0, s, p.d_inst);
  e = hipGetLastError();
  if (e == hipSuccess && p.any_group) {
    hipLaunchKernelGGL(build_qdiag_batched_kernel, dim3((p.max_M + 255) / 256, p.n), dim3(256), 0,
                       s, p.d_inst);
    e = hipGetLastError();
  }
  if (e == hipSuccess && timed) e = timing_end(s);
  if (e == hipSuccess && (p.flags & GBS_MIXED)) {
    if (timed) e = timing_begin(s, GBS_STAGE_NORMALISE, 0);
    const int by = std::min(4096, (p.max_M * p.max_M + 255) / 256);
    if (e == hipSuccess)
      hipLaunchKernelGGL(build_normalised_batched_kernel, dim3(by, p.n), dim3(256), 0, s, p.d_inst);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess && timed) e = timing_end(s);
  }
  if (e != hipSuccess) return e;
  hipError_t ec;
  DeviceContext* ctx = current_context(&ec);
  if (!ctx) return ec;
  if (p.n_items > 0) {
    const int grid = std::max(1, ctx->cu_count * p.tuning.waves_per_cu);
    BatchedFn fn = pick_kernel(p.K, p.tuning.unroll, p.flags);
    if (timed) e = timing_begin(s, GBS_STAGE_BATCHED, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(p.tuning.block), 0, s, p.d_inst, p.d_items,
                       p.n_items, p.d_counter, ctx->binom, p.d_status);
    e = hipGetLastError();
    if (e == hipSuccess && timed) e = timing_end(s);
  }
  for (int d = 3; d <= p.K && e == hipSuccess; ++d) {
    if (p.n_gitems[d] == 0) continue;
    if (timed) e = timing_begin(s, GBS_STAGE_BATCHED, d);
    if (e == hipSuccess)
      e = launch_group_batched(d, p.flags, p.d_ginst[d], p.d_gitems[d], p.n_gitems[d],
                               p.d_counter + d, p.g_grid[d], p.g_max_M[d], p.g_nwin[d],
                               p.g_lds[d], ctx->binom, p.d_status, s);
    if (e == hipSuccess && timed) e = timing_end(s);
  }
  return e;
}

// Allocate and upload the plan's device state (synchronous; once per list).
gbs_status build_plan(BatchPlan* p, int n, const gbs_instance* inst, int K, int flags,
                      const gbs_tuning& t) {
  p->key.assign(inst, inst + n);
  p->K = K;
  p->flags = flags;
  p->tuning = t;
  p->n = n;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return GBS_E_DEVICE;
  hipError_t ec;
  DeviceContext* ctx = current_context(&ec);
  if (!ctx) return to_status(ec);
  const bool mixed = flags & GBS_MIXED;
  std::vector<BatchInstance> host(n);
  std::vector<WorkItem> items;
  std::vector<GroupBatchItem> gitems[kMaxOrder + 1];
  size_t bytes = 0;
  auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
  std::vector<size_t> q_off(n), pk_off(n), e_off(n), qd_off(n), pt_off(n), mt_off(n);
  std::vector<bool> grp(n, false);
  p->max_M = 0;
  p->any_group = false;
  // group items, largest instances first
  std::vector<int> by_M(n);
  for (int i = 0; i < n; ++i) by_M[i] = i;
  std::stable_sort(by_M.begin(), by_M.end(), [&](int x, int y) { return inst[x].M > inst[y].M; });
  std::vector<uint64_t> tiles;
  for (int d = 3; d <= K; ++d) {
    p->g_max_M[d] = 0;
    for (int i : by_M) {
      if (!group_order(d, inst[i].M, flags)) continue;
      tiles.clear();
      group_tiles(d, inst[i].M, (flags & GBS_MIXED) != 0, &tiles);
      for (uint64_t desc : tiles) gitems[d].push_back(GroupBatchItem{(uint32_t)i, 0u, desc});
      p->g_max_M[d] = std::max(p->g_max_M[d], inst[i].M);
      grp[i] = true;
    }
  }
  for (int i = 0; i < n; ++i) {
    const int M = inst[i].M;
    p->max_M = std::max(p->max_M, M);
    BatchInstance& b = host[i];
    b.sigma = inst[i].sigma;
    b.corr = inst[i].corr;
    b.cum = inst[i].cum;
    b.M = M;
    b.K = K;
    b.off[1] = 0;
    for (int d = 1; d <= kMaxOrder; ++d)
      b.off[d + 1] = b.off[d] + (d <= K ? (int64_t)host_binom(M, d) : 0);
    q_off[i] = bytes;
    bytes += a256(4 * (size_t)M * M * sizeof(double));
    if (mixed) {
      pk_off[i] = bytes;
      bytes += a256((size_t)M * sizeof(double));
      e_off[i] = bytes;
      bytes += a256(4 * (size_t)M * M * sizeof(float));
    }
    if (grp[i]) {
      p->any_group = true;
      qd_off[i] = bytes;
      bytes += a256(4 * (size_t)M * sizeof(double));
      pt_off[i] = bytes;  // orders 1 .. K-1
      bytes += a256((size_t)b.off[K] * sizeof(double));
      if (!b.corr) {
        mt_off[i] = bytes;
        bytes += a256((size_t)b.off[K] * sizeof(double));
      }
    }
    for (int d = 1; d <= K; ++d) {
      if (grp[i] && group_order(d, M, flags)) continue;
      const uint64_t cnt = host_binom(M, d);
      for (uint64_t b0 = 0; b0 < cnt; b0 += (uint64_t)t.tile)
        items.push_back(WorkItem{i, d, b0, std::min<uint64_t>(cnt, b0 + (uint64_t)t.tile)});
    }
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const WorkItem& a, const WorkItem& b) { return item_cost(a) > item_cost(b); });
  const size_t o_inst = bytes;
  bytes += a256(sizeof(BatchInstance) * n);
  const size_t o_items = bytes;
  bytes += a256(sizeof(WorkItem) * items.size());
  size_t o_ginst[kMaxOrder + 1] = {}, o_gitems[kMaxOrder + 1] = {};
  for (int d = 3; d <= K; ++d) {
    if (gitems[d].empty()) continue;
    o_ginst[d] = bytes;
    bytes += a256(sizeof(GroupBatchInstance) * n);
    o_gitems[d] = bytes;
    bytes += a256(sizeof(GroupBatchItem) * gitems[d].size());
  }
  const size_t o_cnt = bytes;
  bytes += a256(sizeof(unsigned) * kCounters);
  const size_t o_st = bytes;
  bytes += 256;
  // group launch shapes (occupancy queries stay outside graph capture)
  for (int d = 3; d <= K; ++d) {
    p->n_gitems[d] = (uint32_t)gitems[d].size();
    if (gitems[d].empty()) continue;
    p->g_lds[d] = group_batched_lds(d, flags, p->g_max_M[d], &p->g_nwin[d]);
    e = group_batched_grid(d, flags, p->g_lds[d], ctx->cu_count, &p->g_grid[d]);
    if (e != hipSuccess) return to_status(e);
    if (t.group_wpc > 0) p->g_grid[d] = std::min(p->g_grid[d], ctx->cu_count * t.group_wpc);
  }
  e = hipMalloc(&p->mem, bytes);
  if (e != hipSuccess) return to_status(e);
  char* base = static_cast<char*>(p->mem);
  for (int i = 0; i < n; ++i) {
    BatchInstance& b = host[i];
    b.Qi = reinterpret_cast<double*>(base + q_off[i]);
    b.pk = mixed ? reinterpret_cast<double*>(base + pk_off[i]) : nullptr;
    b.E = mixed ? reinterpret_cast<float*>(base + e_off[i]) : nullptr;
    b.Qd = grp[i] ? reinterpret_cast<double*>(base + qd_off[i]) : nullptr;
    b.ptab = grp[i] ? reinterpret_cast<double*>(base + pt_off[i]) : nullptr;
    b.mtab = !grp[i] ? nullptr : b.corr ? b.corr : reinterpret_cast<double*>(base + mt_off[i]);
  }
  std::vector<GroupBatchInstance> gh(n);
  for (int d = 3; d <= K && e == hipSuccess; ++d) {
    if (gitems[d].empty()) continue;
    for (int i = 0; i < n; ++i) {
      const BatchInstance& b = host[i];
      GroupBatchInstance& g = gh[i];
      g = GroupBatchInstance{};
      g.Qi = b.Qi;
      g.Qd = b.Qd;
      g.pk = b.pk;
      g.E = b.E;
      g.M = b.M;
      if (!grp[i]) continue;  // never referenced by an item
      for (int q = 1; q < d; ++q) {
        g.tab.p[q] = b.ptab + b.off[q];
        g.tab.m[q] = b.mtab + b.off[q];
        g.tab.k[q] = b.cum + b.off[q];
      }
      g.m_out = b.corr ? b.corr + b.off[d] : (d < K ? b.mtab + b.off[d] : nullptr);
      g.k_out = b.cum + b.off[d];
      g.p_out = d < K ? b.ptab + b.off[d] : nullptr;
    }
    p->d_ginst[d] = reinterpret_cast<GroupBatchInstance*>(base + o_ginst[d]);
    p->d_gitems[d] = reinterpret_cast<GroupBatchItem*>(base + o_gitems[d]);
    e = hipMemcpy(p->d_ginst[d], gh.data(), sizeof(GroupBatchInstance) * n,
                  hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_gitems[d], gitems[d].data(), sizeof(GroupBatchItem) * gitems[d].size(),
                    hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return to_status(e);
  p->d_inst = reinterpret_cast<BatchInstance*>(base + o_inst);
  p->d_items = reinterpret_cast<WorkItem*>(base + o_items);
  p->d_counter = reinterpret_cast<unsigned*>(base + o_cnt);
  p->d_status = reinterpret_cast<DeviceStatus*>(base + o_st);
  p->n_items = (int)items.size();
  e = hipMemcpy(p->d_inst, host.data(), sizeof(BatchInstance) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(p->d_items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice);
  return to_status(e);
}

gbs_status capture_plan(BatchPlan* p) {
  hipError_t e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return to_status(e);
  e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return to_status(e);
  hipError_t le = launch_pipeline(*p, p->cap_stream, false);
  e = hipStreamEndCapture(p->cap_stream, &p->graph);
  if (le != hipSuccess) return to_status(le);
  if (e != hipSuccess) return to_status(e);
  e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  return to_status(e);
}

bool valid_batch(int n, const gbs_instance* inst, int K, int flags) {
  if (n < 1 || n > 4096 || !inst) return false;
  if (K < 1 || K > GBS_MAX_ORDER) return false;
  if (flags & ~(GBS_PARITY | GBS_MIXED | GBS_ASYNC | GBS_TIMING | GBS_ALL_MINORS)) return false;
  for (int i = 0; i < n; ++i) {
    const gbs_instance& I = inst[i];
    if (I.M < K || I.M > GBS_MAX_MODES || I.reserved != 0 || !I.sigma || !I.cum) return false;
  }
  return true;
}

}  // namespace

gbs_status run_batched(int n, const gbs_instance* inst, int K, int flags, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  DeviceContext* ctx = current_context(&e);
  if (!ctx) return to_status(e);
  const int key_flags = flags & (GBS_PARITY | GBS_MIXED | GBS_ALL_MINORS);
  const gbs_tuning t = lookup_tuning(ctx->device, K, flags);
  std::shared_ptr<BatchPlan> plan;
  {
    std::lock_guard<std::mutex> lock(g_plan_mutex);
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
      if (same_key(it->get(), ctx->device, s, n, inst, K, key_flags, t)) {
        plan = *it;
        g_plans.erase(it);
        g_plans.push_front(plan);
        break;
      }
    }
  }
  if (!plan) {
    plan = std::make_shared<BatchPlan>();
    plan->stream = s;
    gbs_status st = build_plan(plan.get(), n, inst, K, key_flags, t);
    if (st == GBS_OK) st = capture_plan(plan.get());
    if (st != GBS_OK) return st;  // the destructor releases what was built
    std::lock_guard<std::mutex> lock(g_plan_mutex);
    g_plans.push_front(plan);
    while (g_plans.size() > kMaxPlans) g_plans.pop_back();  // freed by its last holder
  }
  std::lock_guard<std::mutex> launch(plan->launch_mu);
  if (flags & GBS_TIMING) {
    // same kernels, launched one by one so that each gets its event pair
    timing_start_call(true);
    e = launch_pipeline(*plan, s, true);
  } else {
    e = hipGraphLaunch(plan->exec, s);
  }
  if (e != hipSuccess) return to_status(e);
  return finish_status(plan->d_status, flags, s);
}

gbs_status run_autotune(int n, const gbs_instance* inst, int K, int flags, void* stream,
                        gbs_tuning* best_out) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  DeviceContext* ctx = current_context(&e);
  if (!ctx) return to_status(e);
  std::vector<gbs_tuning> cands;
  for (int block : {64, 128, 256})
    for (int unroll : {1, 2, 4})
      for (int tile_mult : {16, 64, 256})
        for (int wpc : {1, 2, 4})
          cands.push_back(gbs_tuning{block, unroll, block * unroll * tile_mult, wpc, 0});
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return GBS_E_DEVICE;
  float best_ms = 1e30f;
  gbs_tuning best = default_tuning();
  gbs_status result = GBS_OK;
  // the whole pipeline with shape t, three timed runs after a warm-up
  auto try_shape = [&](const gbs_tuning& t) -> gbs_status {
    BatchPlan plan;
    gbs_status st =
        build_plan(&plan, n, inst, K, flags & (GBS_PARITY | GBS_MIXED | GBS_ALL_MINORS), t);
    if (st != GBS_OK) {
      plan.release();
      return st;
    }
    float total = 0.f;
    e = launch_pipeline(plan, s, false);  // warm-up
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      e = hipEventRecord(a, s);
      if (e == hipSuccess) e = launch_pipeline(plan, s, false);
      if (e == hipSuccess) e = hipEventRecord(b, s);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      total += ms;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    plan.release();
    if (e != hipSuccess) return to_status(e);
    if (total < best_ms) {
      best_ms = total;
      best = t;
    }
    return GBS_OK;
  };
  // the all-minors launch's shape, then the group launches' workgroups per CU
  for (const gbs_tuning& t : cands) {
    result = try_shape(t);
    if (result != GBS_OK) break;
  }
  for (int gw : {2, 1}) {
    if (result != GBS_OK) break;
    gbs_tuning t = best;
    t.group_wpc = gw;
    result = try_shape(t);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (result != GBS_OK) return result;
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tuning[TuneKey{ctx->device, K, flags & (GBS_PARITY | GBS_MIXED)}] = best;
  }
  if (best_out) *best_out = best;
  return GBS_OK;
}

gbs_status set_tuning(int K, int flags, const gbs_tuning* t) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GBS_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  const TuneKey key{dev, K, flags & (GBS_PARITY | GBS_MIXED)};
  if (!t) {
    g_tuning.erase(key);
    return GBS_OK;
  }
  if (!valid_tuning(*t)) return GBS_E_INVALID_ARG;
  g_tuning[key] = *t;
  return GBS_OK;
}

}  // namespace gbs

using namespace gbs;

extern "C" {

gbs_status gbs_cumulants_batched(int32_t n, const gbs_instance* inst, int32_t max_order,
                                 int32_t flags, void* stream) {
  if (!valid_batch(n, inst, max_order, flags)) return GBS_E_INVALID_ARG;
  return run_batched(n, inst, max_order, flags, stream);
}

gbs_status gbs_autotune_batched(int32_t n, const gbs_instance* inst, int32_t max_order,
                                int32_t flags, void* stream, gbs_tuning* best) {
  if (!valid_batch(n, inst, max_order, flags)) return GBS_E_INVALID_ARG;
  return run_autotune(n, inst, max_order, flags, stream, best);
}

gbs_status gbs_set_tuning(int32_t max_order, int32_t flags, const gbs_tuning* t) {
  if (max_order < 1 || max_order > GBS_MAX_ORDER) return GBS_E_INVALID_ARG;
  if (flags & ~(GBS_PARITY | GBS_MIXED | GBS_ASYNC | GBS_TIMING | GBS_ALL_MINORS))
    return GBS_E_INVALID_ARG;
  return set_tuning(max_order, flags, t);
}

}  // extern "C"
