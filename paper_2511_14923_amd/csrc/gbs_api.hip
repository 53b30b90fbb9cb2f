// C ABI of libgbs: argument checks, per-device context, scratch, launches.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "gbs.h"
#include "gbs_internal.h"

namespace gbs {

uint64_t host_binom(int n, int k) {
  if (k < 0 || n < k) return 0;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}

namespace {

std::mutex g_ctx_mutex;
std::vector<DeviceContext*> g_ctx;  // indexed by device ordinal

struct ThreadError {
  int32_t order = 0;
  int64_t rank = -1;
  bool pending_async = false;
  DeviceStatus* host_status = nullptr;  // pinned, written by the last async call
  // status word of the last asynchronous allocation-free call, read back by
  // gbs_last_error (null for the other entry points)
  const DeviceStatus* pending_dev = nullptr;
};
thread_local ThreadError t_err;

struct TimingRecord {
  int stage, order;
  hipEvent_t a, b;
};
thread_local bool t_timing_on = false;
thread_local std::vector<TimingRecord> t_timing;
thread_local std::vector<hipEvent_t> t_event_pool;
thread_local size_t t_pool_used = 0;

hipError_t pooled_event(hipEvent_t* ev) {
  if (t_pool_used == t_event_pool.size()) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    t_event_pool.push_back(e);
  }
  *ev = t_event_pool[t_pool_used++];
  return hipSuccess;
}

}  // namespace

void timing_start_call(bool enabled) {
  t_timing_on = enabled;
  if (enabled) {
    t_timing.clear();
    t_pool_used = 0;
  }
}

hipError_t timing_begin(hipStream_t s, int stage, int order) {
  if (!t_timing_on) return hipSuccess;
  TimingRecord r{stage, order, nullptr, nullptr};
  hipError_t e = pooled_event(&r.a);
  if (e == hipSuccess) e = pooled_event(&r.b);
  if (e == hipSuccess) e = hipEventRecord(r.a, s);
  if (e == hipSuccess) t_timing.push_back(r);
  return e;
}

hipError_t timing_end(hipStream_t s) {
  if (!t_timing_on || t_timing.empty()) return hipSuccess;
  return hipEventRecord(t_timing.back().b, s);
}

DeviceContext* current_context(hipError_t* err) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *err = e;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_ctx_mutex);
  if ((int)g_ctx.size() <= dev) g_ctx.resize(dev + 1, nullptr);
  if (g_ctx[dev]) {
    *err = hipSuccess;
    return g_ctx[dev];
  }
  auto* c = new DeviceContext();
  c->device = dev;
  std::vector<uint64_t> tab((size_t)kBinRows * kBinLd);
  for (int k = 0; k < kBinRows; ++k)
    for (int n = 0; n < kBinLd; ++n) tab[(size_t)k * kBinLd + n] = host_binom(n, k);
  e = hipMalloc(&c->binom, tab.size() * sizeof(uint64_t));
  if (e == hipSuccess)
    e = hipMemcpy(c->binom, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    if (c->binom) (void)hipFree(c->binom);
    delete c;
    *err = e;
    return nullptr;
  }
  g_ctx[dev] = c;
  *err = hipSuccess;
  return c;
}

gbs_status to_status(hipError_t e) {
  if (e == hipSuccess) return GBS_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return GBS_E_OUT_OF_MEMORY;
  return GBS_E_DEVICE;
}

bool valid_problem(int32_t M, int32_t K, int32_t flags) {
  if (M < 1 || M > GBS_MAX_MODES) return false;
  if (K < 1 || K > GBS_MAX_ORDER || K > M) return false;
  if (flags & ~(GBS_PARITY | GBS_MIXED | GBS_ASYNC | GBS_TIMING | GBS_ALL_MINORS)) return false;
  return true;
}

// Scratch layout of one forward call.
struct ForwardScratch {
  double* Qi;
  double* Qd;
  double* mi;  // interleaved first moments (displaced states), else null
  double* pk;
  float* E;
  DeviceStatus* st;
  size_t bytes;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

ForwardScratch layout_scratch(char* base, int M, bool mixed, bool displaced) {
  ForwardScratch s{};
  size_t off = 0;
  const size_t nq = 4 * (size_t)M * M;
  s.Qi = reinterpret_cast<double*>(base + off);
  off += align256(nq * sizeof(double));
  s.Qd = reinterpret_cast<double*>(base + off);
  off += align256(4 * (size_t)M * sizeof(double));
  if (displaced) {
    s.mi = reinterpret_cast<double*>(base + off);
    off += align256(2 * (size_t)M * sizeof(double));
  } else {
    s.mi = nullptr;
  }
  if (mixed) {
    s.pk = reinterpret_cast<double*>(base + off);
    off += align256((size_t)M * sizeof(double));
    s.E = reinterpret_cast<float*>(base + off);
    off += align256(nq * sizeof(float));
  } else {
    s.pk = nullptr;
    s.E = nullptr;
  }
  s.st = reinterpret_cast<DeviceStatus*>(base + off);
  off += align256(sizeof(DeviceStatus));
  s.bytes = off;
  return s;
}

// Queue the copy of the device status word to this thread's pinned slot.
static gbs_status status_enqueue(DeviceStatus* dev_status, hipStream_t s) {
  t_err.pending_dev = nullptr;
  if (!t_err.host_status) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&t_err.host_status), sizeof(DeviceStatus),
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
      t_err.host_status = nullptr;
      return to_status(e);
    }
  }
  return to_status(hipMemcpyAsync(t_err.host_status, dev_status, sizeof(DeviceStatus),
                                  hipMemcpyDeviceToHost, s));
}

// Wait for the stream (unless ASYNC) and report the copied status.
static gbs_status status_wait(int32_t flags, hipStream_t s) {
  if (flags & GBS_ASYNC) {
    t_err.pending_async = true;
    return GBS_OK;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return to_status(e);
  t_err.pending_async = false;
  if (t_err.host_status->flag) {
    t_err.order = t_err.host_status->order;
    t_err.rank = t_err.host_status->rank;
    return GBS_E_NOT_SPD;
  }
  t_err.order = 0;
  t_err.rank = -1;
  return GBS_OK;
}

gbs_status finish_status(DeviceStatus* dev_status, int32_t flags, hipStream_t s) {
  t_err.order = 0;
  t_err.rank = -1;
  gbs_status st = status_enqueue(dev_status, s);
  if (st != GBS_OK) return st;
  return status_wait(flags, s);
}

// The end of a call that may not allocate: the status word stays on the
// device; a synchronous call waits for the stream and reads it with a blocking
// copy into host memory of its own, an asynchronous one leaves it for
// gbs_last_error.
gbs_status finish_status_device(const DeviceStatus* dev_status, int32_t flags, hipStream_t s) {
  t_err.order = 0;
  t_err.rank = -1;
  if (flags & GBS_ASYNC) {
    t_err.pending_async = true;
    t_err.pending_dev = dev_status;
    return GBS_OK;
  }
  t_err.pending_async = false;
  t_err.pending_dev = nullptr;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return to_status(e);
  DeviceStatus h{};
  e = hipMemcpy(&h, dev_status, sizeof(h), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return to_status(e);
  if (h.flag) {
    t_err.order = h.order;
    t_err.rank = h.rank;
    return GBS_E_NOT_SPD;
  }
  return GBS_OK;
}

// Report the status, then release the call's stream-ordered scratch (the free
// is queued after the status copy on the same stream).
gbs_status finish_call(DeviceStatus* dev_status, void* scratch, int32_t flags, hipStream_t s) {
  gbs_status st = status_enqueue(dev_status, s);
  hipError_t e = hipFreeAsync(scratch, s);
  if (st != GBS_OK) return st;
  if (e != hipSuccess) return to_status(e);
  return status_wait(flags, s);
}

// mu: device first moments (2M, xxpp) of a displaced state, or null.
gbs_status run_forward(int32_t M, const double* sigma, const double* mu, int32_t K, int32_t flags,
                       double* corr, double* cum, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  DeviceContext* ctx = current_context(&e);
  if (!ctx) return to_status(e);
  const bool mixed = (flags & GBS_MIXED) != 0;
  const bool rec = !(flags & GBS_ALL_MINORS);
  ForwardScratch probe = layout_scratch(nullptr, M, mixed, mu != nullptr);
  // lower-order tables of the recursive kernel: p always, m when corr is NULL
  const size_t nlow = K >= 2 ? (size_t)gbs_order_offset(M, K) : 0;
  const size_t tab_bytes = rec ? align256(nlow * sizeof(double)) * (corr ? 1 : 2) : 0;
  void* scratch = nullptr;
  e = hipMallocAsync(&scratch, probe.bytes + tab_bytes, s);
  if (e != hipSuccess) return to_status(e);
  ForwardScratch sc = layout_scratch(static_cast<char*>(scratch), M, mixed, mu != nullptr);
  double* ptab = reinterpret_cast<double*>(static_cast<char*>(scratch) + probe.bytes);
  double* mtab = corr ? corr : ptab + align256(nlow * sizeof(double)) / sizeof(double);
  t_err.order = 0;
  t_err.rank = -1;
  timing_start_call((flags & GBS_TIMING) != 0);
  e = launch_clear_status(sc.st, s);
  if (e == hipSuccess) e = timing_begin(s, GBS_STAGE_BUILD_Q, 0);
  if (e == hipSuccess) e = launch_build_q(sigma, M, sc.Qi, s);
  if (e == hipSuccess) e = launch_build_qdiag(sc.Qi, M, sc.Qd, s);
  if (e == hipSuccess && mu) e = launch_build_mean(mu, M, sc.mi, s);
  if (e == hipSuccess) e = timing_end(s);
  if (e == hipSuccess && mixed) {
    e = timing_begin(s, GBS_STAGE_NORMALISE, 0);
    if (e == hipSuccess) e = launch_build_normalised(sc.Qi, M, sc.pk, sc.E, s);
    if (e == hipSuccess) e = timing_end(s);
  }
  const double* p_tab[kMaxOrder + 1] = {};
  const double* m_tab[kMaxOrder + 1] = {};
  const double* k_tab[kMaxOrder + 1] = {};
  for (int d = 1; d <= K && e == hipSuccess; ++d) {
    const int64_t off = gbs_order_offset(M, d);
    e = timing_begin(s, GBS_STAGE_FORWARD, d);
    if (e != hipSuccess) break;
    if (rec) {
      double* m_out = (corr || d < K) ? mtab + off : nullptr;
      double* k_out = cum ? cum + off : nullptr;
      double* p_out = d < K ? ptab + off : nullptr;
      e = launch_forward_rec(d, M, flags, sc.Qi, sc.Qd, sc.mi, sc.pk, sc.E, ctx->binom, p_tab, m_tab,
                             k_tab, m_out, k_out, p_out, sc.st, s);
      p_tab[d] = ptab + off;
      m_tab[d] = mtab + off;
      k_tab[d] = cum ? cum + off : nullptr;
    } else {
      e = launch_forward(d, M, flags, sc.Qi, sc.mi, sc.pk, sc.E, ctx->binom,
                         corr ? corr + off : nullptr,
                         cum ? cum + off : nullptr, nullptr, sc.st, s);
    }
    if (e == hipSuccess) e = timing_end(s);
  }
  if (e != hipSuccess) {
    (void)hipFreeAsync(scratch, s);
    return to_status(e);
  }
  return finish_call(sc.st, scratch, flags, s);
}

gbs_status run_shard(int32_t M, const double* sigma, int32_t d, int64_t rank0, int64_t count,
                     int32_t flags, double* corr, double* cum, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  DeviceContext* ctx = current_context(&e);
  if (!ctx) return to_status(e);
  const size_t oQ = 0, oSt = align256(4 * (size_t)M * M * sizeof(double));
  void* scratch = nullptr;
  e = hipMallocAsync(&scratch, oSt + align256(sizeof(DeviceStatus)), s);
  if (e != hipSuccess) return to_status(e);
  double* Qi = reinterpret_cast<double*>(static_cast<char*>(scratch) + oQ);
  DeviceStatus* st = reinterpret_cast<DeviceStatus*>(static_cast<char*>(scratch) + oSt);
  t_err.order = 0;
  t_err.rank = -1;
  timing_start_call((flags & GBS_TIMING) != 0);
  e = launch_clear_status(st, s);
  if (e == hipSuccess) e = timing_begin(s, GBS_STAGE_BUILD_Q, 0);
  if (e == hipSuccess) e = launch_build_q(sigma, M, Qi, s);
  if (e == hipSuccess) e = timing_end(s);
  if (e == hipSuccess) e = timing_begin(s, GBS_STAGE_FORWARD, d);
  // orders >= 3: the T-shared kernel; orders 1, 2 and GBS_ALL_MINORS: the all-minors kernel
  if (e == hipSuccess && d >= 3 && !(flags & GBS_ALL_MINORS))
    e = launch_forward_shard(d, M, flags, Qi, (uint64_t)rank0, (uint64_t)count, corr,
                             cum, st, s);
  else if (e == hipSuccess)
    e = launch_forward_range(d, M, flags, Qi, ctx->binom, (uint64_t)rank0, (uint64_t)count, corr,
                             cum, st, s);
  if (e == hipSuccess) e = timing_end(s);
  if (e != hipSuccess) {
    (void)hipFreeAsync(scratch, s);
    return to_status(e);
  }
  return finish_call(st, scratch, flags, s);
}

gbs_status run_adjoint(int32_t M, const double* sigma, int32_t K, int32_t flags,
                       const double* gm, const double* gk, double* gsig, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  DeviceContext* ctx = current_context(&e);
  if (!ctx) return to_status(e);
  const size_t N = (size_t)gbs_total_outputs(M, K);
  const size_t nq = 4 * (size_t)M * M;
  size_t off = 0;
  const size_t oQ = off; off += align256(nq * sizeof(double));
  const size_t oQd = off; off += align256(4 * (size_t)M * sizeof(double));
  const size_t oP = off; off += align256(N * sizeof(double));
  const size_t oM = off; off += align256(N * sizeof(double));
  const size_t oD = off; off += align256(N * sizeof(double));
  const size_t oMb = off; off += align256(N * sizeof(double));
  const size_t oPb = off; off += align256(N * sizeof(double));
  const size_t oSt = off; off += align256(sizeof(DeviceStatus));
  const size_t oPart = off; off += align256(kAdjointPartDoubles * sizeof(double));
  void* scratch = nullptr;
  e = hipMallocAsync(&scratch, off, s);
  if (e != hipSuccess) return to_status(e);
  char* b = static_cast<char*>(scratch);
  double* Qi = reinterpret_cast<double*>(b + oQ);
  double* Qd = reinterpret_cast<double*>(b + oQd);
  double* ptab = reinterpret_cast<double*>(b + oP);
  double* part = reinterpret_cast<double*>(b + oPart);
  double* m = reinterpret_cast<double*>(b + oM);
  double* d1 = reinterpret_cast<double*>(b + oD);
  double* mbar = reinterpret_cast<double*>(b + oMb);
  double* pbar = reinterpret_cast<double*>(b + oPb);
  DeviceStatus* st = reinterpret_cast<DeviceStatus*>(b + oSt);
  t_err.order = 0;
  t_err.rank = -1;
  timing_start_call((flags & GBS_TIMING) != 0);
  e = launch_clear_status(st, s);
  if (e == hipSuccess) e = timing_begin(s, GBS_STAGE_BUILD_Q, 0);
  if (e == hipSuccess) e = launch_build_q(sigma, M, Qi, s);
  if (e == hipSuccess) e = launch_build_qdiag(Qi, M, Qd, s);
  if (e == hipSuccess) e = timing_end(s);
  const double* p_tab[kMaxOrder + 1] = {};
  const double* m_tab[kMaxOrder + 1] = {};
  const double* k_tab[kMaxOrder + 1] = {};
  for (int d = 1; d <= K && e == hipSuccess; ++d) {
    const int64_t o = gbs_order_offset(M, d);
    e = timing_begin(s, GBS_STAGE_FORWARD, d);
    if (e == hipSuccess)
      e = launch_forward_rec(d, M, flags & GBS_PARITY, Qi, Qd, nullptr, nullptr, nullptr, ctx->binom,
                             p_tab, m_tab, k_tab, m + o, nullptr, ptab + o, st, s);
    p_tab[d] = ptab + o;
    m_tab[d] = m + o;
    if (e == hipSuccess) e = timing_end(s);
  }
  if (e == hipSuccess)
    e = launch_adjoint(M, K, flags, Qi, ctx->binom, m, ptab, gm, gk, d1, mbar, pbar, gsig, st, part,
                       s);
  if (e != hipSuccess) {
    (void)hipFreeAsync(scratch, s);
    return to_status(e);
  }
  return finish_call(st, scratch, flags, s);
}

}  // namespace gbs

using namespace gbs;

extern "C" {

int64_t gbs_num_subsets(int32_t M, int32_t d) {
  if (M < 0 || M > GBS_MAX_MODES || d < 0 || d > M) return -1;
  return (int64_t)host_binom(M, d);
}

int64_t gbs_order_offset(int32_t M, int32_t d) {
  if (M < 1 || M > GBS_MAX_MODES || d < 1 || d > GBS_MAX_ORDER + 1 || d > M + 1) return -1;
  int64_t off = 0;
  for (int e = 1; e < d; ++e) off += (int64_t)host_binom(M, e);
  return off;
}

int64_t gbs_total_outputs(int32_t M, int32_t max_order) {
  if (M < 1 || M > GBS_MAX_MODES || max_order < 1 || max_order > GBS_MAX_ORDER || max_order > M)
    return -1;
  return gbs_order_offset(M, max_order + 1);
}

int64_t gbs_colex_rank(int32_t d, const int32_t* S) {
  if (!S || d < 1 || d > GBS_MAX_ORDER) return -1;
  int32_t v[GBS_MAX_ORDER];
  for (int i = 0; i < d; ++i) {
    if (S[i] < 0 || S[i] >= GBS_MAX_MODES) return -1;
    v[i] = S[i];
  }
  for (int i = 1; i < d; ++i)  // insertion sort
    for (int j = i; j > 0 && v[j - 1] > v[j]; --j) {
      const int32_t t = v[j];
      v[j] = v[j - 1];
      v[j - 1] = t;
    }
  for (int i = 1; i < d; ++i)
    if (v[i] == v[i - 1]) return -1;
  int64_t r = 0;
  for (int j = 0; j < d; ++j) r += (int64_t)host_binom(v[j], j + 1);
  return r;
}

gbs_status gbs_colex_unrank(int32_t d, int64_t r, int32_t* S) {
  if (!S || d < 1 || d > GBS_MAX_ORDER || r < 0) return GBS_E_INVALID_ARG;
  if ((uint64_t)r >= host_binom(GBS_MAX_MODES, d)) return GBS_E_INVALID_ARG;
  uint64_t rr = (uint64_t)r;
  for (int j = d; j >= 1; --j) {
    int lo = j - 1, hi = GBS_MAX_MODES - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (host_binom(mid, j) <= rr) lo = mid; else hi = mid - 1;
    }
    S[j - 1] = lo;
    rr -= host_binom(lo, j);
  }
  return GBS_OK;
}

gbs_status gbs_correlators(int32_t M, const double* sigma, int32_t max_order, int32_t flags,
                           double* corr, void* stream) {
  if (!valid_problem(M, max_order, flags) || !sigma || !corr) return GBS_E_INVALID_ARG;
  return run_forward(M, sigma, nullptr, max_order, flags, corr, nullptr, stream);
}

gbs_status gbs_cumulants(int32_t M, const double* sigma, int32_t max_order, int32_t flags,
                         double* corr, double* cum, void* stream) {
  if (!valid_problem(M, max_order, flags) || !sigma || !cum) return GBS_E_INVALID_ARG;
  return run_forward(M, sigma, nullptr, max_order, flags, corr, cum, stream);
}

gbs_status gbs_cumulants_displaced(int32_t M, const double* sigma, const double* mu,
                                   int32_t max_order, int32_t flags, double* corr, double* cum,
                                   void* stream) {
  if (!valid_problem(M, max_order, flags) || !sigma || !mu || !cum) return GBS_E_INVALID_ARG;
  if (flags & GBS_MIXED) return GBS_E_UNSUPPORTED;
  return run_forward(M, sigma, mu, max_order, flags, corr, cum, stream);
}

gbs_status gbs_cumulants_shard(int32_t M, const double* sigma, int32_t order, int64_t rank0,
                               int64_t count, int32_t flags, double* corr, double* cum,
                               void* stream) {
  if (!valid_problem(M, order, flags) || !sigma || (!corr && !cum)) return GBS_E_INVALID_ARG;
  if (rank0 < 0 || count < 0) return GBS_E_INVALID_ARG;
  if ((uint64_t)rank0 + (uint64_t)count > host_binom(M, order)) return GBS_E_INVALID_ARG;
  if (flags & GBS_MIXED) return GBS_E_UNSUPPORTED;
  return run_shard(M, sigma, order, rank0, count, flags, corr, cum, stream);
}

gbs_status gbs_cumulant_grad(int32_t M, const double* sigma, int32_t max_order, int32_t flags,
                             const double* grad_corr, const double* grad_cum, double* grad_sigma,
                             void* stream) {
  if (!valid_problem(M, max_order, flags) || !sigma || !grad_sigma) return GBS_E_INVALID_ARG;
  if (flags & GBS_MIXED) return GBS_E_UNSUPPORTED;
  return run_adjoint(M, sigma, max_order, flags, grad_corr, grad_cum, grad_sigma, stream);
}

gbs_status gbs_sample(int32_t M, const double* kappa, int32_t max_order, int64_t nsamples,
                      const double* uniforms, uint8_t* bits, double* prob, double* cond,
                      int64_t batch, int32_t flags, void* stream) {
  if (M < 1 || max_order < 1 || max_order > M || nsamples < 0 || batch < 0) return GBS_E_INVALID_ARG;
  if (flags & ~(GBS_ASYNC | GBS_TIMING)) return GBS_E_INVALID_ARG;
  if (!kappa || (nsamples > 0 && (!uniforms || !bits))) return GBS_E_INVALID_ARG;
  if (max_order != 3 && max_order != 5) return GBS_E_UNSUPPORTED;
  if (M > (max_order == 3 ? 256 : 200)) return GBS_E_INVALID_ARG;
  if (nsamples == 0) return GBS_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  timing_start_call((flags & GBS_TIMING) != 0);
  hipError_t e = timing_begin(s, GBS_STAGE_SAMPLE, max_order);
  if (e == hipSuccess)
    e = run_sampler(M, max_order, kappa, nsamples, uniforms, bits, prob, cond, batch, s);
  if (e == hipSuccess) e = timing_end(s);
  if (e != hipSuccess) return to_status(e);
  if (flags & GBS_ASYNC) return GBS_OK;
  return to_status(hipStreamSynchronize(s));
}

gbs_status gbs_sample_cumulants(int32_t M, int64_t nsamples, const uint8_t* bits,
                                int32_t max_order, double* cum, int32_t flags, void* stream) {
  if (M < 1 || M > 256 || max_order < 1 || max_order > GBS_MAX_ORDER || max_order > M)
    return GBS_E_INVALID_ARG;
  if (nsamples < max_order || nsamples >= (int64_t)1 << 32 || !bits || !cum) return GBS_E_INVALID_ARG;
  if (flags & ~(GBS_ASYNC | GBS_TIMING)) return GBS_E_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  DeviceContext* ctx = current_context(&e);
  if (!ctx) return to_status(e);
  timing_start_call((flags & GBS_TIMING) != 0);
  e = timing_begin(s, GBS_STAGE_ESTIMATE, max_order);
  if (e == hipSuccess) e = run_sample_cumulants(M, nsamples, bits, max_order, ctx->binom, cum, s);
  if (e == hipSuccess) e = timing_end(s);
  if (e != hipSuccess) return to_status(e);
  if (flags & GBS_ASYNC) return GBS_OK;
  return to_status(hipStreamSynchronize(s));
}

gbs_status gbs_pearson(int64_t n, const double* x, const double* y, double* r, int32_t flags,
                       void* stream) {
  if (n < 2 || !x || !y || !r) return GBS_E_INVALID_ARG;
  if (flags & ~(GBS_ASYNC | GBS_TIMING)) return GBS_E_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  timing_start_call((flags & GBS_TIMING) != 0);
  hipError_t e = timing_begin(s, GBS_STAGE_ESTIMATE, 0);
  if (e == hipSuccess) e = run_pearson((uint64_t)n, x, y, r, s);
  if (e == hipSuccess) e = timing_end(s);
  if (e != hipSuccess) return to_status(e);
  if (flags & GBS_ASYNC) return GBS_OK;
  return to_status(hipStreamSynchronize(s));
}

gbs_status gbs_last_error(int32_t* order, int64_t* rank) {
  if (t_err.pending_async && t_err.pending_dev) {
    // an allocation-free call: its status word is still on the device
    DeviceStatus h{};
    if (hipMemcpy(&h, t_err.pending_dev, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
      return GBS_E_DEVICE;
    t_err.order = h.flag ? h.order : 0;
    t_err.rank = h.flag ? h.rank : -1;
  } else if (t_err.pending_async && t_err.host_status) {
    // valid once the stream of the last asynchronous call has completed
    if (t_err.host_status->flag) {
      t_err.order = t_err.host_status->order;
      t_err.rank = t_err.host_status->rank;
    } else {
      t_err.order = 0;
      t_err.rank = -1;
    }
  }
  if (order) *order = t_err.order;
  if (rank) *rank = t_err.rank;
  return t_err.order ? GBS_E_NOT_SPD : GBS_OK;
}

int32_t gbs_last_timings(int32_t capacity, gbs_kernel_time* out) {
  int32_t n = 0;
  for (const auto& r : t_timing) {
    if (n < capacity && out) {
      if (hipEventSynchronize(r.b) != hipSuccess) return -1;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return -1;
      out[n].stage = r.stage;
      out[n].order = r.order;
      out[n].ms = ms;
    }
    ++n;
  }
  return n;
}

const char* gbs_status_string(gbs_status s) {
  switch (s) {
    case GBS_OK: return "ok";
    case GBS_E_INVALID_ARG: return "invalid argument";
    case GBS_E_NOT_SPD: return "a principal block of sigma + I/2 is not positive definite";
    case GBS_E_OUT_OF_MEMORY: return "out of device memory";
    case GBS_E_DEVICE: return "HIP runtime error";
    case GBS_E_UNSUPPORTED: return "unsupported request";
    case GBS_E_SCRATCH_LIMIT:
      return "the problem needs more than the allocation-free entry point's static scratch "
             "(GBS_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

}  // extern "C"

