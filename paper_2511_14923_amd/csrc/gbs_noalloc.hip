// Allocation-free variant of gbs_cumulants: every scratch buffer of the call
// (Q, its diagonal blocks, the mixed-precision operands, the status word, the
// group kernel's tile plans and the lower-order probability and correlator
// tables) is carved out of one file-scope device array, `scratch`, of
// GBS_NOALLOC_SCRATCH_BYTES per device.  The kernels are the ones
// gbs_cumulants runs; only where their scratch lives differs.
//
// Host code never names the array directly except in the one symbol lookup
// below: the array's name is a host-side stand-in, not a device address.  Each
// device's address comes from hipGetSymbolAddress, taken once per device with
// that device current, and every kernel argument, fill and copy uses it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "gbs.h"
#include "gbs_internal.h"

namespace gbs {

namespace {

static __device__ __align__(256) unsigned char scratch[GBS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct NoAllocDevice {
  bool ready = false;
  char* base = nullptr;  // device address of this device's `scratch`
  int cu_count = 0;
  // layout of the last call whose tile plans are in place (M, max_order, mixed), or 0
  uint64_t plan_key = 0;
};

std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[kMaxDevices];

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr size_t kBinBytes = (size_t)kBinRows * kBinLd * sizeof(uint64_t);

// Once per device, with the device current: the array's address on this
// device, its compute-unit count, and the binomial table written into the
// array's first kBinBytes (the table is constant; no call writes there again).
hipError_t setup_device(int dev, NoAllocDevice** out) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoAllocDevice& d = g_noalloc[dev];
  if (!d.ready) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    e = hipDeviceGetAttribute(&d.cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    std::vector<uint64_t> tab((size_t)kBinRows * kBinLd);
    for (int k = 0; k < kBinRows; ++k)
      for (int n = 0; n < kBinLd; ++n) tab[(size_t)k * kBinLd + n] = host_binom(n, k);
    e = hipMemcpy(ptr, tab.data(), kBinBytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    d.base = static_cast<char*>(ptr);
    d.ready = true;
  }
  *out = &d;
  return hipSuccess;
}

// Byte offsets of one call's regions inside the array.
struct NoAllocLayout {
  size_t Qi, Qd, pk, E, st, plan[kMaxOrder + 1], ptab, mtab, total;
  uint32_t ntiles[kMaxOrder + 1];
};

NoAllocLayout layout(int M, int K, int flags, bool corr_given) {
  NoAllocLayout L{};
  const bool mixed = flags & GBS_MIXED;
  const bool rec = !(flags & GBS_ALL_MINORS);
  const size_t nq = 4 * (size_t)M * M;
  size_t off = align256(kBinBytes);
  L.Qi = off; off += align256(nq * sizeof(double));
  L.Qd = off; off += align256(4 * (size_t)M * sizeof(double));
  if (mixed) {
    L.pk = off; off += align256((size_t)M * sizeof(double));
    L.E = off; off += align256(nq * sizeof(float));
  }
  L.st = off; off += align256(sizeof(DeviceStatus));
  for (int d = 3; d <= K && rec; ++d) {
    if (!group_supported(d, M, flags, false)) continue;
    const std::vector<uint64_t>& t = group_plan_host(d, M, mixed);
    L.ntiles[d] = (uint32_t)t.size();
    L.plan[d] = off;
    off += align256(t.size() * sizeof(uint64_t));
  }
  const size_t nlow = K >= 2 ? (size_t)gbs_order_offset(M, K) : 0;
  if (rec) {
    L.ptab = off; off += align256(nlow * sizeof(double));
    if (!corr_given) {
      L.mtab = off; off += align256(nlow * sizeof(double));
    }
  }
  L.total = off;
  return L;
}

}  // namespace

}  // namespace gbs

using namespace gbs;

extern "C" GBS_API gbs_status gbs_cumulants_noalloc(int32_t M, const double* sigma,
                                                    int32_t max_order, int32_t flags,
                                                    double* corr, double* cum, void* stream) {
  if (!valid_problem(M, max_order, flags) || !sigma || !cum) return GBS_E_INVALID_ARG;
  if (flags & GBS_TIMING) return GBS_E_UNSUPPORTED;  // event pairs are library resources
  const NoAllocLayout L = layout(M, max_order, flags, corr != nullptr);
  if (L.total > (size_t)GBS_NOALLOC_SCRATCH_BYTES) return GBS_E_SCRATCH_LIMIT;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return to_status(e);
  if (dev < 0 || dev >= kMaxDevices) return GBS_E_DEVICE;
  NoAllocDevice* D = nullptr;
  e = setup_device(dev, &D);
  if (e != hipSuccess) return to_status(e);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* b = D->base;
  const uint64_t* binom = reinterpret_cast<const uint64_t*>(b);
  double* Qi = reinterpret_cast<double*>(b + L.Qi);
  double* Qd = reinterpret_cast<double*>(b + L.Qd);
  double* pk = (flags & GBS_MIXED) ? reinterpret_cast<double*>(b + L.pk) : nullptr;
  float* E = (flags & GBS_MIXED) ? reinterpret_cast<float*>(b + L.E) : nullptr;
  DeviceStatus* st = reinterpret_cast<DeviceStatus*>(b + L.st);
  const bool rec = !(flags & GBS_ALL_MINORS);

  // tile plans: uploaded when this device's array does not already hold the
  // plans of this layout (calls that overlap on one device race, as documented)
  GroupPlanRef plans[kMaxOrder + 1] = {};
  bool any_plan = false;
  for (int d = 3; d <= max_order; ++d) {
    if (!L.ntiles[d]) continue;
    plans[d].dev = reinterpret_cast<const uint64_t*>(b + L.plan[d]);
    plans[d].ntiles = L.ntiles[d];
    plans[d].grid = group_plan_grid(L.ntiles[d], D->cu_count);
    any_plan = true;
  }
  {
    // the plans' offsets depend on M, max_order and the mixed operands before them
    const uint64_t key =
        any_plan ? ((uint64_t)M << 8 | (uint64_t)max_order << 1 | ((flags & GBS_MIXED) ? 1 : 0))
                 : 0;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (any_plan && D->plan_key != key) {
      for (int d = 3; d <= max_order && e == hipSuccess; ++d) {
        if (!L.ntiles[d]) continue;
        const std::vector<uint64_t>& t = group_plan_host(d, M, (flags & GBS_MIXED) != 0);
        e = hipMemcpyAsync(b + L.plan[d], t.data(), t.size() * sizeof(uint64_t),
                           hipMemcpyHostToDevice, s);
      }
    }
    // a call of another layout overwrites the plan region
    D->plan_key = (e == hipSuccess) ? key : 0;
  }
  if (e != hipSuccess) return to_status(e);

  double* ptab = rec ? reinterpret_cast<double*>(b + L.ptab) : nullptr;
  double* mtab = rec ? (corr ? corr : reinterpret_cast<double*>(b + L.mtab)) : nullptr;
  e = launch_clear_status(st, s);
  if (e == hipSuccess) e = launch_build_q(sigma, M, Qi, s);
  if (e == hipSuccess) e = launch_build_qdiag(Qi, M, Qd, s);
  if (e == hipSuccess && (flags & GBS_MIXED)) e = launch_build_normalised(Qi, M, pk, E, s);
  const double* p_tab[kMaxOrder + 1] = {};
  const double* m_tab[kMaxOrder + 1] = {};
  const double* k_tab[kMaxOrder + 1] = {};
  for (int d = 1; d <= max_order && e == hipSuccess; ++d) {
    const int64_t off = gbs_order_offset(M, d);
    if (rec) {
      double* m_out = (corr || d < max_order) ? mtab + off : nullptr;
      double* p_out = d < max_order ? ptab + off : nullptr;
      e = launch_forward_rec(d, M, flags, Qi, Qd, nullptr, pk, E, binom, p_tab, m_tab, k_tab,
                             m_out, cum + off, p_out, st, s, plans);
      p_tab[d] = ptab + off;
      m_tab[d] = mtab + off;
      k_tab[d] = cum + off;
    } else {
      e = launch_forward(d, M, flags, Qi, nullptr, pk, E, binom, corr ? corr + off : nullptr,
                         cum + off, nullptr, st, s);
    }
  }
  if (e != hipSuccess) return to_status(e);
  return finish_status_device(st, flags, s);
}
