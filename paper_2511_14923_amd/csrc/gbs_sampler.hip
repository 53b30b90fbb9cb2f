// Stage-2 sampler: click patterns drawn bit by bit from the parity cumulants.
//
// The chain rule p(x_n | x_{n-1}, .., x_1) = p(x_n, .., x_1) / p(x_{n-1}, .., x_1)
// with the joint probability expanded in the parity cumulants kappa(S) up to
// order K (Sec. II "The sampling algorithm", Eq. samplecumulant; App. B, Eq.
// probs_corr_cumulants_3): every term of the expansion that involves bit n
// carries chi_n = (-1)^x_n, so
//     p(x_n, .., x_1) = p(n - 1) / 2 + chi_n D_n,
// and D_n (half the bias of Eq. delta_bias) decides the bit: x_n = 1 iff
// u_n < (p(n - 1) / 2 - D_n) / p(n - 1).  The marginals over all but one, two or
// a range of the earlier bits that the expansion needs are approximations kept
// in per-sample tables and updated after every bit:
//   K = 3, single elision (Methods): Eq. methprob for p, Eq. b for the
//          one-elided marginals p1(a, e), Eq. a for the partial marginals
//          p+(b, a);
//   K = 5, double elision (App. C.1): Eq. probade for p, Eq. probpartialade for
//          p+, Eq. probelidedade for p1, Eq. probdoubleelidedade for the
//          two-elided marginals p2(a, e, d).
// Bits are numbered 1..M (bit n is mode n - 1); a marginal whose top variable
// is traced out is the marginal with the next top (p1(a, a) = p(a - 1),
// p2(a, a, d) = p1(a - 1, d)); p+(b, a) = 1 for b < a.
//
// Layout: one lane per sample; a workgroup of 16 (K = 5) or 4 (K = 3) waves owns 64 samples
// and splits every step's sums between its waves (single indices and index
// pairs dealt round-robin, so that the waves get near-equal work), reducing the
// partial D_n through LDS.  The tables of all tops live in
// HBM, one contiguous block per workgroup, entry-major with the workgroup's 64
// samples interleaved (entry t of lane l at t * 64 + l): every table access of
// a wavefront is one contiguous 512-byte read, and the runs of consecutive
// entries that the sums walk are consecutive in memory.  Cumulant indices depend only on loop counters and are the
// same for every lane: they are scalar loads.  Each workgroup's samples are
// independent of every other workgroup's, so one launch runs all M steps with
// workgroup barriers between the phases of a step.
#include <hip/hip_runtime.h>

#include "gbs_internal.h"

namespace gbs {

namespace {

// Waves per workgroup: the double-elision steps have enough work to split
// over 16 waves; the single-elision ones are short, and 4 waves pay fewer
// barriers.
template <int K>
constexpr int samp_waves() { return K == 5 ? 16 : 4; }
// i values per unit of the blocked order-5 sum
constexpr int kIB = 8;

// Entry counts of the tables (1-based bit indices):
//   p(a)         a = 0..M                                  entry a
//   p1(a, e)     1 <= e < a                                (a-1)(a-2)/2 + e - 1
//   p+(b, a)     1 <= a <= b                               b(b-1)/2 + a - 1
//   p2(a, e, d)  1 <= d < e < a                            C(a-1,3) + C(e-1,2) + d - 1
__host__ __device__ constexpr uint32_t c2(uint32_t x) { return x * (x - 1) / 2; }
__host__ __device__ constexpr uint32_t c3(uint32_t x) { return x < 3 ? 0u : x * (x - 1) * (x - 2) / 6; }

struct SampLayout {
  uint32_t n0, n1, npp, n2;  // entries of p, p1, p+, p2
  __host__ __device__ static SampLayout make(int M, int K) {
    SampLayout L;
    L.n0 = (uint32_t)M + 1;
    L.n1 = c2((uint32_t)M) + 1;
    L.npp = c2((uint32_t)M + 1) + 1;
    L.n2 = K == 5 ? c3((uint32_t)M) + 1 : 0;
    return L;
  }
  __host__ __device__ uint32_t entries() const { return n0 + n1 + npp + n2; }
};

struct KapOffsets {
  uint32_t off[6];  // start of the order-d block of the cumulant array
};

// Per-lane view of one sample's tables.
struct Tables {
  double* P0;
  double* P1;
  double* PP;
  double* P2;
  uint64_t ld;
  uint32_t s;
  __device__ __forceinline__ double at(const double* base, uint32_t entry) const {
    return base[(uint64_t)entry * ld + s];
  }
  __device__ __forceinline__ void put(double* base, uint32_t entry, double v) const {
    base[(uint64_t)entry * ld + s] = v;
  }
  __device__ __forceinline__ double p(int a) const { return at(P0, (uint32_t)a); }
  __device__ __forceinline__ double p1(int a, int e) const {
    return e == a ? p(a - 1) : at(P1, c2((uint32_t)a - 1) + (uint32_t)e - 1);
  }
  __device__ __forceinline__ double p2(int a, int e, int d) const {
    return e == a ? p1(a - 1, d) : at(P2, c3((uint32_t)a - 1) + c2((uint32_t)e - 1) + (uint32_t)d - 1);
  }
  __device__ __forceinline__ double pp(int b, int a) const {
    return b < a ? 1.0 : at(PP, c2((uint32_t)b) + (uint32_t)a - 1);
  }
};

// Bits of one sample (M <= 256), one 64-bit word per 64 bits.
struct Bits {
  uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
  __device__ __forceinline__ uint32_t get(int i) const {  // bit i (1-based)
    const int q = (i - 1) >> 6;
    const uint64_t w = q == 0 ? w0 : q == 1 ? w1 : q == 2 ? w2 : w3;
    return (uint32_t)(w >> ((i - 1) & 63)) & 1u;
  }
  __device__ __forceinline__ void set(int i) {
    const int q = (i - 1) >> 6;
    const uint64_t m = 1ull << ((i - 1) & 63);
    if (q == 0) w0 |= m; else if (q == 1) w1 |= m; else if (q == 2) w2 |= m; else w3 |= m;
  }
};

__device__ __forceinline__ double flip(double v, uint32_t parity) { return parity ? -v : v; }

// C(x - 1, k) for the colex rank of 1-based bits
__device__ __forceinline__ uint32_t r1(int x) { return (uint32_t)x - 1; }
__device__ __forceinline__ uint32_t r2(int x) { return c2((uint32_t)x - 1); }
__device__ __forceinline__ uint32_t r3(int x) { return c3((uint32_t)x - 1); }
__device__ __forceinline__ uint32_t r4(int x) {
  const uint32_t y = (uint32_t)x - 1;
  return y < 4 ? 0u : y * (y - 1) * (y - 2) * (y - 3) / 24;
}
__device__ __forceinline__ uint32_t r5(int x) {
  const uint64_t y = (uint64_t)x - 1;
  return y < 5 ? 0u : (uint32_t)(y * (y - 1) * (y - 2) * (y - 3) * (y - 4) / 120);
}

template <int K, int kSampWaves = samp_waves<K>()>
__global__ __launch_bounds__(64 * kSampWaves) void sampler_kernel(
    const double* __restrict__ kap, KapOffsets ko, int M, const double* __restrict__ u,
    uint64_t ldu, int64_t nsamp, double* __restrict__ tab, SampLayout L,
    uint8_t* __restrict__ bits_out, double* __restrict__ prob, double* __restrict__ cond) {
  __shared__ double red[kSampWaves][64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int64_t s = (int64_t)blockIdx.x * 64 + lane;
  const bool live = s < nsamp;
  Tables t;
  t.ld = 64;
  t.s = (uint32_t)lane;  // dead lanes of the last workgroup work on their own columns
  t.P0 = tab + (uint64_t)blockIdx.x * L.entries() * 64;
  t.P1 = t.P0 + (uint64_t)L.n0 * 64;
  t.PP = t.P1 + (uint64_t)L.n1 * 64;
  t.P2 = t.PP + (uint64_t)L.npp * 64;
  if (w == 0) t.put(t.P0, 0, 1.0);
  Bits x;
  __syncthreads();

  for (int n = 1; n <= M; ++n) {
    const uint32_t o2 = ko.off[2] + r2(n), o3 = ko.off[3] + r3(n);
    // ---- phase A: this wave's part of D_n ----
    // order 2 by i, orders 3-5 by the pairs (i > j), each dealt round-robin to
    // the waves (pair (i, j) has index C(i-1, 2) + j - 1)
    double D = 0.0;
    const double pprev = t.p(n - 1);
    if (w == 0) D = 0.5 * kap[ko.off[1] + r1(n)] * pprev;
    for (int i = 1 + w; i < n; i += kSampWaves)
      D += flip(0.25 * kap[o2 + r1(i)] * t.p1(n - 1, i), x.get(i));
    for (int i = 2; i < n; ++i) {
      const uint32_t xi = x.get(i);
      const int j0 = 1 + (w + kSampWaves - (int)(c2((uint32_t)i - 1) % kSampWaves)) % kSampWaves;
      if (j0 >= i) continue;
      const double A = t.pp(n - 1, i + 1);  // the same for every j of this i
      for (int j = j0; j < i; j += kSampWaves) {
        const uint32_t sij = xi ^ x.get(j);
        if constexpr (K == 3) {
          D += flip(0.125 * kap[o3 + r2(i) + r1(j)] * A * t.p1(i - 1, j), sij);
        } else {
          const uint32_t o4 = ko.off[4] + r4(n);
          double v = 0.125 * kap[o3 + r2(i) + r1(j)] * t.p2(n - 1, i, j);
          double a4 = 0.0;
          const uint32_t ok4 = o4 + r3(i) + r2(j);
#pragma unroll 4
          for (int k = 1; k < j; ++k)
            a4 += flip(kap[ok4 + r1(k)] * t.p2(i - 1, j, k), x.get(k));
          v += A * a4 * (1.0 / 16.0);
          D += flip(v, sij);
        }
      }
    }
    if constexpr (K == 5) {
      // order 5: sum_{i>j>k>l} gamma_{ijkln} p+(n-1..i+1) p+(i-1..j+1) p2(j-1; k, l).
      // Units (j, block of kIB consecutive i > j) are dealt round-robin; a unit
      // keeps chi_i p+(n-1..i+1) p+(i-1..j+1) of its i in registers and reads
      // every p2(j-1; k, l) once for all of them.
      const uint32_t o5 = ko.off[5] + r5(n);
      int unit = 0;
      for (int j = 3; j < n - 1; ++j) {
        const int nblk = (n - 1 - j + kIB - 1) / kIB;
        for (int b = 0; b < nblk; ++b, ++unit) {
          if (unit % kSampWaves != w) continue;
          double wv[kIB];
          uint32_t kb[kIB];
#pragma unroll
          for (int ib = 0; ib < kIB; ++ib) {
            const int i = j + 1 + b * kIB + ib;
            const bool in = i < n;
            const int ic = in ? i : n - 1;  // a valid cumulant index; its weight is 0
            kb[ib] = o5 + r4(ic) + r3(j);
            wv[ib] = in ? flip(t.pp(n - 1, i + 1) * t.pp(i - 1, j + 1), x.get(i)) : 0.0;
          }
          double acc = 0.0;
          for (int k = 2; k < j; ++k) {
            double ak = 0.0;
            const uint32_t rk = r2(k);
#pragma unroll 4
            for (int l = 1; l < k; ++l) {
              double kw = 0.0;
#pragma unroll
              for (int ib = 0; ib < kIB; ++ib) kw = fma(kap[kb[ib] + rk + r1(l)], wv[ib], kw);
              ak += flip(kw * t.p2(j - 1, k, l), x.get(l));
            }
            acc += flip(ak, x.get(k));
          }
          D += flip(acc * (1.0 / 32.0), x.get(j));
        }
      }
    }
    red[w][lane] = D;
    __syncthreads();
    D = 0.0;
#pragma unroll
    for (int v = 0; v < kSampWaves; ++v) D += red[v][lane];

    // ---- the bit ----
    const double q = pprev > 0.0 ? (0.5 * pprev - D) / pprev : 0.5;
    const double un = live ? u[(uint64_t)(n - 1) * ldu + s] : 1.0;
    const uint32_t xn = un < q ? 1u : 0u;
    if (xn) x.set(n);
    const double pn = 0.5 * pprev + (xn ? -D : D);
    if (w == 0) {
      t.put(t.P0, (uint32_t)n, pn);
      if (live) {
        bits_out[s * M + (n - 1)] = (uint8_t)xn;
        if (cond) cond[(uint64_t)(n - 1) * ldu + s] = q;
      }
    }

    // ---- phase B: the tables of top n (entries split between the waves) ----
    const double h = 0.5 + flip(0.5 * kap[ko.off[1] + r1(n)], xn);
    if constexpr (K == 3) {
      for (int e = 1 + w; e < n; e += kSampWaves) {
        // terms i < e share the factor p+(n-1..e+1); terms i > e carry p+(n-1..i+1)
        double below = 0.0, above = 0.0;
        for (int i = 1; i < e; ++i)
          below += flip(kap[o2 + r1(i)] * t.p1(e - 1, i), x.get(i) ^ xn);
        for (int i = e + 1; i < n; ++i)
          above += flip(kap[o2 + r1(i)] * t.pp(n - 1, i + 1) * t.p1(i - 1, e), x.get(i) ^ xn);
        const double v = h * t.p1(n - 1, e) + 0.25 * fma(t.pp(n - 1, e + 1), below, above);
        t.put(t.P1, c2((uint32_t)n - 1) + (uint32_t)e - 1, v);
      }
      for (int l = 1 + w; l <= n; l += kSampWaves) {
        double v = h * t.pp(n - 1, l);
        for (int i = l; i < n; ++i)
          v += flip(0.25 * kap[o2 + r1(i)] * t.pp(n - 1, i + 1) * t.pp(i - 1, l), x.get(i) ^ xn);
        t.put(t.PP, c2((uint32_t)n) + (uint32_t)l - 1, v);
      }
    } else {
      for (int l = 1 + w; l <= n; l += kSampWaves) {
        double v = h * t.pp(n - 1, l);
        for (int i = l; i < n; ++i) {
          const double Ai = t.pp(n - 1, i + 1);  // shared by the order-3 and order-4 terms of i
          double ai = 0.25 * kap[o2 + r1(i)] * t.pp(i - 1, l);
          double a3 = 0.0;
          for (int j = l; j < i; ++j)
            a3 += flip(kap[o3 + r2(i) + r1(j)] * t.pp(i - 1, j + 1) * t.pp(j - 1, l), x.get(j));
          ai = fma(0.125, a3, ai);
          v += flip(Ai * ai, x.get(i) ^ xn);
        }
        t.put(t.PP, c2((uint32_t)n) + (uint32_t)l - 1, v);
      }
      for (int e = 1 + w; e < n; e += kSampWaves) {
        // Loops are split where the order of the elided bits changes, so
        // that each runs over consecutive table entries without a branch.
        double v3 = 0.0;
#pragma unroll 4
        for (int i = 1; i < e; ++i)
          v3 += flip(kap[o2 + r1(i)] * t.p2(n - 1, e, i), x.get(i) ^ xn);
#pragma unroll 4
        for (int i = e + 1; i < n; ++i)
          v3 += flip(kap[o2 + r1(i)] * t.p2(n - 1, i, e), x.get(i) ^ xn);
        double v = fma(0.25, v3, h * t.p1(n - 1, e));
        for (int i = 2; i < n; ++i) {
          if (i == e) continue;
          // (a, b, c): i, j, e in decreasing order; a = max(i, e) does not depend on j
          const int a = e > i ? e : i;
          const double A = t.pp(n - 1, a + 1);
          const uint32_t ki = o3 + r2(i);
          double ai = 0.0;
          if (i < e) {
#pragma unroll 4
            for (int j = 1; j < i; ++j) ai += flip(kap[ki + r1(j)] * t.p2(e - 1, i, j), x.get(j));
          } else {
#pragma unroll 4
            for (int j = 1; j < e; ++j) ai += flip(kap[ki + r1(j)] * t.p2(i - 1, e, j), x.get(j));
#pragma unroll 4
            for (int j = e + 1; j < i; ++j) ai += flip(kap[ki + r1(j)] * t.p2(i - 1, j, e), x.get(j));
          }
          v += flip(0.125 * A * ai, x.get(i) ^ xn);
        }
        t.put(t.P1, c2((uint32_t)n - 1) + (uint32_t)e - 1, v);
      }
      for (int e = 2; e < n; ++e) {
        const int d0 = 1 + (w + kSampWaves - (int)(c2((uint32_t)e - 1) % kSampWaves)) % kSampWaves;
        for (int d = d0; d < e; d += kSampWaves) {
          // (a, b, c): i, e, d in decreasing order.  Terms i < e have a = e and
          // share the factor p+(n-1..e+1); terms i > e have (a, b, c) = (i, e, d).
          double below = 0.0, above = 0.0;
#pragma unroll 4
          for (int i = 1; i < d; ++i)
            below += flip(kap[o2 + r1(i)] * t.p2(e - 1, d, i), x.get(i) ^ xn);
#pragma unroll 4
          for (int i = d + 1; i < e; ++i)
            below += flip(kap[o2 + r1(i)] * t.p2(e - 1, i, d), x.get(i) ^ xn);
#pragma unroll 4
          for (int i = e + 1; i < n; ++i)
            above += flip(kap[o2 + r1(i)] * t.pp(n - 1, i + 1) * t.p2(i - 1, e, d), x.get(i) ^ xn);
          const double v = h * t.p2(n - 1, e, d) + 0.25 * fma(t.pp(n - 1, e + 1), below, above);
          t.put(t.P2, c3((uint32_t)n - 1) + c2((uint32_t)e - 1) + (uint32_t)d - 1, v);
        }
      }
    }
    __syncthreads();
  }
  if (w == 0 && live && prob) prob[s] = t.p(M);
}

}  // namespace

// Samples per launch for a table budget of `bytes`.
static int64_t samp_batch(int M, int K, size_t bytes) {
  const uint64_t per = (uint64_t)SampLayout::make(M, K).entries() * sizeof(double);
  return (int64_t)((bytes / per) / 64 * 64);
}

hipError_t run_sampler(int M, int K, const double* kap, int64_t nsamples, const double* u,
                       uint8_t* bits, double* prob, double* cond, int64_t batch, hipStream_t s) {
  if (nsamples == 0) return hipSuccess;
  const SampLayout L = SampLayout::make(M, K);
  KapOffsets ko{};
  ko.off[1] = 0;
  for (int d = 2; d <= 5; ++d)
    ko.off[d] = ko.off[d - 1] + (d - 1 <= K ? (uint32_t)host_binom(M, d - 1) : 0u);
  if (batch <= 0) {
    size_t free_b = 0, total_b = 0;
    hipError_t e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return e;
    batch = samp_batch(M, K, free_b / 4);
  }
  batch = std::max<int64_t>(64, std::min<int64_t>(batch, (nsamples + 63) / 64 * 64));
  // equal launches: a small last launch would run for as long as a full one
  const int64_t nlaunch = (nsamples + batch - 1) / batch;
  batch = ((nsamples + nlaunch - 1) / nlaunch + 63) / 64 * 64;
  const uint64_t ldt = (uint64_t)(batch + 63) / 64 * 64;  // table columns: 64 per workgroup
  void* scratch = nullptr;
  hipError_t e = hipMallocAsync(&scratch, (size_t)L.entries() * ldt * sizeof(double), s);
  if (e != hipSuccess) return e;
  double* tab = static_cast<double*>(scratch);
  for (int64_t s0 = 0; s0 < nsamples && e == hipSuccess; s0 += batch) {
    const int64_t nb = std::min<int64_t>(batch, nsamples - s0);
    const unsigned grid = (unsigned)((nb + 63) / 64);
    if (K == 3)
      hipLaunchKernelGGL(sampler_kernel<3>, dim3(grid), dim3(64 * samp_waves<3>()), 0, s, kap, ko, M,
                         u + s0, (uint64_t)nsamples, nb, tab, L, bits + s0 * M,
                         prob ? prob + s0 : nullptr, cond ? cond + s0 : nullptr);
    else
      hipLaunchKernelGGL(sampler_kernel<5>, dim3(grid), dim3(64 * samp_waves<5>()), 0, s, kap, ko, M,
                         u + s0, (uint64_t)nsamples, nb, tab, L, bits + s0 * M,
                         prob ? prob + s0 : nullptr, cond ? cond + s0 : nullptr);
    e = hipGetLastError();
  }
  hipError_t f = hipFreeAsync(scratch, s);
  return e != hipSuccess ? e : f;
}

}  // namespace gbs
