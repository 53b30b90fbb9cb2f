// Sample-side validation: click cumulants estimated from samples, and the
// Pearson coefficient against the ground truth (App. F, "Click cumulants,
// Pearson and Spearman coefficients"; Eqs. cumulants_test_def and
// pearson_correlation).
//
// The estimator is the unbiased one: every product of |pi| click moments in
// the partition sum of kappa~(S) becomes its average over ordered tuples of
// distinct samples.  Written through the power sums s_B (the number of samples
// in which every mode of B clicked), by Moebius inversion on the partitions of
// the |pi| blocks, it is
//     k(S) = sum_{tau in P(S)} c_N(tau) prod_{B in tau} s_B / N,
// with coefficients c_N(tau) that depend only on the block structure of tau
// and on N (computed on the host).  The work is therefore the power sums of
// every subset of orders <= K:
//   * the samples are packed into one bit column per mode, 64 samples a word;
//   * s_S = sum_w popcount(AND_{k in S} column_k[w]) is a bit-matrix product:
//     S = L + H with L its lowest one or two modes and H the rest; for a fixed
//     c = min(H) the valid L are exactly the subsets of [0, c), so the products
//     run over rectangles (C(c, |L|) x C(M-1-c, |H|-1)) cut into 64 x 64 tiles
//     planned on the host; a tile streams word chunks of its row and column
//     operands through LDS, each thread keeping a 4 x 4 block of counts;
//   * k(S) gathers the power sums of the 2^|S| - 1 subsets of S from the count
//     tables of the lower orders (colex ranks) and evaluates the sum over the
//     partitions of S.
#include <hip/hip_runtime.h>

#include <cstring>
#include <functional>
#include <vector>

#include "gbs_internal.h"

namespace gbs {

namespace {

constexpr int kEstTile = 64;     // rows and columns of a count tile
constexpr int kEstChunk = 32;    // words per LDS chunk
constexpr int kEstThreads = 256;
constexpr int kEstMaxModes = 256;

// ---- pack: bits (N x M bytes, sample-major) -> columns C[k][w] ----
__global__ void pack_columns_kernel(const uint8_t* __restrict__ bits, int64_t N, int M, int64_t W,
                                    uint64_t* __restrict__ cols) {
  // one wavefront per word: lane = sample within the word
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= W) return;
  const int64_t s = w * 64 + lane;
  const bool live = s < N;
  const uint8_t* row = bits + (live ? s : 0) * (int64_t)M;
  for (int k0 = 0; k0 < M; k0 += 64) {
    uint64_t mine = 0;
    const int kn = min(64, M - k0);
    for (int q = 0; q < kn; ++q) {
      const uint64_t m = __ballot(live && row[k0 + q] != 0);
      if (lane == q) mine = m;
    }
    if (lane < kn) cols[(int64_t)(k0 + lane) * W + w] = mine;
  }
}

// ---- order 1: s_k = popcount of column k ----
__global__ void count1_kernel(const uint64_t* __restrict__ cols, int M, int64_t W,
                              uint32_t* __restrict__ out) {
  __shared__ uint32_t part[kEstThreads];
  const int k = blockIdx.x;
  uint32_t c = 0;
  for (int64_t w = threadIdx.x; w < W; w += blockDim.x) c += __popcll(cols[(int64_t)k * W + w]);
  part[threadIdx.x] = c;
  __syncthreads();
  for (int h = blockDim.x / 2; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = part[0];
}

// Tile of the bit-matrix product: rows = L (|L| = DL, all modes < c), columns =
// H = {c} + R (|R| = DH - 1, modes > c).
struct CountTile {
  int32_t c;       // min H
  int32_t r0;      // first row (colex rank of L among the DL-subsets of [0, c))
  int32_t h0;      // first column (colex rank of R among the (DH-1)-subsets of (c, M), shifted by c + 1)
  int32_t pad;
};

__device__ __forceinline__ uint32_t bin_at(const uint32_t* bin, int ld, int k, int n) {
  return bin[k * ld + n];
}

// colex unranking of a small subset (k <= 3) from the binomial table, ascending
template <int K>
__device__ __forceinline__ void unrank_small(uint32_t r, const uint32_t* bin, int ld, int hi,
                                             int (&s)[K > 0 ? K : 1]) {
  for (int j = K; j >= 1; --j) {
    int x = j - 1;
    // largest x < hi with C(x, j) <= r
    int lo = j - 1, h = hi - 1;
    while (lo < h) {
      const int mid = (lo + h + 1) >> 1;
      if (bin_at(bin, ld, j, mid) <= r) lo = mid; else h = mid - 1;
    }
    x = lo;
    s[j - 1] = x;
    r -= bin_at(bin, ld, j, x);
    hi = x;
  }
}

template <int DL, int DH>
__global__ __launch_bounds__(kEstThreads) void count_kernel(const uint64_t* __restrict__ cols,
                                                            int M, int64_t W,
                                                            const CountTile* __restrict__ tiles,
                                                            const uint64_t* __restrict__ binom,
                                                            uint32_t* __restrict__ out) {
  constexpr int D = DL + DH;
  __shared__ uint64_t sa[kEstChunk][kEstTile + 1];
  __shared__ uint64_t sb[kEstChunk][kEstTile + 1];
  __shared__ int rowm[kEstTile][DL];
  __shared__ int colm[kEstTile][DH];
  __shared__ uint32_t bin[(kMaxOrder + 1) * (kEstMaxModes + 1)];
  const int ld = M + 1;
  for (int i = threadIdx.x; i < (D + 1) * ld; i += blockDim.x) {
    const int kk = i / ld, nn = i - kk * ld;
    bin[i] = (uint32_t)binom[kk * kBinLd + nn];
  }
  __syncthreads();
  const CountTile T = tiles[blockIdx.x];
  const int c = T.c;
  const uint32_t nrow = bin_at(bin, ld, DL, c);               // L: DL-subsets of [0, c)
  const uint32_t ncol = bin_at(bin, ld, DH - 1, M - 1 - c);   // R: (DH-1)-subsets of (c, M)
  // modes of this tile's rows and columns
  if (threadIdx.x < kEstTile) {
    const uint32_t r = (uint32_t)T.r0 + threadIdx.x;
    int s[DL];
    unrank_small<DL>(r < nrow ? r : 0, bin, ld, c, s);
    for (int j = 0; j < DL; ++j) rowm[threadIdx.x][j] = s[j];
  } else if (threadIdx.x < 2 * kEstTile) {
    const int t = threadIdx.x - kEstTile;
    const uint32_t h = (uint32_t)T.h0 + t;
    colm[t][0] = c;
    if constexpr (DH > 1) {
      int s[DH - 1];
      unrank_small<DH - 1>(h < ncol ? h : 0, bin, ld, M - 1 - c, s);
      for (int j = 0; j < DH - 1; ++j) colm[t][j + 1] = c + 1 + s[j];
    }
  }
  __syncthreads();
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;  // 4 x 4 block at (4 tr, 4 tc)
  uint32_t acc[4][4] = {};
  for (int64_t w0 = 0; w0 < W; w0 += kEstChunk) {
    // operands of this chunk: AND of the columns of each row / column set
    for (int i = threadIdx.x; i < kEstTile * kEstChunk; i += blockDim.x) {
      const int e = i / kEstChunk, q = i % kEstChunk;
      const int64_t w = w0 + q;
      uint64_t va = 0, vb = 0;
      if (w < W) {
        va = cols[(int64_t)rowm[e][0] * W + w];
        for (int j = 1; j < DL; ++j) va &= cols[(int64_t)rowm[e][j] * W + w];
        vb = cols[(int64_t)colm[e][0] * W + w];
        for (int j = 1; j < DH; ++j) vb &= cols[(int64_t)colm[e][j] * W + w];
      }
      sa[q][e] = va;
      sb[q][e] = vb;
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < kEstChunk; ++q) {
      uint64_t a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = sa[q][4 * tr + i];
        b[i] = sb[q][4 * tc + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += __popcll(a[i] & b[j]);
    }
    __syncthreads();
  }
  // colex rank of S = L + H: rank(L) + sum over H's elements at positions DL..D-1
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t r = (uint32_t)T.r0 + 4 * tr + i;
    if (r >= nrow) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t h = (uint32_t)T.h0 + 4 * tc + j;
      if (h >= ncol) continue;
      uint64_t rank = r;  // rank of L among subsets of [0, c) = its colex rank
#pragma unroll
      for (int q = 0; q < DH; ++q) rank += binom[(DL + q + 1) * kBinLd + colm[4 * tc + j][q]];
      out[rank] = acc[i][j];
    }
  }
}

// ---- k-statistics from the power sums ----
struct KstatCoef {
  int n;                       // partitions of [d]
  float pad;
  double coef[52];             // c_N(tau) for the moment form (prod of s_B / N), partitions
                               // in make_parts order
};

// The partitions of [D] in the order kstat_coefficients lists them (restricted
// growth strings in lexicographic order), each as its block masks in ascending
// order (0 = no block), built at compile time so that the kernel's loop over
// them unrolls with constant indices into the register array of moments.
template <int D>
struct PartTable {
  int n = 0;
  uint32_t blk[52][5] = {};
};

template <int D>
constexpr PartTable<D> make_parts() {
  PartTable<D> T;
  int lab[D] = {};
  for (;;) {
    uint32_t mk[D] = {};
    int nb = 0;
    for (int i = 0; i < D; ++i) {
      mk[lab[i]] |= 1u << i;
      nb = lab[i] + 1 > nb ? lab[i] + 1 : nb;
    }
    for (int i = 1; i < nb; ++i)  // ascending masks (insertion sort)
      for (int j = i; j > 0 && mk[j - 1] > mk[j]; --j) {
        const uint32_t t = mk[j];
        mk[j] = mk[j - 1];
        mk[j - 1] = t;
      }
    for (int b = 0; b < nb; ++b) T.blk[T.n][b] = mk[b];
    ++T.n;
    // next restricted growth string: the last position that can grow
    int i = D - 1;
    for (; i >= 1; --i) {
      int mx = 0;
      for (int j = 0; j < i; ++j) mx = lab[j] > mx ? lab[j] : mx;
      if (lab[i] <= mx) break;
    }
    if (i < 1) break;
    ++lab[i];
    for (int j = i + 1; j < D; ++j) lab[j] = 0;
  }
  return T;
}

template <int D>
__global__ void kstat_kernel(const uint32_t* const* __restrict__ cnt, int M, uint64_t count,
                             const uint64_t* __restrict__ binom, double invN, const KstatCoef* cf,
                             double* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < count; r += stride) {
    int s[D];
    colex_unrank<D>(r, M, binom, kBinLd, s);
    double m[1 << D];
    m[0] = 1.0;
#pragma unroll
    for (int B = 1; B < (1 << D); ++B) {
      uint64_t rk = 0;
      int j = 0;
#pragma unroll
      for (int i = 0; i < D; ++i)
        if (B & (1 << i)) rk += binom[(++j) * kBinLd + s[i]];
      m[B] = (double)cnt[popcount_c((unsigned)B)][rk] * invN;
    }
    constexpr PartTable<D> kParts = make_parts<D>();
    double k = 0.0, comp = 0.0;
#pragma unroll
    for (int t = 0; t < kParts.n; ++t) {
      double v = cf->coef[t];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const uint32_t blk = kParts.blk[t][b];
        if (blk) v *= m[blk];
      }
      const double y = k + v;  // compensated sum
      comp += (fabs(k) >= fabs(v)) ? ((k - y) + v) : ((v - y) + k);
      k = y;
    }
    out[r] = k + comp;
  }
}

// ---- Pearson coefficient: two passes of FP64 block reductions ----
__global__ void sums_kernel(const double* __restrict__ x, const double* __restrict__ y, uint64_t n,
                            const double* __restrict__ mean, double* __restrict__ part) {
  __shared__ double sh[3][kEstThreads];
  const bool centered = mean != nullptr;
  const double mx = centered ? mean[0] : 0.0, my = centered ? mean[1] : 0.0;
  double a = 0.0, b = 0.0, c = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (centered) {
      const double dx = x[i] - mx, dy = y[i] - my;
      a = fma(dx, dy, a);
      b = fma(dx, dx, b);
      c = fma(dy, dy, c);
    } else {
      a += x[i];
      b += y[i];
    }
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = c;
  __syncthreads();
  for (int h = blockDim.x / 2; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void finish_kernel(const double* __restrict__ part, int nblk, uint64_t n, int stage,
                              double* __restrict__ mean, double* __restrict__ r) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = 0; i < nblk; ++i) {  // fixed order: deterministic
    a += part[3 * i];
    b += part[3 * i + 1];
    c += part[3 * i + 2];
  }
  if (stage == 0) {
    mean[0] = a / (double)n;
    mean[1] = b / (double)n;
  } else {
    r[0] = a / sqrt(b * c);
  }
}

// Coefficients c_N(tau) N^|tau| of k(S) = sum_tau coef(tau) prod_{B in tau} (s_B / N).
void kstat_coefficients(int d, double N, KstatCoef* out) {
  // all partitions of [d] as label vectors (restricted growth strings)
  std::vector<std::vector<int>> parts;
  std::vector<int> lab(d, 0);
  std::function<void(int, int)> rec = [&](int i, int nb) {
    if (i == d) {
      parts.push_back(lab);
      return;
    }
    for (int b = 0; b <= nb; ++b) {
      lab[i] = b;
      rec(i + 1, std::max(nb, b + 1));
    }
  };
  rec(0, 0);
  auto nblocks = [](const std::vector<int>& l) {
    int m = 0;
    for (int v : l) m = std::max(m, v + 1);
    return m;
  };
  auto masks = [&](const std::vector<int>& l) {
    std::vector<uint32_t> mk(nblocks(l), 0u);
    for (int i = 0; i < (int)l.size(); ++i) mk[l[i]] |= 1u << i;
    std::sort(mk.begin(), mk.end());
    return mk;
  };
  std::vector<double> coef(parts.size(), 0.0);
  std::vector<std::vector<uint32_t>> pm(parts.size());
  for (size_t t = 0; t < parts.size(); ++t) pm[t] = masks(parts[t]);
  for (size_t pi = 0; pi < parts.size(); ++pi) {
    const int p = nblocks(parts[pi]);
    // w(pi) / (N)_p
    double fall = 1.0;
    for (int i = 0; i < p; ++i) fall *= (N - i);
    double fact = 1.0;
    for (int i = 2; i < p; ++i) fact *= i;
    const double w = ((p - 1) % 2 ? -fact : fact) / fall;
    // coarsenings sigma of the p blocks: partitions of [p]
    std::vector<int> sl(p, 0);
    std::function<void(int, int)> rs = [&](int i, int nb) {
      if (i == p) {
        // tau = union of pi's blocks by sigma's labels; Moebius factor
        std::vector<int> tl(d);
        for (int e = 0; e < d; ++e) tl[e] = sl[parts[pi][e]];
        std::vector<int> cnt(nb, 0);
        for (int j = 0; j < p; ++j) cnt[sl[j]]++;
        double mob = 1.0;
        for (int C = 0; C < nb; ++C) {
          double f = 1.0;
          for (int i2 = 2; i2 < cnt[C]; ++i2) f *= i2;
          mob *= ((cnt[C] - 1) % 2 ? -f : f);
        }
        const std::vector<uint32_t> tm = masks(tl);
        for (size_t t = 0; t < parts.size(); ++t)
          if (pm[t] == tm) {
            coef[t] += w * mob;
            break;
          }
        return;
      }
      for (int b = 0; b <= nb; ++b) {
        sl[i] = b;
        rs(i + 1, std::max(nb, b + 1));
      }
    };
    rs(0, 0);
  }
  out->n = (int)parts.size();
  for (size_t t = 0; t < parts.size(); ++t) {
    double Np = 1.0;
    for (size_t b = 0; b < pm[t].size(); ++b) Np *= N;
    out->coef[t] = coef[t] * Np;
  }
}

template <int DL, int DH>
std::vector<CountTile> plan_count_tiles(int M) {
  std::vector<CountTile> tiles;
  for (int c = DL; c + (DH - 1) < M; ++c) {
    const uint64_t nrow = host_binom(c, DL), ncol = host_binom(M - 1 - c, DH - 1);
    for (uint64_t r = 0; r < nrow; r += kEstTile)
      for (uint64_t h = 0; h < ncol; h += kEstTile) tiles.push_back({c, (int32_t)r, (int32_t)h, 0});
  }
  return tiles;
}

template <int DL, int DH>
hipError_t launch_counts(const uint64_t* cols, int M, int64_t W, const uint64_t* binom,
                         uint32_t* out, CountTile* tiles_dev, size_t ntiles, hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL((count_kernel<DL, DH>), dim3((unsigned)ntiles), dim3(kEstThreads), 0, s, cols,
                     M, W, tiles_dev, binom, out);
  return hipGetLastError();
}

}  // namespace

// Power sums and k-statistics of orders 1..K from nsamples samples.
hipError_t run_sample_cumulants(int M, int64_t N, const uint8_t* bits, int K,
                                const uint64_t* binom, double* out, hipStream_t s) {
  const int64_t W = (N + 63) / 64;
  // scratch: columns, per-order counts, tile lists, coefficient blocks, count pointers
  std::vector<std::vector<CountTile>> plans(K + 1);
  if (K >= 2) plans[2] = plan_count_tiles<1, 1>(M);
  if (K >= 3) plans[3] = plan_count_tiles<1, 2>(M);
  if (K >= 4) plans[4] = plan_count_tiles<2, 2>(M);
  if (K >= 5) plans[5] = plan_count_tiles<2, 3>(M);
  size_t off = 0;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t oc = off; off += al((size_t)M * W * sizeof(uint64_t));
  size_t ocnt[kMaxOrder + 1] = {};
  for (int d = 1; d <= K; ++d) { ocnt[d] = off; off += al(host_binom(M, d) * sizeof(uint32_t)); }
  size_t otile[kMaxOrder + 1] = {};
  for (int d = 2; d <= K; ++d) { otile[d] = off; off += al(plans[d].size() * sizeof(CountTile)); }
  const size_t ocoef = off; off += al((size_t)(K + 1) * sizeof(KstatCoef));
  const size_t optr = off; off += al((kMaxOrder + 1) * sizeof(uint32_t*));
  void* scratch = nullptr;
  hipError_t e = hipMallocAsync(&scratch, off, s);
  if (e != hipSuccess) return e;
  char* b = static_cast<char*>(scratch);
  uint64_t* cols = reinterpret_cast<uint64_t*>(b + oc);
  // host-side staging: tile lists, coefficients, count pointers (one pinned block)
  size_t hbytes = 0;
  for (int d = 2; d <= K; ++d) hbytes += plans[d].size() * sizeof(CountTile);
  hbytes += (K + 1) * sizeof(KstatCoef) + (kMaxOrder + 1) * sizeof(uint32_t*);
  std::vector<char> host(hbytes);
  size_t ho = 0;
  std::vector<size_t> htile(K + 1, 0);
  for (int d = 2; d <= K; ++d) {
    htile[d] = ho;
    memcpy(host.data() + ho, plans[d].data(), plans[d].size() * sizeof(CountTile));
    ho += plans[d].size() * sizeof(CountTile);
  }
  const size_t hcoef = ho;
  for (int d = 1; d <= K; ++d)
    kstat_coefficients(d, (double)N, reinterpret_cast<KstatCoef*>(host.data() + hcoef) + d);
  ho += (K + 1) * sizeof(KstatCoef);
  const size_t hptr = ho;
  uint32_t** cp = reinterpret_cast<uint32_t**>(host.data() + hptr);
  for (int d = 0; d <= kMaxOrder; ++d) cp[d] = d >= 1 && d <= K ? reinterpret_cast<uint32_t*>(b + ocnt[d]) : nullptr;
  for (int d = 2; d <= K && e == hipSuccess; ++d)
    e = hipMemcpyAsync(b + otile[d], host.data() + htile[d], plans[d].size() * sizeof(CountTile),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b + ocoef, host.data() + hcoef, (K + 1) * sizeof(KstatCoef),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b + optr, host.data() + hptr, (kMaxOrder + 1) * sizeof(uint32_t*),
                       hipMemcpyHostToDevice, s);
  // the staging buffer must outlive the copies
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && W > 0) {
    const int wpb = 4;  // words (wavefronts) per block
    hipLaunchKernelGGL(pack_columns_kernel, dim3((unsigned)((W + wpb - 1) / wpb)), dim3(64 * wpb), 0,
                       s, bits, N, M, W, cols);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(count1_kernel, dim3(M), dim3(kEstThreads), 0, s, cols, M, W,
                       reinterpret_cast<uint32_t*>(b + ocnt[1]));
    e = hipGetLastError();
  }
  auto tl = [&](int d) { return reinterpret_cast<CountTile*>(b + otile[d]); };
  auto co = [&](int d) { return reinterpret_cast<uint32_t*>(b + ocnt[d]); };
  if (e == hipSuccess && K >= 2) e = launch_counts<1, 1>(cols, M, W, binom, co(2), tl(2), plans[2].size(), s);
  if (e == hipSuccess && K >= 3) e = launch_counts<1, 2>(cols, M, W, binom, co(3), tl(3), plans[3].size(), s);
  if (e == hipSuccess && K >= 4) e = launch_counts<2, 2>(cols, M, W, binom, co(4), tl(4), plans[4].size(), s);
  if (e == hipSuccess && K >= 5) e = launch_counts<2, 3>(cols, M, W, binom, co(5), tl(5), plans[5].size(), s);
  const uint32_t* const* cptr = reinterpret_cast<const uint32_t* const*>(b + optr);
  const KstatCoef* cf = reinterpret_cast<const KstatCoef*>(b + ocoef);
  const double invN = 1.0 / (double)N;
  for (int d = 1; d <= K && e == hipSuccess; ++d) {
    const uint64_t count = host_binom(M, d);
    const unsigned grid = (unsigned)std::min<uint64_t>((count + 255) / 256, 1u << 20);
    double* o = out + gbs_order_offset(M, d);
    switch (d) {
      case 1: hipLaunchKernelGGL(kstat_kernel<1>, dim3(grid), dim3(256), 0, s, cptr, M, count, binom, invN, cf + 1, o); break;
      case 2: hipLaunchKernelGGL(kstat_kernel<2>, dim3(grid), dim3(256), 0, s, cptr, M, count, binom, invN, cf + 2, o); break;
      case 3: hipLaunchKernelGGL(kstat_kernel<3>, dim3(grid), dim3(256), 0, s, cptr, M, count, binom, invN, cf + 3, o); break;
      case 4: hipLaunchKernelGGL(kstat_kernel<4>, dim3(grid), dim3(256), 0, s, cptr, M, count, binom, invN, cf + 4, o); break;
      default: hipLaunchKernelGGL(kstat_kernel<5>, dim3(grid), dim3(256), 0, s, cptr, M, count, binom, invN, cf + 5, o); break;
    }
    e = hipGetLastError();
  }
  hipError_t f = hipFreeAsync(scratch, s);
  return e != hipSuccess ? e : f;
}

hipError_t run_pearson(uint64_t n, const double* x, const double* y, double* r, hipStream_t s) {
  const int nblk = (int)std::min<uint64_t>((n + kEstThreads - 1) / kEstThreads, 1024);
  void* scratch = nullptr;
  hipError_t e = hipMallocAsync(&scratch, (size_t)(3 * nblk + 2) * sizeof(double), s);
  if (e != hipSuccess) return e;
  double* part = static_cast<double*>(scratch);
  double* mean = part + 3 * nblk;
  hipLaunchKernelGGL(sums_kernel, dim3(nblk), dim3(kEstThreads), 0, s, x, y, n, (const double*)nullptr, part);
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, part, nblk, n, 0, mean, r);
  hipLaunchKernelGGL(sums_kernel, dim3(nblk), dim3(kEstThreads), 0, s, x, y, n, (const double*)mean, part);
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, part, nblk, n, 1, mean, r);
  e = hipGetLastError();
  hipError_t f = hipFreeAsync(scratch, s);
  return e != hipSuccess ? e : f;
}

}  // namespace gbs
