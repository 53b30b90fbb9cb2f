// Group-tiled forward kernel (FP64, orders 3..5).
//
// For S = {a} + B, B = {b_0 < b_1 < .. < e}, write B = {b_0} + T with
// T = P + {e}, P = B \ {b_0, e}.  The subsets that share T form a group: the
// pairs (a, b_0) with a < b_0 < min T, at consecutive colex ranks.  Q_S is
// factored in the block order [P, b_0, e, a], so the work splits by what it
// depends on:
//   (T)         the Cholesky rows of P and of e against P;
//   (T, a)      y_P = L_P^{-1} Q_{P,a}, the Schur complement Q_aa - y_P^T y_P of
//               Q_P in Q_{P + a}, t_e = Q_{e,a} - L_{e,P} y_P, and p({a} + U) for
//               every U subset of T;
//   (B)         the Cholesky rows of b_0 and e (against P and b_0);
//   (a, B)      y_{b_0}, y_e: two block rows of the forward substitution.
// With det(Q_{U + a}) = det(Q_U) det(Q_aa - y_U^T y_U) for every leading set U
// of the order (App. D.1, Eq. vacuum_gaussian_prob: p(T) = det(Q_T)^(-1/2)),
// the subset itself needs only p(B' + a) = p(S \ e) and p(S), from two 2x2
// determinants, plus the p({a} + U) with b_0 in U that are not leading sets,
// read from the tables of the lower orders.  Correlators and cumulants follow
// as in the tile kernel (gbs_forward_tile.hip): subset zeta transforms for
// nu(W) and nu(W + e), m({a} + W) = m(W) - nu(W) (Eq. corre_cov_main split by
// whether T contains a), and the fixed-element recursion on e for the
// cumulants (Eq. cumulant_corr_main grouped by the block containing e; App. B,
// Eq. correlators_expanded_2).
//
// Displaced states (first moments mu, Eq. vacuum_gaussian_prob): the same
// factorisation also gives z = L^{-1} mu in the order [P, b_0, e] (z_P and
// z_e(T) once per group, z_{b_0} and z_e(B) once per B), and for a leading set
// U of the order the quadratic form splits as
//   mu_{U+a}^T Q_{U+a}^{-1} mu_{U+a} = |z_U|^2 + r^T (Q_aa - y_U^T y_U)^{-1} r,
//   r = mu_a - y_U^T z_U,
// so every probability computed here gains exp(-q/2) from two more 2-vectors
// per block row; |z|^2 of the T, B' and B parts is folded into the per-group
// and per-B probabilities.
//
// A tile is a run of consecutive B's (at most GL::kB) whose groups need at
// most rmax (T, a) records; the host plans the tiles once per (M, d).  Per
// tile: phase 1 builds the per-B records (lane = B, one part per wave) and the
// group list; phase 1b builds the (T, a) records (one per thread); phase 2
// takes one subset per lane, consecutive ranks across a wavefront.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "gbs_internal.h"
#include "gbs_subset.h"

namespace gbs {

namespace {

// B's and groups per tile at most (per precision: GroupLayout::kB, kG) bound
// these; the walk and descriptor limits below cover every layout
constexpr int kGroupBMax = 64;
constexpr int kGroupGMax = 16;
constexpr int kGroupThreads = 256;  // threads per workgroup (4 waves)
constexpr int kGroupRmax = 148;     // (T, a) records per tile at most (M - d + 1 needed)
// Workgroups per CU in one single-instance launch; beyond that a workgroup takes
// every grid-th tile (order 5 at M = 144: 7.31 -> 6.83 ms against one workgroup
// per tile, ~430,000 tiles).
constexpr uint32_t kGroupWgPerCU = 192;
// Tile descriptor (64 bits): the colex rank of the tile's first B (29 bits),
// the number of B's (7 bits), and the modes of that B's T (8 bits each, at most
// three), so that each lane finds its B by walking the groups from the first
// one instead of unranking.  The group kernel runs only where every rank fits
// in 29 bits and M <= 152 (group_supported).
constexpr int kDescNbShift = 29;
constexpr int kDescNbBits = 7;
constexpr int kDescTShift = kDescNbShift + kDescNbBits;
constexpr uint64_t kDescBetaMask = (1ull << kDescNbShift) - 1;
constexpr uint64_t kDescNbMask = (1ull << kDescNbBits) - 1;
static_assert(kGroupBMax <= (int)kDescNbMask, "the B count of a tile must fit its descriptor field");
static_assert(kDescTShift + 3 * 8 <= 64, "the descriptor holds three 8-bit modes");
// steps of a lane's walk at most: the groups of a tile (kGroupGMax) and the empty
// T (min T = 0) between them, at most two per group
constexpr int kWalkMax = 3 * kGroupGMax + 4;

template <int NB, bool DISP, bool MIXED = false>
struct GroupLayout {
  // B's and groups per tile: as many as let three workgroups (order 5) or four
  // (orders 3 and 4, whose records are smaller) share a compute unit's 160 KB
  // of LDS at M = 144 (order 5 at M = 144: FP64 40 -> 52 B's 5.57 -> 5.27 ms;
  // mixed 40 -> 64 B's 5.22 -> 4.70 ms); the smaller FP32 factor rows and
  // records of the mixed form leave room for a full wavefront of B's.  kG is
  // a power of two (the record builder's binary search).
  static constexpr bool kWide = MIXED || NB < 4;
  static constexpr int kB = DISP ? 48 : (kWide ? 64 : 54);
  static constexpr int kG = (kWide && !DISP) ? 16 : 8;
  static_assert(kB <= kGroupBMax && kG <= kGroupGMax && (kG & (kG - 1)) == 0, "tile shape");
  static constexpr int NPm = NB - 2;       // |P|
  static constexpr int NT = NB - 1;        // |T|
  static constexpr int NTS = 1 << NT;      // subsets of T
  static constexpr int N = 2 * NB;         // rows of Q_B
  static constexpr int NU = 1 << NB;       // subsets of B (bit 0: b_0, bit i: b_i)
  static constexpr int NP = 1 << (NB - 1); // subsets of B' = B \ {e}
  static constexpr int FULL = NU - 1;
  static constexpr int FULLP = NP - 1;
  // Factor entries (rows of Cholesky factors, forward substitutions, Schur
  // complements) are FP64, or FP32 deviations from the identity of the
  // normalised Q in the mixed form; probabilities, correlators and cumulants
  // are FP64 in both.
  // per-B record: the factor rows first (in factor-entry units), then doubles
  static constexpr int dLb = 0;                 // b_0 rows: [r][k < 2|P|], then 1/L, L, 1/L of the b_0 block
  static constexpr int nLb = 4 * NPm + 3;
  static constexpr int dLe = dLb + nLb;         // e rows against b_0 ([r][2]), then the e block
  static constexpr int nLe = 7;
  static constexpr int nL = nLb + nLe;
  static constexpr int dP = MIXED ? (nL + 1) / 2 : nL;  // p(B'), p(B) (displaced: with exp(-|z|^2 / 2))
  // coefficients c_B(V), V subset of B, of k(S) = sum_V c_B(V) p({a} + V); 16-byte aligned pairs
  static constexpr int dC = (dP + 2 + 1) & ~1;
  static constexpr int dMB = dC + NU;           // m(B)
  static constexpr int dZ = dMB + 1;            // displaced: z_{b_0} [2], z_e(B) [2]
  static constexpr int nD = dZ + (DISP ? 4 : 0);
  static constexpr int wOff = nD * 8;          // byte offset of the 32-bit words
  // per-B record, 32-bit words
  static constexpr int wStart = 0;              // first rank of the B-block, tile relative
  static constexpr int wRow = 1;                // byte offset of row 2 b_0 of Q (of E, mixed)
  static constexpr int wRbase = 2;              // (T, a) record of a = 0 for this B's group
  static constexpr int wOP = 3;                 // rank parts (less start) of p({a} + U), b_0 in U
  static constexpr int nOP = NP - 2;            // all U containing b_0 except B' and B
  static constexpr int wG = wOP + nOP;          // this B's group (displaced states)
  static constexpr int nW = wG + (DISP ? 1 : 0);

  // record stride: whole 16-byte units (16-byte LDS reads in phase 2), an odd
  // number of them, so that the lane-per-B accesses of the setup phases (lane
  // c at c * bytes) spread over the 32 LDS banks; an even number at least
  // doubles their bank conflicts (order 5 FP64: 22 units, 16-way)
  static constexpr int bytes0 = (wOff + nW * 4 + 15) & ~15;
  static constexpr int bytes = ((bytes0 / 16) % 2 == 0) ? bytes0 + 16 : bytes0;
  // (T, a) record in 16-byte units, unit q of record i at [q][i], so that
  // consecutive records (consecutive a across a wavefront) fall in consecutive
  // LDS banks.  FP64: y_P row k is unit uY + k (two columns); mixed: unit
  // uY + k/2 holds rows k, k + 1.
  static constexpr int I0 = 2 * NPm;            // rows of P
  static constexpr int uY = 0;                  // y_P [k < 2|P|][2]
  static constexpr int uT = MIXED ? I0 / 2 : I0;        // t_e [r][2]
  static constexpr int uS = uT + (MIXED ? 1 : 2);       // Schur complement of Q_P in Q_{P + a}: s00, s10, s11
  // FP64: s11 and nu_T share the second unit of uS; mixed: p_a = det(Q_aa)^(-1/2)
  // and nu_T (FP64) share uPK.  nu_T = sum_{U subset T} s(U) p({a} + U).
  static constexpr int uPK = uS + (MIXED ? 1 : 2);
  static constexpr int uPT = uPK + (MIXED ? 1 : 0);     // p({a} + U), U subset of T (FP64)
  static constexpr int rUnits = uPT + NTS / 2;
  static constexpr int rbytes = rUnits * 16;    // per record
  // per-group record (Cholesky of Q_T in the order P, e), doubles
  static constexpr int gP = 0;                  // L_P: tri(i, j), 1/L_ii on the diagonal
  static constexpr int gE = gP + tri_size(I0);  // e rows against P: [r][k < I0]
  static constexpr int gS = gE + 2 * I0;        // Q_ee - L_eP L_eP^T: s00, s10, s11
  static constexpr int gEd = gS + 3;            // e block of Q_T: 1/L, L, 1/L
  static constexpr int gpP = gEd + 3;           // p(P) (displaced: with exp(-|z_P|^2 / 2); mixed: P_P)
  static constexpr int gpT = gpP + 1;           // p(T) (displaced: with exp(-|z_T|^2 / 2); mixed: P_T)
  static constexpr int gZ = gpT + 1;            // displaced: z_P [2|P|], z_e(T) [2]
  // mixed: per block j of P, rho and P = prod p_k of the leading modes P_0..P_j,
  // then rho_T (P_T is gpT)
  static constexpr int gRho = gpT + 1;
  static constexpr int gPP = gRho + NPm;
  static constexpr int gRT = gPP + NPm;
  static constexpr int gN = ((MIXED ? gRT + 1 : gZ + (DISP ? I0 + 2 : 0)) + 1) & ~1;
  static constexpr int gbytes = gN * 8;
};

// Index among the per-subset table reads of a B-subset U that contains b_0.
template <int NB>
__host__ __device__ constexpr int gop_index(int u) {
  int n = 0;
  for (int v = 0; v < u; ++v)
    n += ((v & 1) && v != (1 << (NB - 1)) - 1 && v != (1 << NB) - 1) ? 1 : 0;
  return n;
}

// Colex successor of the NT-subset t of [0, M) (unchanged for the last one).
template <int NT>
__device__ __forceinline__ void colex_next(int (&t)[NT], int M) {
  bool done = false;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const int lim = (i + 1 < NT) ? t[i + 1] : M;
    if (!done && t[i] + 1 < lim) {
      ++t[i];
#pragma unroll
      for (int j = 0; j < i; ++j) t[j] = j;
      done = true;
    }
  }
}

// Mixed form (FP32 deviations from the identity of the normalised Q):
// det(I + S) - 1 of a 2x2 deviation S, without forming 1 + s_ii
__device__ __forceinline__ float det_dev(float s00, float s10, float s11) {
  return s00 + s11 + fmaf(s00, s11, -s10 * s10);
}
// (1 + delta)^(-1/2) - 1 = -delta y^2 / (1 + y), y = (1 + delta)^(-1/2)
__device__ __forceinline__ float inv_sqrt_dev(float delta, float y) {
  return -delta * y * y * __builtin_amdgcn_rcpf(1.0f + y);
}
// (1 + r)(1 + e) - 1
__device__ __forceinline__ float dev_compose(float r, float e) { return r + fmaf(r, e, e); }
// Two floats at a 32-bit byte offset (8-byte aligned) from a uniform base.
__device__ __forceinline__ float2 load_f2_at(const float* __restrict__ base, uint32_t byte_off) {
  return *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Leading sets of T in the order [P, e]: empty, {P_0}, .., P, T.
template <int NT>
__host__ __device__ constexpr bool t_leading(int t) {
  return t == (1 << NT) - 1 || ((t & (t + 1)) == 0 && t < (1 << (NT - 1)));
}

}  // namespace

// One instance: one workgroup per tile of the plan.  FP64 reads Q (and the
// interleaved first moments mi of a displaced state); the mixed form reads the
// single-mode vacuum probabilities pk and the FP32 normalised couplings E.
template <int D, int CONV, bool WANT_CUM, bool DISP, bool MIXED>
__global__ __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu(1, 3))) void forward_group_kernel(
    const double* __restrict__ Qi, const double* __restrict__ Qd,
    const double* __restrict__ mi, const double* __restrict__ pk, const float* __restrict__ E,
    int M,
    const uint64_t* __restrict__ plan, uint32_t ntiles, const uint64_t* __restrict__ binom,
    OrderTables tab, double* __restrict__ m_out, double* __restrict__ k_out,
    double* __restrict__ p_out, DeviceStatus* __restrict__ st, int nwin_max) {
  constexpr int rmax = kGroupRmax;
  constexpr int NB = D - 1;
  using GL = GroupLayout<NB, DISP, MIXED>;
  constexpr int NPm = GL::NPm;
  constexpr int NT = GL::NT;
  constexpr int NTS = GL::NTS;
  constexpr int N = GL::N;
  constexpr int NP = GL::NP;
  constexpr int FULL = GL::FULL;
  constexpr int FULLP = GL::FULLP;
  constexpr int EBIT = 1 << (NB - 1);

  extern __shared__ __align__(16) unsigned char smem[];
  // [B records][(T, a) records][group records][binomials][bitmap][first run per window]
  unsigned char* brec = smem;
  unsigned char* rrec = smem + GL::kB * GL::bytes;
  double* grec = reinterpret_cast<double*>(rrec + (size_t)rmax * GL::rbytes);
  uint32_t* bin = reinterpret_cast<uint32_t*>(grec + GL::kG * GL::gN);
  const int ld = M + 1;
  uint64_t* bits = reinterpret_cast<uint64_t*>(bin + (((D + 1) * ld + 1) & ~1));
  unsigned char* first = reinterpret_cast<unsigned char*>(bits + nwin_max);
  __shared__ uint32_t s_ntile, s_r0;

  for (int i = threadIdx.x; i < (D + 1) * ld; i += blockDim.x) {
    const int kk = i / ld, nn = i - kk * ld;
    bin[i] = (uint32_t)binom[kk * kBinLd + nn];
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint32_t ldq8 = 2u * (uint32_t)M * (uint32_t)sizeof(double);
  const double* Qodd = MIXED ? nullptr : Qi + 2 * (size_t)M;  // odd rows (p quadratures)
  const uint32_t lde4 = 2u * (uint32_t)M * (uint32_t)sizeof(float);
  const float* Eodd = MIXED ? E + 2 * (size_t)M : nullptr;

  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t desc = plan[tile];
#include "gbs_group_tile.inc"
  }
}

// Many instances: a fixed grid claims (instance, tile) items of one order from
// a device work list with one atomic counter until the list is exhausted.  The
// binomial table is filled once for the largest M (C(n, k) does not depend on
// M); every workgroup leaves the loop when the counter passes the list's end.
template <int D, int CONV, bool WANT_CUM, bool MIXED>
__global__ __launch_bounds__(kGroupThreads) void forward_group_batched_kernel(
    const GroupBatchInstance* __restrict__ inst, const GroupBatchItem* __restrict__ items,
    uint32_t n_items, unsigned* __restrict__ counter, const uint64_t* __restrict__ binom,
    int max_M, DeviceStatus* __restrict__ st, int nwin_max) {
  constexpr bool DISP = false;
  constexpr int rmax = kGroupRmax;
  constexpr int NB = D - 1;
  using GL = GroupLayout<NB, DISP, MIXED>;
  constexpr int NPm = GL::NPm;
  constexpr int NT = GL::NT;
  constexpr int NTS = GL::NTS;
  constexpr int N = GL::N;
  constexpr int NP = GL::NP;
  constexpr int FULL = GL::FULL;
  constexpr int FULLP = GL::FULLP;
  constexpr int EBIT = 1 << (NB - 1);

  extern __shared__ __align__(16) unsigned char smem[];
  // [B records][(T, a) records][group records][binomials][bitmap][first run per window]
  unsigned char* brec = smem;
  unsigned char* rrec = smem + GL::kB * GL::bytes;
  double* grec = reinterpret_cast<double*>(rrec + (size_t)rmax * GL::rbytes);
  uint32_t* bin = reinterpret_cast<uint32_t*>(grec + GL::kG * GL::gN);
  const int ld = max_M + 1;
  uint64_t* bits = reinterpret_cast<uint64_t*>(bin + (((D + 1) * ld + 1) & ~1));
  unsigned char* first = reinterpret_cast<unsigned char*>(bits + nwin_max);
  __shared__ uint32_t s_ntile, s_r0;
  __shared__ uint32_t s_item;

  for (int i = threadIdx.x; i < (D + 1) * ld; i += blockDim.x) {
    const int kk = i / ld, nn = i - kk * ld;
    bin[i] = (uint32_t)binom[kk * kBinLd + nn];
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const double* const mi = nullptr;

  for (;;) {
    __syncthreads();  // every reader of the previous item index is done
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= n_items) break;  // uniform: every workgroup reaches this once the list is drained
    const GroupBatchItem w = items[it];
    const GroupBatchInstance& I = inst[__builtin_amdgcn_readfirstlane(w.inst)];
    const double* __restrict__ Qi = I.Qi;
    const double* __restrict__ Qd = I.Qd;
    const int M = I.M;
    const OrderTables& tab = I.tab;
    double* __restrict__ m_out = I.m_out;
    double* __restrict__ k_out = I.k_out;
    double* __restrict__ p_out = I.p_out;
    const double* __restrict__ pk = I.pk;
    const float* __restrict__ E = I.E;
    const uint32_t ldq8 = 2u * (uint32_t)M * (uint32_t)sizeof(double);
    const double* Qodd = MIXED ? nullptr : Qi + 2 * (size_t)M;  // odd rows (p quadratures)
    const uint32_t lde4 = 2u * (uint32_t)M * (uint32_t)sizeof(float);
    const float* Eodd = MIXED ? E + 2 * (size_t)M : nullptr;
    const uint64_t desc = w.desc;
#include "gbs_group_tile.inc"
  }
}


// ---------------- host: tile plans ----------------

namespace {

// Tiles of consecutive B's (colex order of the (d-1)-subsets) such that each
// holds at most kB B's of at most kG groups, which need at most rmax
// (T, a) records.  A group is all B = {b_0} + T with b_0 < min T; within a tile
// it needs the records a < (largest b_0 of the group in the tile).
std::vector<uint64_t> plan_tiles(int M, int NB, int rmax, int kB, int kG) {
  std::vector<uint64_t> tiles;
  uint32_t beta = 0, tstart = 0;
  uint64_t tfirst = 0;  // modes of the T of the tile's first B, 8 bits each
  int nB = 0, rec = 0, ng = 0;
  auto close = [&]() {
    if (nB > 0)  // never an empty tile; every field within its width
      tiles.push_back(((uint64_t)tstart & kDescBetaMask) |
                      (((uint64_t)nB & kDescNbMask) << kDescNbShift) | (tfirst << kDescTShift));
    nB = 0;
    rec = 0;
    ng = 0;
  };
  // T runs over the (NB-1)-subsets of [0, M) in colex order; its group has min T B's
  const int nt = NB - 1;
  std::vector<int> t(nt);
  for (int i = 0; i < nt; ++i) t[i] = i;
  while (true) {
    const int gsize = t[0];  // b_0 = 0 .. t_0 - 1
    int k = 0;
    while (k < gsize) {
      int n = std::min(gsize - k, kB - nB);
      int need = k + n - 1;  // records a < max b_0 = k + n - 1
      if (rec + need > rmax || ng == kG) {
        close();
        n = std::min(gsize - k, kB);
        need = k + n - 1;
      }
      if (nB == 0) {  // the tile starts at B = {k} + T, colex rank beta
        tstart = beta;
        tfirst = 0;
        for (int j = 0; j < nt; ++j) tfirst |= (uint64_t)t[j] << (8 * j);
      }
      nB += n;
      rec += need;
      ++ng;
      beta += (uint32_t)n;
      k += n;
      if (nB == kB) close();
    }
    // next T in colex order
    int i = 0;
    while (i < nt && t[i] + 1 == (i + 1 < nt ? t[i + 1] : M)) ++i;
    if (i == nt) break;
    ++t[i];
    for (int j = 0; j < i; ++j) t[j] = j;
  }
  close();
  return tiles;
}

struct PlanKey {
  int device, M, NB, kB, kG;
  bool operator<(const PlanKey& o) const {
    return std::tie(device, M, NB, kB, kG) < std::tie(o.device, o.M, o.NB, o.kB, o.kG);
  }
};
struct Plan {
  uint64_t* dev = nullptr;
  uint32_t ntiles = 0;
  uint32_t grid = 0;  // workgroups launched: min(ntiles, kGroupWgPerCU x CUs)
};
std::mutex g_plan_mu;
std::map<PlanKey, Plan> g_plans;

int group_rmax(int M, int NB) { return M - NB <= kGroupRmax ? M - NB : -1; }

hipError_t get_plan(int M, int NB, int kB, int kG, Plan* out) {
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_plan_mu);
  auto it = g_plans.find(PlanKey{device, M, NB, kB, kG});
  if (it != g_plans.end()) {
    *out = it->second;
    return hipSuccess;
  }
  const std::vector<uint64_t> tiles = plan_tiles(M, NB, group_rmax(M, NB), kB, kG);
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  Plan p;
  p.ntiles = (uint32_t)tiles.size();
  p.grid = std::min<uint32_t>(p.ntiles, (uint32_t)std::max(cus, 1) * kGroupWgPerCU);
  if (!tiles.empty()) {
    e = hipMalloc(&p.dev, tiles.size() * sizeof(uint64_t));
    if (e != hipSuccess) return e;
    e = hipMemcpy(p.dev, tiles.data(), tiles.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p.dev);
      return e;
    }
  }
  g_plans[PlanKey{device, M, NB, kB, kG}] = p;
  *out = p;
  return hipSuccess;
}

std::mutex g_host_plan_mu;
std::map<PlanKey, std::vector<uint64_t>> g_host_plans;

template <int NB, bool DISP, bool MIXED = false>
int group_windows(int M) {
  return (GroupLayout<NB, DISP, MIXED>::kB * (M - NB) + 63) / 64 + 1;
}

template <int NB, bool DISP, bool MIXED = false>
size_t group_lds(int M) {
  using GL = GroupLayout<NB, DISP, MIXED>;
  const int D = NB + 1;
  return (size_t)GL::kB * GL::bytes + (size_t)kGroupRmax * GL::rbytes +
         (size_t)GL::kG * GL::gbytes +
         (size_t)(((D + 1) * (M + 1) + 1) & ~1) * sizeof(uint32_t) +
         (size_t)group_windows<NB, DISP, MIXED>(M) * (sizeof(uint64_t) + 1);
}

template <bool DISP, bool MIXED = false>
size_t group_lds_d(int d, int M) {
  switch (d) {
    case 3: return group_lds<2, DISP, MIXED>(M);
    case 4: return group_lds<3, DISP, MIXED>(M);
    default: return group_lds<4, DISP, MIXED>(M);
  }
}

template <bool MIXED>
int group_windows_d(int d, int M) {
  switch (d) {
    case 3: return group_windows<2, false, MIXED>(M);
    case 4: return group_windows<3, false, MIXED>(M);
    default: return group_windows<4, false, MIXED>(M);
  }
}

// Tile shape of the zero-mean plans of order d.
template <int NB>
int plan_kb_t(bool mixed) { return mixed ? GroupLayout<NB, false, true>::kB : GroupLayout<NB, false>::kB; }
template <int NB>
int plan_kg_t(bool mixed) { return mixed ? GroupLayout<NB, false, true>::kG : GroupLayout<NB, false>::kG; }
int plan_kb(int d, bool mixed) {
  return d == 3 ? plan_kb_t<2>(mixed) : d == 4 ? plan_kb_t<3>(mixed) : plan_kb_t<4>(mixed);
}
int plan_kg(int d, bool mixed) {
  return d == 3 ? plan_kg_t<2>(mixed) : d == 4 ? plan_kg_t<3>(mixed) : plan_kg_t<4>(mixed);
}

}  // namespace

bool group_supported(int d, int M, int flags, bool displaced) {
  if (d < 3 || d > kMaxOrder || (displaced && (flags & GBS_MIXED))) return false;
  for (int q = 1; q <= d; ++q)
    if (host_binom(M, q) >= (1ull << 29)) return false;
  if (group_rmax(M, d - 1) < 0 || M > 255) return false;
  const size_t lds = displaced ? group_lds_d<true>(d, M)
                    : (flags & GBS_MIXED) ? group_lds_d<false, true>(d, M)
                                          : group_lds_d<false>(d, M);
  return lds <= 64 * 1024;
}

const std::vector<uint64_t>& group_plan_host(int d, int M, bool mixed) {
  const int NB = d - 1;
  const int kB = plan_kb(d, mixed), kG = plan_kg(d, mixed);
  std::lock_guard<std::mutex> lock(g_host_plan_mu);
  const PlanKey key{-1, M, NB, kB, kG};
  auto it = g_host_plans.find(key);
  if (it == g_host_plans.end())
    it = g_host_plans.emplace(key, plan_tiles(M, NB, group_rmax(M, NB), kB, kG)).first;
  return it->second;  // map nodes are never erased: the reference stays valid
}

uint32_t group_plan_grid(uint32_t ntiles, int cu_count) {
  return std::min<uint32_t>(ntiles, (uint32_t)std::max(cu_count, 1) * kGroupWgPerCU);
}

// The operands of one single-instance launch.
struct GroupArgs {
  const double* Qi;
  const double* Qd;
  const double* mi;
  const double* pk;
  const float* E;
};

template <int D, int CONV, bool WC, bool DISP, bool MIXED>
static hipError_t launch_group_t(int M, const GroupArgs& g, const uint64_t* binom,
                                 const OrderTables& tab, double* m_out, double* k_out,
                                 double* p_out, DeviceStatus* st, hipStream_t s,
                                 const GroupPlanRef* ext) {
  constexpr int NB = D - 1;
  if (host_binom(M, D) == 0) return hipSuccess;
  Plan plan;
  if (ext) {
    plan.dev = const_cast<uint64_t*>(ext->dev);
    plan.ntiles = ext->ntiles;
    plan.grid = ext->grid;
  } else {
    using GL = GroupLayout<NB, DISP, MIXED>;
    hipError_t e = get_plan(M, NB, GL::kB, GL::kG, &plan);
    if (e != hipSuccess) return e;
  }
  if (plan.ntiles == 0) return hipSuccess;
  const int nwin = group_windows<NB, DISP, MIXED>(M);
  const size_t lds = group_lds<NB, DISP, MIXED>(M);
  hipLaunchKernelGGL((forward_group_kernel<D, CONV, WC, DISP, MIXED>), dim3(plan.grid),
                     dim3(kGroupThreads), lds, s, g.Qi, g.Qd, g.mi, g.pk, g.E, M, plan.dev,
                     plan.ntiles, binom, tab, m_out, k_out, p_out, st, nwin);
  return hipGetLastError();
}

template <int D, int CONV, bool DISP, bool MIXED>
static hipError_t launch_group_w(int M, const GroupArgs& g, const uint64_t* binom,
                                 const OrderTables& tab, double* m_out, double* k_out,
                                 double* p_out, DeviceStatus* st, hipStream_t s,
                                 const GroupPlanRef* ext) {
  if (k_out)
    return launch_group_t<D, CONV, true, DISP, MIXED>(M, g, binom, tab, m_out, k_out, p_out, st,
                                                      s, ext);
  return launch_group_t<D, CONV, false, DISP, MIXED>(M, g, binom, tab, m_out, k_out, p_out, st, s,
                                                     ext);
}

template <int D, int CONV>
static hipError_t launch_group_v(int M, int flags, const GroupArgs& g, const uint64_t* binom,
                                 const OrderTables& tab, double* m_out, double* k_out,
                                 double* p_out, DeviceStatus* st, hipStream_t s,
                                 const GroupPlanRef* ext) {
  // displaced states plan their own (narrower) tiles
  if (g.mi)
    return launch_group_w<D, CONV, true, false>(M, g, binom, tab, m_out, k_out, p_out, st, s,
                                                nullptr);
  if (flags & GBS_MIXED)
    return launch_group_w<D, CONV, false, true>(M, g, binom, tab, m_out, k_out, p_out, st, s, ext);
  return launch_group_w<D, CONV, false, false>(M, g, binom, tab, m_out, k_out, p_out, st, s, ext);
}

template <int D>
static hipError_t launch_group_c(int M, int flags, const GroupArgs& g, const uint64_t* binom,
                                 const OrderTables& tab, double* m_out, double* k_out,
                                 double* p_out, DeviceStatus* st, hipStream_t s,
                                 const GroupPlanRef* ext) {
  if (flags & GBS_PARITY)
    return launch_group_v<D, GBS_PARITY>(M, flags, g, binom, tab, m_out, k_out, p_out, st, s, ext);
  return launch_group_v<D, GBS_CLICK>(M, flags, g, binom, tab, m_out, k_out, p_out, st, s, ext);
}

void group_tiles(int d, int M, bool mixed, std::vector<uint64_t>* out) {
  const int NB = d - 1;
  const std::vector<uint64_t> t =
      plan_tiles(M, NB, group_rmax(M, NB), plan_kb(d, mixed), plan_kg(d, mixed));
  out->insert(out->end(), t.begin(), t.end());
}

size_t group_batched_lds(int d, int flags, int max_M, int* nwin_max) {
  *nwin_max = (flags & GBS_MIXED) ? group_windows_d<true>(d, max_M) : group_windows_d<false>(d, max_M);
  return (flags & GBS_MIXED) ? group_lds_d<false, true>(d, max_M) : group_lds_d<false>(d, max_M);
}

namespace {

template <int D, int CONV, bool MIXED>
const void* batched_fn() {
  return reinterpret_cast<const void*>(&forward_group_batched_kernel<D, CONV, true, MIXED>);
}

template <int D>
const void* batched_fn_f(int flags) {
  if (flags & GBS_MIXED)
    return (flags & GBS_PARITY) ? batched_fn<D, GBS_PARITY, true>() : batched_fn<D, GBS_CLICK, true>();
  return (flags & GBS_PARITY) ? batched_fn<D, GBS_PARITY, false>() : batched_fn<D, GBS_CLICK, false>();
}

const void* pick_batched(int d, int flags) {
  switch (d) {
    case 3: return batched_fn_f<3>(flags);
    case 4: return batched_fn_f<4>(flags);
    default: return batched_fn_f<5>(flags);
  }
}

}  // namespace

hipError_t group_batched_grid(int d, int flags, size_t lds, int cu_count, int* grid) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pick_batched(d, flags),
                                                             kGroupThreads, lds);
  if (e != hipSuccess) return e;
  *grid = std::max(1, per_cu) * std::max(1, cu_count);
  return hipSuccess;
}

template <int D, int CONV, bool MIXED>
static void launch_batched_t(const GroupBatchInstance* inst, const GroupBatchItem* items,
                             uint32_t n_items, unsigned* counter, int grid, int max_M,
                             int nwin_max, size_t lds, const uint64_t* binom, DeviceStatus* st,
                             hipStream_t s) {
  hipLaunchKernelGGL((forward_group_batched_kernel<D, CONV, true, MIXED>), dim3(grid),
                     dim3(kGroupThreads), lds, s, inst, items, n_items, counter, binom, max_M, st,
                     nwin_max);
}

using BatchedLaunch = void (*)(const GroupBatchInstance*, const GroupBatchItem*, uint32_t,
                               unsigned*, int, int, int, size_t, const uint64_t*, DeviceStatus*,
                               hipStream_t);

template <int D>
static BatchedLaunch pick_batched_launch(bool parity, bool mixed) {
  if (mixed)
    return parity ? launch_batched_t<D, GBS_PARITY, true> : launch_batched_t<D, GBS_CLICK, true>;
  return parity ? launch_batched_t<D, GBS_PARITY, false> : launch_batched_t<D, GBS_CLICK, false>;
}

hipError_t launch_group_batched(int d, int flags, const GroupBatchInstance* inst,
                                const GroupBatchItem* items, uint32_t n_items, unsigned* counter,
                                int grid, int max_M, int nwin_max, size_t lds,
                                const uint64_t* binom, DeviceStatus* st, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const bool parity = flags & GBS_PARITY, mixed = flags & GBS_MIXED;
  BatchedLaunch fn;
  switch (d) {
    case 3: fn = pick_batched_launch<3>(parity, mixed); break;
    case 4: fn = pick_batched_launch<4>(parity, mixed); break;
    case 5: fn = pick_batched_launch<5>(parity, mixed); break;
    default: return hipErrorInvalidValue;
  }
  fn(inst, items, n_items, counter, grid, max_M, nwin_max, lds, binom, st, s);
  return hipGetLastError();
}

hipError_t launch_forward_group(int d, int M, int flags, const double* Qi, const double* Qd,
                                const double* mi, const double* pk, const float* E,
                                const uint64_t* binom, const OrderTables& tab, double* m_out,
                                double* k_out, double* p_out, DeviceStatus* st, hipStream_t s,
                                const GroupPlanRef* plan) {
  if (mi && (flags & GBS_MIXED)) return hipErrorInvalidValue;
  const GroupArgs g{Qi, Qd, mi, pk, E};
  switch (d) {
    case 3: return launch_group_c<3>(M, flags, g, binom, tab, m_out, k_out, p_out, st, s, plan);
    case 4: return launch_group_c<4>(M, flags, g, binom, tab, m_out, k_out, p_out, st, s, plan);
    case 5: return launch_group_c<5>(M, flags, g, binom, tab, m_out, k_out, p_out, st, s, plan);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gbs
