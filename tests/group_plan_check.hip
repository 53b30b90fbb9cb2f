// Host check of the group kernel's tile plans and descriptors (built and run
// by tests/test_group_plan.py; no GPU needed).  For every (M, order) the group
// kernel takes, the plan must cover every subset exactly once, and each tile's
// descriptor must decode to its first B, its B count (1 .. kB) and the T
// of that B, with every lane's walk over the groups (the kernel's way of
// finding its B) landing on the B that colex unranking gives, within the
// walk's step limit; each tile's groups and (T, a) records must fit the
// kernel's LDS bounds.  Both tile shapes are checked: the FP64 one and the
// wider one of the mixed form.
#include <cstdio>

#include "gbs_forward_group.hip"

namespace gbs {
uint64_t host_binom(int n, int k) {
  if (k < 0 || n < k) return 0;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}
}  // namespace gbs

using namespace gbs;

// the kernel's colex successor, on the host
static void next_t(int* t, int nt, int M) {
  for (int i = 0; i < nt; ++i) {
    const int lim = (i + 1 < nt) ? t[i + 1] : M;
    if (t[i] + 1 < lim) {
      ++t[i];
      for (int j = 0; j < i; ++j) t[j] = j;
      return;
    }
  }
}

int main() {
  long fails = 0, tiles_total = 0, lanes = 0;
  int max_walk = 0;
  const int Ms[] = {3, 4, 5, 6, 12, 13, 16, 17, 40, 64, 100, 143, 144, 145, 150, 152};
  for (int mixed = 0; mixed < 2; ++mixed)
  for (int M : Ms) {
    for (int d = 3; d <= 5; ++d) {
      if (d > M || !group_supported(d, M, mixed ? GBS_MIXED : 0, false)) continue;
      const int NB = d - 1, nt = NB - 1;
      const int kB = plan_kb(d, mixed != 0), kG = plan_kg(d, mixed != 0);
      const std::vector<uint64_t>& tiles = group_plan_host(d, M, mixed != 0);
      uint64_t beta = 0, subsets = 0;
      for (uint64_t desc : tiles) {
        ++tiles_total;
        const uint32_t beta0 = (uint32_t)(desc & kDescBetaMask);
        const int nB = (int)((desc >> kDescNbShift) & kDescNbMask);
        int t0[3] = {0, 0, 0};
        for (int j = 0; j < nt; ++j) t0[j] = (int)((desc >> (kDescTShift + 8 * j)) & 255);
        if (beta0 != beta || nB < 1 || nB > kB) {
          if (fails++ < 10) printf("M=%d d=%d tile at %u: beta0 %u, nB %d\n", M, d, (unsigned)beta, beta0, nB);
        }
        uint32_t tpart = 0;
        for (int j = 0; j < nt; ++j) tpart += (uint32_t)host_binom(t0[j], j + 2);
        int groups = 0, records = 0, prev_key = -1, group_max_b0 = 0;
        for (int lane = 0; lane < nB; ++lane) {
          int tt[3] = {t0[0], t0[1], t0[2]};
          int o = (int)(beta0 - tpart) + lane, it = 0;
          for (; it < kWalkMax && o >= tt[0]; ++it) {
            o -= tt[0];
            next_t(tt, nt, M);
          }
          if (it > max_walk) max_walk = it;
          // the walk's B = {o} + T must be a subset (o < min T) of colex rank beta0 + lane
          int ref[4];
          ref[0] = o;
          for (int j = 0; j < nt; ++j) ref[j + 1] = tt[j];
          uint64_t rank = 0;
          for (int j = 0; j < NB; ++j) rank += host_binom(ref[j], j + 1);
          const bool ok = o >= 0 && (nt == 0 || o < tt[0]) && rank == (uint64_t)beta0 + lane;
          if (!ok && fails++ < 10) printf("M=%d d=%d rank %u: walk disagrees\n", M, d, beta0 + lane);
          const int key = ref[1] + 256 * (nt > 1 ? ref[2] : 0) + 65536 * (nt > 2 ? ref[3] : 0);
          if (key != prev_key) {
            records += group_max_b0 > 0 ? group_max_b0 : 0;
            ++groups;
            prev_key = key;
            group_max_b0 = 0;
          }
          group_max_b0 = ref[0] > group_max_b0 ? ref[0] : group_max_b0;
          subsets += (uint64_t)ref[0];
          ++lanes;
        }
        records += group_max_b0;
        if ((groups > kG || records > M - NB) && fails++ < 10)
          printf("M=%d d=%d tile at %u: %d groups, %d records\n", M, d, beta0, groups, records);
        beta += (uint64_t)nB;
      }
      if (beta != host_binom(M, NB) || subsets != host_binom(M, d)) {
        if (fails++ < 10) printf("M=%d d=%d: %llu B's, %llu subsets\n", M, d,
                                 (unsigned long long)beta, (unsigned long long)subsets);
      }
    }
  }
  printf("tiles %ld lanes %ld max walk %d (limit %d) failures %ld\n", tiles_total, lanes, max_walk,
         kWalkMax, fails);
  return fails != 0;
}
