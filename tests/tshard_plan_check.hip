// Host check of the T-shared shard kernel's work decomposition (built and run
// by tests/test_group_plan.py; no GPU needed).  For order-d colex rank ranges
// [rank0, rank0 + count), run as the library runs them (consecutive chunks of
// at most a given number of T's): the T lists cover every rank exactly once
// through their tiles, each tile's lanes (a = al + lane) and b_0 (bl .. bl + nb - 1) name
// subsets {a, b_0} + T whose colex rank is the one the kernel writes, within
// the kernel's bounds (a < b_0 < min T, nb <= kTsB), and the kernel's binary
// search from a tile index lands on the tile's T.
#include <cstdio>

#include "gbs_forward_shard.hip"

namespace gbs {
uint64_t host_binom(int n, int k) {
  if (k < 0 || n < k) return 0;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}
}  // namespace gbs

// colex unranking (greedy from the top element), as the library's gbs_colex_unrank
extern "C" gbs_status gbs_colex_unrank(int32_t d, int64_t r, int32_t* S) {
  uint64_t rem = (uint64_t)r;
  int n = 1 << 12;
  for (int i = d - 1; i >= 0; --i) {
    int c = i;
    while (gbs::host_binom(c + 1, i + 1) <= rem && c + 1 < n) ++c;
    S[i] = c;
    rem -= gbs::host_binom(c, i + 1);
    n = c;
  }
  return GBS_OK;
}

using namespace gbs;

static long fails = 0;

// One chunk: the list of the start of [r0, r0 + left), covering `covered` ranks.
static void check_chunk(int d, int M, uint64_t rank0, uint64_t done, uint64_t left,
                        size_t max_t, std::vector<unsigned char>& seen, uint64_t* covered_out,
                        uint64_t* written) {
  std::vector<ShardT> tl;
  uint32_t ntiles = 0;
  const uint64_t r0 = rank0 + done;
  const uint64_t covered = ts_build(d, M, r0, left, tl, &ntiles, max_t);
  *covered_out = covered;
  if (tl.empty() || tl.size() > max_t || covered == 0 || covered > left) {
    if (fails++ < 10) printf("d=%d M=%d chunk at %llu: %zu T's, %llu covered\n", d, M,
                             (unsigned long long)r0, tl.size(), (unsigned long long)covered);
    *covered_out = left;
    return;
  }
  const int NT = d - 2;
  for (uint32_t tile = 0; tile < ntiles; ++tile) {
    // the kernel's search
    uint32_t lo = 0, hi = (uint32_t)tl.size() - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (tl[mid].tile0 <= tile) lo = mid;
      else hi = mid - 1;
    }
    const ShardT& T = tl[lo];
    const uint32_t next0 = lo + 1 < tl.size() ? tl[lo + 1].tile0 : ntiles;
    if (!(T.tile0 <= tile && tile < next0) && fails++ < 10) printf("tile %u: wrong T\n", tile);
    uint32_t al = 0, bl = 0, nb = 0;
    (void)ts_tiles(T.b0lo, T.b0hi, (int64_t)(tile - T.tile0), &al, &bl, &nb);
    if ((nb < 1 || nb > (uint32_t)kTsB || bl + nb - 1 >= T.t[0] || al >= bl + nb - 1) &&
        fails++ < 10)
      printf("d=%d M=%d tile %u: al %u bl %u nb %u t1 %u\n", d, M, tile, al, bl, nb, T.t[0]);
    for (uint32_t j = 0; j < nb; ++j) {
      const uint32_t b0 = bl + j;
      for (uint32_t lane = 0; lane < (uint32_t)kTsA; ++lane) {
        const uint32_t a = al + lane;
        const uint32_t off = b0 * (b0 - 1) / 2 + a;
        if (!(a < b0 && off >= T.lo && off < T.hi)) continue;
        const int64_t out = T.out0 + (int64_t)off;  // relative to this chunk's r0
        if (out < 0 || (uint64_t)out >= covered) {
          if (fails++ < 10) printf("d=%d M=%d: output %lld outside the chunk\n", d, M, (long long)out);
          continue;
        }
        // the colex rank of {a, b_0} + T
        uint64_t rk = a + host_binom(b0, 2);
        for (int k = 0; k < NT; ++k) rk += host_binom(T.t[k], k + 3);
        if (rk != r0 + (uint64_t)out && fails++ < 10)
          printf("d=%d M=%d: subset rank %llu, written at %llu\n", d, M, (unsigned long long)rk,
                 (unsigned long long)(r0 + out));
        bool order_ok = b0 < T.t[0] && (int)T.t[NT - 1] < M;
        for (int k = 1; k < NT; ++k) order_ok = order_ok && T.t[k - 1] < T.t[k];
        if (!order_ok && fails++ < 10) printf("d=%d M=%d: T not a subset\n", d, M);
        if (seen[done + out]++ && fails++ < 10) printf("d=%d M=%d: rank %lld twice\n", d, M, (long long)(done + out));
        ++*written;
      }
    }
  }
}

// A whole range as the library runs it: consecutive chunks of at most max_t T's.
static void check(int d, int M, uint64_t rank0, uint64_t count, size_t max_t = kTsMaxT) {
  std::vector<unsigned char> seen(count, 0);
  uint64_t done = 0, written = 0;
  int chunks = 0;
  while (done < count) {
    uint64_t covered = 0;
    check_chunk(d, M, rank0, done, count - done, max_t, seen, &covered, &written);
    done += covered;
    ++chunks;
  }
  if (written != count && fails++ < 10)
    printf("d=%d M=%d [%llu, +%llu) in %d chunks: %llu written\n", d, M, (unsigned long long)rank0,
           (unsigned long long)count, chunks, (unsigned long long)written);
}

int main() {
  long cases = 0;
  for (int d = 3; d <= 5; ++d) {
    for (int M : {5, 6, 13, 17, 40}) {
      if (d > M) continue;
      const uint64_t n = host_binom(M, d);
      const uint64_t cuts[] = {0, 1, 2, 7, 30, n / 3, n / 2, n / 2 + 1, n - 3, n};
      check(d, M, 0, n);
      ++cases;
      for (int i = 0; i + 1 < 10; ++i)
        for (int j = i + 1; j < 10; ++j)
          if (cuts[j] > cuts[i] && cuts[j] <= n) {
            check(d, M, cuts[i], cuts[j] - cuts[i]);
            ++cases;
          }
    }
  }
  // the pseudo-PNR size: shards at the start, in the middle and at the end of
  // an order (order-5 ranks beyond 2^32), and the whole of order 5 at M = 144
  for (int d = 3; d <= 5; ++d) {
    const uint64_t total = host_binom(1152, d), cnt = 262144;
    for (uint64_t r0 : {(uint64_t)0, total / 2 - cnt / 2, total - cnt}) {
      check(d, 1152, r0, cnt);
      ++cases;
    }
  }
  check(5, 1152, host_binom(1152, 5) / 2, host_binom(144, 5));
  check(5, 144, 0, host_binom(144, 5));
  cases += 2;
  // chunked runs: lists of a few T's, and order 5 at M = 100 (161,700 T's,
  // three chunks of the default size)
  for (size_t mt : {(size_t)1, (size_t)3, (size_t)50})
    for (int d = 3; d <= 5; ++d) {
      const uint64_t n = host_binom(17, d);
      check(d, 17, 0, n, mt);
      check(d, 17, 5, n - 11, mt);
      cases += 2;
    }
  check(5, 100, 0, host_binom(100, 5));
  check(5, 1152, 0, 20000000);
  cases += 2;
  printf("cases %ld failures %ld\n", cases, fails);
  return fails != 0;
}
