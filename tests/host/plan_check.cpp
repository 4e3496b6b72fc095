// Host check of the merge-tree plan (paper_2508_11467_amd/csrc/plan.cpp),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizer.py: plans for many seeded batches and leaf sizes,
// each checked against the properties of the recursive split at k = m / 2.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "plan.h"

using namespace bdc;

static int fails = 0;
#define CHECK(c)                                                 \
  do {                                                           \
    if (!(c)) {                                                  \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                   \
    }                                                            \
  } while (0)

static void check_plan(const std::vector<int64_t>& sizes, int leaf) {
  const int64_t batch = (int64_t)sizes.size();
  const HostPlan p = build_host_plan(sizes.data(), batch, leaf);
  // leaves run left to right over every problem's rows; the rows between
  // them are the merges' middle rows: sum of leaf rows + merges = n
  size_t li = 0;
  int64_t vo = 0, mo = 0, merges = 0;
  for (int64_t i = 0; i < batch; ++i) {
    const int64_t n = sizes[i];
    CHECK(p.prob[i] == n && p.prob[batch + i] == vo && p.prob[2 * batch + i] == mo);
    int64_t r = 0, rows = 0, nl = 0;
    while (li < p.leaves.size() && p.leaves[li].vec_off == vo && n > 0) {
      const LeafDesc& L = p.leaves[li++];
      CHECK(L.mat_off == mo && L.ld == n && L.r0 >= r);
      CHECK(L.m >= 1 && L.m <= leaf && (L.s == 0 || L.s == 1));
      CHECK((L.s == 0) == (L.r0 + L.m == n));  // only the last leaf is square
      r = L.r0 + L.m;
      rows += L.m;
      ++nl;
    }
    CHECK(r == n);
    if (n > 0) {
      CHECK(nl >= 1);
      merges += nl - 1;
      CHECK(rows + (nl - 1) == n);
    }
    vo += n;
    mo += n * n;
  }
  CHECK(li == p.leaves.size());
  CHECK(p.total_n == vo && p.total_n2 == mo);
  CHECK((int64_t)p.nodes.size() == merges);
  // merges: ids in order, grouped by height, sizes consistent
  size_t off = 0;
  for (size_t h = 0; h < p.level_count.size(); ++h) {
    int mx = 0;
    for (int q = 0; q < p.level_count[h]; ++q) {
      CHECK(off < p.nodes.size());
      if (off >= p.nodes.size()) return;
      const NodeDesc& d = p.nodes[off];
      CHECK(d.id == (int)off);
      CHECK(d.k == d.m / 2 && d.m > leaf && d.r0 >= 0 && d.r0 + d.m + d.s <= d.ld + 1);
      mx = d.m > mx ? d.m : mx;
      ++off;
    }
    CHECK(mx == p.level_max_m[h]);
  }
  CHECK(off == p.nodes.size());
  // final-pass work items map to their problems in order
  for (size_t q = 1; q < p.uprob.size(); ++q) CHECK(p.uprob[q] >= p.uprob[q - 1]);
  for (size_t q = 1; q < p.vprob.size(); ++q) CHECK(p.vprob[q] >= p.vprob[q - 1]);
  for (int64_t i = 0; i < batch; ++i) {
    const int64_t u0 = p.prob[3 * batch + i], v0 = p.prob[4 * batch + i];
    if (sizes[i] > 0 && u0 < p.total_cols) CHECK(p.uprob[u0] == (int32_t)i);
    if (sizes[i] > 0 && v0 < p.total_tiles) CHECK(p.vprob[v0] == (int32_t)i);
  }
}

int main() {
  std::mt19937_64 g(2508);
  const int leaves[] = {4, 6, 8, 12, 16, 20, 24, 32};
  for (int leaf : leaves)
    for (int64_t n : {0, 1, 2, 3, 4, 5, 31, 32, 33, 34, 64, 65, 100, 255, 256, 257, 1000, 4096, 16384, 32768})
      check_plan({n}, leaf);
  for (int t = 0; t < 200; ++t) {
    const int batch = 1 + (int)(g() % 40);
    std::vector<int64_t> sizes(batch);
    for (auto& s : sizes) s = (int64_t)(g() % 3000);
    check_plan(sizes, leaves[g() % 8]);
  }
  std::vector<int64_t> big(2000);
  for (auto& s : big) s = 32 + (int64_t)(g() % 2017);
  check_plan(big, 16);
  std::printf("plan checks: %d failures\n", fails);
  return fails == 0 ? 0 : 1;
}
