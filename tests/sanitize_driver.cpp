// Host-only exercise of the option validation, the cluster tree, the level
// schedule and the structure query, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Exits non-zero
// on a wrong answer; the sanitizers abort on a memory or undefined-behaviour
// error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "../paper_1701_00182_amd/csrc/plan.h"

extern "C" acr_status_t acr_plan_structure(int32_t, int32_t, int32_t, int32_t, acr_structure_t*, int32_t*,
                                           int32_t*, int32_t*, int32_t*, int32_t*, int32_t*);

static int fails = 0;
#define EXPECT(c)                                              \
  do {                                                         \
    if (!(c)) {                                                \
      std::fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #c); \
      ++fails;                                                 \
    }                                                          \
  } while (0)

static acr_options_t base() {
  acr_options_t o;
  std::memset(&o, 0, sizeof(o));
  o.nx = o.ny = o.nplanes = 8;
  o.eps = 1e-3;
  o.leaf = 16;
  o.inner_eps_ratio = 1.0;
  return o;
}

static void dummy_release(void*, void*, hipStream_t) {}
static void* dummy_alloc(size_t, void*, hipStream_t) { return nullptr; }

int main() {
  using acr::options_valid;
  const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
  acr_options_t o = base();
  EXPECT(options_valid(&o));
  EXPECT(!options_valid(nullptr));
  o = base(); o.nx = 0; EXPECT(!options_valid(&o));
  o = base(); o.ny = -3; EXPECT(!options_valid(&o));
  o = base(); o.nplanes = 0; EXPECT(!options_valid(&o));
  o = base(); o.leaf = 0; EXPECT(!options_valid(&o));
  o = base(); o.eps = -1e-3; EXPECT(!options_valid(&o));
  o = base(); o.eps = nan; EXPECT(!options_valid(&o));
  o = base(); o.eps = inf; EXPECT(!options_valid(&o));
  o = base(); o.max_rank = -1; EXPECT(!options_valid(&o));
  o = base(); o.precision = 6; EXPECT(!options_valid(&o));
  o = base(); o.precision = 5; EXPECT(options_valid(&o));
  o = base(); o.stencil_points = 9; EXPECT(!options_valid(&o));
  o = base(); o.stencil_points = 27; EXPECT(options_valid(&o));
  o = base(); o.precision = -1; EXPECT(!options_valid(&o));
  o = base(); o.inner_eps_ratio = nan; EXPECT(!options_valid(&o));
  o = base(); o.inner_eps_ratio = -1.0; EXPECT(!options_valid(&o));
  o = base(); o.inner_eps_ratio = inf; EXPECT(!options_valid(&o));
  o = base(); o.alloc = dummy_alloc; EXPECT(!options_valid(&o));
  o = base(); o.release = dummy_release; EXPECT(!options_valid(&o));
  o = base(); o.alloc = dummy_alloc; o.release = dummy_release; EXPECT(options_valid(&o));
  // sizes whose products overflow 32-bit integers
  o = base(); o.nx = 1 << 16; o.ny = 1 << 16; EXPECT(!options_valid(&o));
  o = base(); o.nx = 1 << 14; o.ny = 1 << 14; o.nplanes = 1 << 30; EXPECT(!options_valid(&o));
  o = base(); o.nx = 0x7fffffff; o.ny = 0x7fffffff; EXPECT(!options_valid(&o));

  // cluster tree invariants over many shapes: segments tile their parent,
  // the permutation is a bijection, the leaves hold at most `leaf` points
  for (int nx = 1; nx <= 24; ++nx)
    for (int ny = 1; ny <= 24; ny += 3)
      for (int leaf : {1, 2, 3, 5, 16, 64}) {
        acr::Tree t;
        if (!t.build(nx, ny, leaf)) continue;
        EXPECT(t.M == nx * ny);
        std::vector<int> seen(t.M, 0);
        for (int p : t.perm) {
          EXPECT(p >= 0 && p < t.M);
          if (p >= 0 && p < t.M) seen[p]++;
        }
        for (int c : seen) EXPECT(c == 1);
        for (int d = 0; d < t.L; ++d)
          for (int s = 0; s < (1 << d); ++s) {
            EXPECT(t.off[d + 1][2 * s] == t.off[d][s]);
            EXPECT(t.sz[d + 1][2 * s] + t.sz[d + 1][2 * s + 1] == t.sz[d][s]);
          }
        for (int s = 0; s < (1 << t.L); ++s) EXPECT(t.sz[t.L][s] <= leaf);
        EXPECT(t.leaf_max <= leaf);
      }

  // level schedule: every plane but the last is eliminated exactly once
  for (int nz = 1; nz <= 70; ++nz) {
    int last = -2;
    auto sched = acr::level_schedule(nz, &last);
    std::vector<int> elim(nz, 0);
    for (auto& lv : sched)
      for (size_t q = 0; q < lv.size(); q += 2) elim[lv[q]]++;
    for (int k = 0; k < nz; ++k) EXPECT(elim[k] == (k == last ? 0 : 1));
  }

  // the structure query: sizes first, then every array
  for (int leaf : {4, 7, 32}) {
    acr_structure_t info;
    EXPECT(acr_plan_structure(13, 9, 11, leaf, &info, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
           ACR_SUCCESS);
    std::vector<int32_t> perm(info.M), noff(info.nodes), nsz(info.nodes), lsz(info.levels),
        sp(info.schedule_len), se(info.schedule_len);
    EXPECT(acr_plan_structure(13, 9, 11, leaf, &info, perm.data(), noff.data(), nsz.data(), lsz.data(), sp.data(),
                              se.data()) == ACR_SUCCESS);
    EXPECT(nsz[0] == 13 * 9 && noff[0] == 0);
  }
  acr_structure_t info;
  EXPECT(acr_plan_structure(3, 3, 2, 0, &info, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
         ACR_ERROR_INVALID_VALUE);
  EXPECT(acr_plan_structure(3, 3, 2, 1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
         ACR_ERROR_INVALID_VALUE);
  if (fails) return 1;
  std::printf("sanitize driver: all checks passed\n");
  return 0;
}
