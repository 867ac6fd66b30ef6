// Sanitizer driver for the library's host code (planner, block-product
// symbolic stage, halo plans) -- test infrastructure, built with g++ and
// -fsanitize=address,undefined or -fsanitize=thread by tests/test_sanitizers.py.
// The device launchers the halo entry points reference are stubbed: no
// device code is built or called here.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../../include/vbcsr.h"
#include "../../paper_2609_04397_amd/csrc/common.hpp"
#include "../../paper_2609_04397_amd/csrc/kernels.hpp"

namespace vbcsr {
static thread_local std::string g_err;
int set_error(int code, const std::string &msg) {
  g_err = msg;
  return code;
}
int api_exception(const char *where) {
  g_err = where;
  return VBCSR_EINVAL;
}
hipError_t launch_rows_pack(const void *, int64_t, int64_t, const int32_t *, int64_t, int32_t, int,
                            void *, int64_t, hipStream_t) {
  std::abort();
}
hipError_t launch_rows_reduce(void *, int64_t, int64_t, const int32_t *, const int64_t *,
                              const int64_t *, int64_t, int64_t, const void *, int64_t, int32_t, int,
                              hipStream_t) {
  std::abort();
}
}  // namespace vbcsr
extern "C" const char *hipGetErrorString(hipError_t) { return "stub"; }

using namespace vbcsr;

struct Graph {
  int32_t n;
  std::vector<int32_t> b, ci;
  std::vector<int64_t> rp;
  int64_t nval = 0;
};

// Random block graph: unsorted columns, empty rows, block sizes 1..20.
static Graph random_graph(int32_t n, int deg, uint64_t seed, bool symmetric) {
  std::mt19937_64 rng(seed);
  Graph g;
  g.n = n;
  g.b.resize(n);
  for (auto &x : g.b) x = 1 + (int32_t)(rng() % 20);
  std::vector<std::vector<int32_t>> rows(n);
  for (int32_t i = 0; i < n; ++i) {
    if (rng() % 50 == 0) continue;  // empty row
    const int d = (int)(rng() % (2 * deg + 1));
    for (int t = 0; t < d; ++t) {
      const int32_t j = (int32_t)((i + (int64_t)(rng() % 2001) - 1000 + n) % n);
      rows[i].push_back(j);
      if (symmetric && j != i) rows[j].push_back(i);
    }
  }
  g.rp.assign((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; ++i) {
    std::sort(rows[i].begin(), rows[i].end());
    rows[i].erase(std::unique(rows[i].begin(), rows[i].end()), rows[i].end());
    std::shuffle(rows[i].begin(), rows[i].end(), rng);
    for (int32_t j : rows[i]) {
      g.ci.push_back(j);
      g.nval += (int64_t)g.b[i] * g.b[j];
    }
    g.rp[i + 1] = (int64_t)g.ci.size();
  }
  return g;
}

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                     \
    }                                                              \
  } while (0)

int main() {
  // planner: threaded stages (n >= 8192), every order, square and rank-local
  for (int rep = 0; rep < 2; ++rep) {
    Graph g = random_graph(12000, 8, 11 + rep, rep == 1);
    std::string err;
    CHECK(validate_graph(g.n, g.b.data(), g.rp.data(), g.ci.data(), g.nval, err) == VBCSR_OK);
    for (int order = 0; order <= 3; ++order) {
      HostPlan p;
      build_plan(g.n, g.b.data(), g.rp.data(), g.ci.data(), order, p, true);
      CHECK(p.nnz == g.nval);
      CHECK((int64_t)p.fwd.colx.size() == p.fwd.n_cols);
    }
    // rank-local: the last 3000 atoms have empty rows
    std::vector<int64_t> rp(g.rp);
    const int32_t nr = g.n - 3000;
    for (int32_t i = nr + 1; i <= g.n; ++i) rp[i] = rp[nr];
    int64_t nv = 0;
    for (int32_t i = 0; i < nr; ++i)
      for (int64_t k = rp[i]; k < rp[i + 1]; ++k) nv += (int64_t)g.b[i] * g.b[g.ci[k]];
    CHECK(validate_graph(g.n, g.b.data(), rp.data(), g.ci.data(), nv, err) == VBCSR_OK);
    HostPlan p;
    build_plan(g.n, g.b.data(), rp.data(), g.ci.data(), VBCSR_ORDER_CLUSTER, p, true, nr);
    CHECK((int32_t)p.fwd.rows.size() == nr && (int32_t)p.tr.rows.size() == g.n);
    // malformed inputs are statuses
    std::vector<int32_t> bad(g.ci);
    bad[bad.size() / 2] = g.n + 5;
    CHECK(validate_graph(g.n, g.b.data(), g.rp.data(), bad.data(), g.nval, err) == VBCSR_EINVAL);
    CHECK(validate_graph(g.n, g.b.data(), g.rp.data(), g.ci.data(), g.nval + 1, err) ==
          VBCSR_ESHAPE);
  }
  // halo plans of an 8-rank split of a random graph
  {
    Graph g = random_graph(6000, 6, 9, true);
    std::vector<int32_t> owner(g.n);
    for (int32_t i = 0; i < g.n; ++i) owner[i] = (int32_t)((int64_t)i * 8 / g.n);
    for (int32_t r = 0; r < 8; ++r) {
      vbcsr_halo *H = nullptr;
      CHECK(vbcsr_halo_create(&H, g.n, g.b.data(), g.rp.data(), g.ci.data(), owner.data(), r, 8) ==
            VBCSR_OK);
      int32_t no = 0, ng = 0;
      int64_t nb = 0, nv = 0, ns = 0, nr = 0;
      CHECK(vbcsr_halo_info(H, &no, &ng, &nb, &nv, &ns, &nr) == VBCSR_OK);
      std::vector<int32_t> gid(no + ng), bb(no + ng), ci(nb), sr(ns), rr(nr);
      std::vector<int64_t> rp(no + 1), sp(9), rcp(9), rptr(nr + 1), rpos(ns);
      CHECK(vbcsr_halo_graph(H, gid.data(), bb.data(), rp.data(), ci.data()) == VBCSR_OK);
      CHECK(vbcsr_halo_lists(H, sp.data(), sr.data(), rcp.data(), rr.data(), rptr.data(),
                             rpos.data()) == VBCSR_OK);
      std::vector<double> gv((size_t)g.nval, 1.0), lv((size_t)nv);
      CHECK(vbcsr_halo_local_values(H, gv.data(), lv.data()) == VBCSR_OK);
      vbcsr_halo_destroy(H);
    }
  }
  std::printf("host driver: %d failed checks\n", fails);
  return fails ? 1 : 0;
}
