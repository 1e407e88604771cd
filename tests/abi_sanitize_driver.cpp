// The C ABI's argument checks under AddressSanitizer and UBSan (host code
// only), with no GPU: the bad-argument calls of the CPU ABI tests, each
// expected to return GC_EINVAL with its message. Built with the library's
// sources by tests/test_host_sanitizers.py; exits non-zero on a failed
// expectation.
#include <cstdio>
#include <cstring>
#include <vector>
#include "graphcage.h"
#define EXPECT(c) do { if (!(c)) { std::printf("FAIL line %d: %s (%s)\n", __LINE__, #c, gc_last_error()); ++fails; } } while (0)
int main() {
  int fails = 0;
  gc_graph g = nullptr;
  int32_t rp[3] = {0, 1, 2}, ci[2] = {1, 0};
  EXPECT(graph_load_csr(0, 0, rp, ci, nullptr, 0, nullptr, &g) == GC_EINVAL);
  EXPECT(std::strstr(gc_last_error(), "positive") != nullptr);
  EXPECT(graph_load_csr(2, 2, nullptr, ci, nullptr, 0, nullptr, &g) == GC_EINVAL);
  EXPECT(graph_load_csr(2, 2, rp, ci, nullptr, 0, nullptr, nullptr) == GC_EINVAL);
  EXPECT(graph_load_csr(2, 2, rp, ci, nullptr, 0x10, nullptr, &g) == GC_EINVAL);
  EXPECT(graph_load_csr(2, int64_t(1) << 31, rp, ci, nullptr, 0, nullptr, &g) == GC_EINVAL);
  EXPECT(graph_load_csr(2, 1, rp, ci, nullptr, 0, nullptr, &g) == GC_EINVAL);
  struct Bad { std::vector<int32_t> rp, ci, w; const char* needle; };
  const Bad bad[] = {{{0, 2, 1, 2}, {1, 2}, {}, "decreases"},  {{0, 1, 2}, {1, 5}, {}, "out of range"},
                     {{0, 1, 2}, {0, 0}, {}, "self-loop"},      {{0, 2, 2, 2}, {2, 1}, {}, "ascending"},
                     {{0, 2, 2, 2}, {1, 1}, {}, "ascending"},   {{0, 1, 2}, {1, 0}, {3, 0}, "not positive"}};
  for (const Bad& b : bad) {
    const int rc = graph_load_csr(static_cast<int32_t>(b.rp.size()) - 1, static_cast<int64_t>(b.ci.size()), b.rp.data(),
                                  b.ci.data(), b.w.empty() ? nullptr : b.w.data(), GC_VALIDATE, nullptr, &g);
    EXPECT(rc == GC_EINVAL);
    EXPECT(std::strstr(gc_last_error(), b.needle) != nullptr);
  }
  gc_tocab t = nullptr;
  float buf[8] = {};
  EXPECT(tocab_partition(nullptr, GC_PULL, 1 << 12, 0, nullptr, &t) == GC_EINVAL);
  EXPECT(pagerank_iter(nullptr, nullptr, GC_PULL, 0.85f, 0, buf, buf, 1, nullptr) == GC_EINVAL);
  EXPECT(bfs_pull(nullptr, nullptr, 0, reinterpret_cast<int32_t*>(buf), nullptr, 0, nullptr) == GC_EINVAL);
  EXPECT(sssp_pull(nullptr, nullptr, 0, reinterpret_cast<int32_t*>(buf), nullptr, 0, nullptr) == GC_EINVAL);
  EXPECT(graph_free(nullptr) == GC_EINVAL);
  EXPECT(tocab_free(nullptr) == GC_EINVAL);
  EXPECT(graph_info(nullptr, nullptr, nullptr, nullptr) == GC_EINVAL);
  EXPECT(tocab_info(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == GC_EINVAL);
  EXPECT(graph_export_transpose(nullptr, nullptr, nullptr, nullptr, nullptr) == GC_EINVAL);
  EXPECT(tocab_export(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == GC_EINVAL);
  int64_t cnt = 0;
  EXPECT(sched_param_count(3, &cnt) == GC_OK && cnt > 0);
  float f[GC_SCHED_INPUTS];
  EXPECT(sched_features(1 << 20, 16 << 20, 1000, 60000, 3, 0.25f, 50000, f) == GC_OK);
  std::printf("fails %d\n", fails);
  return fails != 0;
}
