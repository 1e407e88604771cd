// Memory and undefined-behaviour check of the graph generators: each
// generator at small sizes (including degenerate ones), exported, checked
// for a well-formed CSR, then weights and sources drawn over it. Built
// with AddressSanitizer and UBSan by tests/test_host_sanitizers.py; exits
// non-zero on a malformed graph.
#include <cstdint>
#include <cstdio>
#include <vector>

struct gg_csr;
extern "C" {
gg_csr* gg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, uint64_t seed,
                int32_t permute);
gg_csr* gg_grid(int32_t rows, int32_t cols, double p_rewire, uint64_t seed);
gg_csr* gg_uniform(int32_t n, int64_t m, uint64_t seed);
gg_csr* gg_from_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, int32_t symmetrize);
int32_t gg_n(const gg_csr* g);
int64_t gg_m(const gg_csr* g);
void gg_export(const gg_csr* g, int32_t* rowptr, int32_t* colidx);
void gg_free(gg_csr* g);
void gg_weights(int32_t n, const int32_t* rowptr, const int32_t* colidx, uint64_t seed, int32_t undirected,
                int32_t* w);
int32_t gg_sources(int32_t n, const int32_t* rowptr, uint64_t seed, int32_t count, int32_t* out);
}

static int check(gg_csr* g, const char* what) {
  if (!g) {
    std::printf("%s: no graph\n", what);
    return 1;
  }
  const int32_t n = gg_n(g);
  const int64_t m = gg_m(g);
  std::vector<int32_t> rowptr(static_cast<size_t>(n) + 1), col(static_cast<size_t>(m) + 1), w(static_cast<size_t>(m) + 1);
  gg_export(g, rowptr.data(), col.data());
  int bad = rowptr[0] != 0 || rowptr[n] != m;
  for (int32_t v = 0; v < n; ++v) bad |= rowptr[v + 1] < rowptr[v];
  for (int64_t e = 0; e < m; ++e) bad |= col[e] < 0 || col[e] >= n;
  gg_weights(n, rowptr.data(), col.data(), 7, 1, w.data());
  for (int64_t e = 0; e < m; ++e) bad |= w[e] < 1 || w[e] > 255;
  std::vector<int32_t> src(8);
  const int32_t found = gg_sources(n, rowptr.data(), 3, 8, src.data());
  for (int32_t k = 0; k < found; ++k) bad |= src[k] < 0 || src[k] >= n || rowptr[src[k] + 1] == rowptr[src[k]];
  gg_free(g);
  if (bad) std::printf("%s: malformed\n", what);
  return bad;
}

int main() {
  int fails = 0;
  for (int32_t scale = 1; scale <= 12; ++scale) fails += check(gg_rmat(scale, 1 + scale % 8, 0.57, 0.19, 0.19, scale, scale & 1), "rmat");
  for (int32_t r = 1; r <= 40; r += 13)
    for (int32_t c = 1; c <= 40; c += 7) fails += check(gg_grid(r, c, 0.05 * (r % 3), r * 100 + c), "grid");
  for (int32_t n = 1; n <= 2000; n = 3 * n + 1) fails += check(gg_uniform(n, 4 * static_cast<int64_t>(n), n), "uniform");
  fails += check(gg_uniform(5, 0, 1), "uniform, no edges");
  const int32_t s[] = {0, 1, 2, 2, 3}, d[] = {1, 2, 0, 2, 3};
  fails += check(gg_from_edges(4, 5, s, d, 1), "edges");
  fails += check(gg_from_edges(4, 5, s, d, 0), "edges, directed");
  std::printf("fails %d\n", fails);
  return fails != 0;
}
