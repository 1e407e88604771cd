/* Memory and undefined-behaviour check of the OpenMP CPU baseline: random
 * small graphs (up to 400 vertices, some without arcs) through the
 * transpose, the FP32 pull PageRank and the direction-optimising BFS.
 * Built with AddressSanitizer and UBSan by tests/test_host_sanitizers.py;
 * exits non-zero if a call fails or a result is malformed. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int cpub_transpose(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx, int32_t* t_rowptr,
                   int32_t* t_colidx);
double cpub_pagerank_pull(int32_t n, const int32_t* rowptr, const int32_t* t_rowptr, const int32_t* t_colidx,
                          float d, int32_t iters, float* r_out);
double cpub_bfs(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx, const int32_t* t_rowptr,
                const int32_t* t_colidx, int32_t source, int32_t* depth);

/* xorshift64 (Marsaglia), fixed seed */
static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return (uint32_t)s; }

int main(void) {
  int fails = 0;
  for (int trial = 0; trial < 100; ++trial) {
    const int32_t n = 1 + rnd() % 400;
    const int32_t deg = rnd() % 12;
    int32_t* rowptr = malloc(sizeof(int32_t) * ((size_t)n + 1));
    rowptr[0] = 0;
    for (int32_t v = 0; v < n; ++v) rowptr[v + 1] = rowptr[v] + (deg ? (int32_t)(rnd() % (2 * deg + 1)) : 0);
    const int64_t m = rowptr[n];
    int32_t* col = malloc(sizeof(int32_t) * ((size_t)m + 1));
    for (int64_t e = 0; e < m; ++e) col[e] = rnd() % n;
    int32_t* trp = malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t* tc = malloc(sizeof(int32_t) * ((size_t)m + 1));
    float* r = malloc(sizeof(float) * (size_t)n);
    int32_t* depth = malloc(sizeof(int32_t) * (size_t)n);
    fails += cpub_transpose(n, m, rowptr, col, trp, tc) != 0;
    fails += trp[n] != m;
    fails += cpub_pagerank_pull(n, rowptr, trp, tc, 0.85f, 5, r) < 0.0;
    const int32_t src = rnd() % n;
    fails += cpub_bfs(n, m, rowptr, col, trp, tc, src, depth) < 0.0;
    fails += depth[src] != 0;
    free(rowptr); free(col); free(trp); free(tc); free(r); free(depth);
  }
  printf("fails %d\n", fails);
  return fails != 0;
}
