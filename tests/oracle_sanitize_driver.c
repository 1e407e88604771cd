/* Memory and undefined-behaviour check of the C oracle: random small
 * graphs (up to 300 vertices, mean out-degree up to 8, weights in
 * [1, 255]) through every oracle entry point, including the partition's
 * two-call size protocol. Built with AddressSanitizer and UBSan by
 * tests/test_host_sanitizers.py; exits non-zero if a call fails. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int oracle_pagerank(int32_t n, const int32_t* rowptr, const int32_t* colidx, double d, int32_t mode, int32_t iters, const double* r0, double* r_out);
int oracle_ppr(int32_t n, const int32_t* rowptr, const int32_t* colidx, double d, int32_t iters, const double* p, double* r_out);
int oracle_bfs(int32_t n, const int32_t* rowptr, const int32_t* colidx, int32_t source, int32_t* depth);
int oracle_dijkstra(int32_t n, const int32_t* rowptr, const int32_t* colidx, const int32_t* w, int32_t source, int32_t* dist);
int oracle_transpose(int32_t n, const int32_t* rowptr, const int32_t* colidx, const int32_t* w, int32_t* t_rowptr, int32_t* t_colidx, int32_t* t_w);
int oracle_partition(int32_t n_rows, int32_t n_cols, const int32_t* rowptr, const int32_t* colidx, const int32_t* w, int32_t W, int32_t k, int64_t* out_B, int64_t* out_P, int64_t* blk_rowoff, int64_t* row_ptr, int32_t* id_map, int32_t* col, int32_t* wout, int64_t* range_ptr);
/* xorshift64 (Marsaglia), fixed seed */
static uint64_t s = 88172645463325252ull;
static uint32_t rnd(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return (uint32_t)s; }
int main(void) {
  int fails = 0;
  for (int trial = 0; trial < 200; ++trial) {
    const int32_t n = 1 + rnd() % 300;
    const int32_t deg = rnd() % 9;
    int32_t* rowptr = malloc(sizeof(int32_t) * (n + 1));
    rowptr[0] = 0;
    for (int32_t v = 0; v < n; ++v) rowptr[v + 1] = rowptr[v] + (deg ? (int32_t)(rnd() % (2 * deg + 1)) : 0);
    const int32_t m = rowptr[n];
    int32_t* col = malloc(sizeof(int32_t) * (m + 1));
    int32_t* w = malloc(sizeof(int32_t) * (m + 1));
    for (int32_t e = 0; e < m; ++e) { col[e] = rnd() % n; w[e] = 1 + rnd() % 255; }
    double* r0 = malloc(sizeof(double) * n); double* r = malloc(sizeof(double) * n);
    for (int32_t v = 0; v < n; ++v) r0[v] = 1.0 / n;
    fails += oracle_pagerank(n, rowptr, col, 0.85, trial & 1, 5, r0, r) != 0;
    fails += oracle_ppr(n, rowptr, col, 0.85, 5, r0, r) != 0;
    int32_t* d = malloc(sizeof(int32_t) * n);
    const int32_t src = rnd() % n;
    fails += oracle_bfs(n, rowptr, col, src, d) != 0;
    fails += oracle_dijkstra(n, rowptr, col, w, src, d) != 0;
    int32_t* trp = malloc(sizeof(int32_t) * (n + 1)); int32_t* tc = malloc(sizeof(int32_t) * (m + 1)); int32_t* tw = malloc(sizeof(int32_t) * (m + 1));
    fails += oracle_transpose(n, rowptr, col, w, trp, tc, tw) != 0;
    const int32_t W = 1 << (rnd() % 9), k = 1 + rnd() % 64;
    int64_t B = 0, P = 0;
    fails += oracle_partition(n, n, trp, tc, tw, W, k, &B, &P, NULL, NULL, NULL, NULL, NULL, NULL) != 0;
    const int64_t R = (n + k - 1) / k;
    int64_t* blk = malloc(sizeof(int64_t) * (B + 1)); int64_t* rp = malloc(sizeof(int64_t) * (P + 1));
    int32_t* idm = malloc(sizeof(int32_t) * (P + 1)); int32_t* pc = malloc(sizeof(int32_t) * (m + 1));
    int32_t* pw = malloc(sizeof(int32_t) * (m + 1)); int64_t* rg = malloc(sizeof(int64_t) * (B * (R + 1) + 1));
    fails += oracle_partition(n, n, trp, tc, tw, W, k, &B, &P, blk, rp, idm, pc, pw, rg) != 0;
    free(blk); free(rp); free(idm); free(pc); free(pw); free(rg);
    free(trp); free(tc); free(tw); free(d); free(r0); free(r); free(rowptr); free(col); free(w);
  }
  printf("fails %d\n", fails);
  return fails != 0;
}
