/*
 * CPU oracle for GraphCage / TOCAB ("GraphCage: Cache Aware Graph Processing
 * on GPUs", Chen 2019). TEST INFRASTRUCTURE ONLY: nothing outside tests/, the
 * smoke check and the benchmark's CPU-baseline leg may load this library, and
 * the GPU library shares no code with it.
 *
 * Plain, single-threaded, obviously correct definitions in FP64 / int64.
 * Every graph is an out-edge CSR: rowptr[n+1], colidx[m]; arc u -> colidx[j]
 * for j in [rowptr[u], rowptr[u+1]).
 *
 * Build: gcc -O2 -std=c11 -shared -fPIC (oracle/build.py).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_INF32 INT32_MAX

/* ------------------------------------------------------------------------ */
/* PageRank (Section 2.2, Algorithm 1: pull; Algorithm 2: push).
 *
 * Per iteration:
 *   c[u]  = r[u] / outdeg[u]             (outdeg[u] > 0; else 0)
 *   s[v]  = sum over arcs u -> v of c[u]
 *   r'[v] = (1 - d)/N + d * s[v]                       mode 1 (LEAK)
 *   r'[v] = (1 - d)/N + d * (s[v] + D/N),  D = sum of r over outdeg 0
 *                                                       mode 0 (UNIFORM)
 * The paper's update is the LEAK line; it never says what happens to the
 * rank of vertices without out-arcs. UNIFORM spreads it evenly, which keeps
 * sum(r) = 1. r0 is given by the caller. The sum s[v] is formed by scattering
 * over out-arcs, which is the same set of terms Algorithm 1 gathers. */
int oracle_pagerank(int32_t n, const int32_t* rowptr, const int32_t* colidx, double d,
                    int32_t mode, int32_t iters, const double* r0, double* r_out) {
  if (n <= 0 || iters < 0 || (mode != 0 && mode != 1)) return -1;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* s = (double*)malloc(sizeof(double) * (size_t)n);
  if (!r || !s) { free(r); free(s); return -2; }
  memcpy(r, r0, sizeof(double) * (size_t)n);
  for (int32_t t = 0; t < iters; ++t) {
    double dangling = 0.0;
    for (int32_t v = 0; v < n; ++v) s[v] = 0.0;
    for (int32_t u = 0; u < n; ++u) {
      const int32_t deg = rowptr[u + 1] - rowptr[u];
      if (deg == 0) { dangling += r[u]; continue; }
      const double c = r[u] / (double)deg;
      for (int32_t j = rowptr[u]; j < rowptr[u + 1]; ++j) s[colidx[j]] += c;
    }
    for (int32_t v = 0; v < n; ++v) {
      const double extra = (mode == 0) ? dangling / (double)n : 0.0;
      r[v] = (1.0 - d) / (double)n + d * (s[v] + extra);
    }
  }
  memcpy(r_out, r, sizeof(double) * (size_t)n);
  free(r);
  free(s);
  return 0;
}

/* Personalised PageRank: teleport and dangling mass both go to the
 * personalisation vector p (sum p = 1):
 *   r'[v] = (1 - d) * p[v] + d * (s[v] + D * p[v]),   r0 = p. */
int oracle_ppr(int32_t n, const int32_t* rowptr, const int32_t* colidx, double d, int32_t iters,
               const double* p, double* r_out) {
  if (n <= 0 || iters < 0) return -1;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* s = (double*)malloc(sizeof(double) * (size_t)n);
  if (!r || !s) { free(r); free(s); return -2; }
  memcpy(r, p, sizeof(double) * (size_t)n);
  for (int32_t t = 0; t < iters; ++t) {
    double dangling = 0.0;
    for (int32_t v = 0; v < n; ++v) s[v] = 0.0;
    for (int32_t u = 0; u < n; ++u) {
      const int32_t deg = rowptr[u + 1] - rowptr[u];
      if (deg == 0) { dangling += r[u]; continue; }
      const double c = r[u] / (double)deg;
      for (int32_t j = rowptr[u]; j < rowptr[u + 1]; ++j) s[colidx[j]] += c;
    }
    for (int32_t v = 0; v < n; ++v) r[v] = (1.0 - d) * p[v] + d * (s[v] + dangling * p[v]);
  }
  memcpy(r_out, r, sizeof(double) * (size_t)n);
  free(r);
  free(s);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Breadth-first search over out-arcs with a FIFO queue (the frontier queue of
 * Section 2.1). depth[source] = 0, unreached = INT32_MAX. */
int oracle_bfs(int32_t n, const int32_t* rowptr, const int32_t* colidx, int32_t source,
               int32_t* depth) {
  if (n <= 0 || source < 0 || source >= n) return -1;
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return -2;
  for (int32_t v = 0; v < n; ++v) depth[v] = ORACLE_INF32;
  int32_t head = 0, tail = 0;
  depth[source] = 0;
  queue[tail++] = source;
  while (head < tail) {
    const int32_t u = queue[head++];
    for (int32_t j = rowptr[u]; j < rowptr[u + 1]; ++j) {
      const int32_t v = colidx[j];
      if (depth[v] == ORACLE_INF32) {
        depth[v] = depth[u] + 1;
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Dijkstra's algorithm with a binary min-heap keyed by tentative distance
 * (lazy deletion), int64 distances, positive weights. Unreached vertices get
 * INT32_MAX; returns -3 if a finite distance does not fit below INT32_MAX. */
typedef struct { int64_t key; int32_t v; } heap_item;

static void heap_push(heap_item* h, int64_t* size, heap_item x) {
  int64_t i = (*size)++;
  h[i] = x;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].key <= h[i].key) break;
    heap_item t = h[p]; h[p] = h[i]; h[i] = t;
    i = p;
  }
}

static heap_item heap_pop(heap_item* h, int64_t* size) {
  heap_item top = h[0];
  h[0] = h[--(*size)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < *size && h[l].key < h[m].key) m = l;
    if (r < *size && h[r].key < h[m].key) m = r;
    if (m == i) break;
    heap_item t = h[m]; h[m] = h[i]; h[i] = t;
    i = m;
  }
  return top;
}

int oracle_dijkstra(int32_t n, const int32_t* rowptr, const int32_t* colidx, const int32_t* w,
                    int32_t source, int32_t* dist) {
  if (n <= 0 || source < 0 || source >= n) return -1;
  const int64_t m = rowptr[n];
  for (int64_t j = 0; j < m; ++j)
    if (w[j] <= 0) return -1;
  int64_t* best = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  heap_item* heap = (heap_item*)malloc(sizeof(heap_item) * (size_t)(m + 1));
  if (!best || !heap) { free(best); free(heap); return -2; }
  for (int32_t v = 0; v < n; ++v) best[v] = INT64_MAX;
  int64_t size = 0;
  best[source] = 0;
  heap_item s0 = {0, source};
  heap_push(heap, &size, s0);
  while (size > 0) {
    heap_item it = heap_pop(heap, &size);
    if (it.key != best[it.v]) continue; /* stale entry */
    const int32_t u = it.v;
    for (int32_t j = rowptr[u]; j < rowptr[u + 1]; ++j) {
      const int32_t v = colidx[j];
      const int64_t nd = best[u] + (int64_t)w[j];
      if (nd < best[v]) {
        best[v] = nd;
        heap_item x = {nd, v};
        heap_push(heap, &size, x);
      }
    }
  }
  int rc = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (best[v] == INT64_MAX) dist[v] = ORACLE_INF32;
    else if (best[v] >= (int64_t)ORACLE_INF32) { dist[v] = ORACLE_INF32; rc = -3; }
    else dist[v] = (int32_t)best[v];
  }
  free(best);
  free(heap);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Transpose of a CSR: arc u -> v becomes row v, column u. Filling rows in
 * ascending u keeps every transposed row sorted by column. */
int oracle_transpose(int32_t n, const int32_t* rowptr, const int32_t* colidx, const int32_t* w,
                     int32_t* t_rowptr, int32_t* t_colidx, int32_t* t_w) {
  if (n <= 0) return -1;
  const int64_t m = rowptr[n];
  int64_t* cur = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cur) return -2;
  for (int64_t j = 0; j < m; ++j) cur[colidx[j] + 1]++;
  for (int32_t v = 0; v < n; ++v) cur[v + 1] += cur[v];
  for (int32_t v = 0; v <= n; ++v) t_rowptr[v] = (int32_t)cur[v];
  for (int32_t u = 0; u < n; ++u) {
    for (int32_t j = rowptr[u]; j < rowptr[u + 1]; ++j) {
      const int32_t v = colidx[j];
      const int64_t pos = cur[v]++;
      t_colidx[pos] = u;
      if (w && t_w) t_w[pos] = w[j];
    }
  }
  free(cur);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* TOCAB static 1D partition (Section 3.1, "preprocessing phase").
 *
 * Input: a CSR A with n_rows rows whose columns lie in [0, n_cols) and are
 * sorted within each row. For pull, A is the transposed graph (row = dst,
 * column = src) and the blocks are column blocks; for push, A is the graph
 * itself (row = src, column = dst) and the same code does row blocking.
 *
 * Block s holds every arc whose column c has floor(c / W) = s; there are
 * B = ceil(n_cols / W) blocks. Only rows with at least one arc in block s get
 * a local ID in it, in ascending order of their global row id; id_map gives
 * the global id back. All blocks are concatenated (block-major):
 *   blk_rowoff[s]  first local row of block s (int64[B+1]; total P)
 *   row_ptr[l]     first arc of local row l   (int64[P+1])
 *   id_map[l]      global row id of local row l (int32[P])
 *   col[e], wout[e] column and weight of arc e (int32[m]) in that order
 *   range_ptr[s*(R+1)+j] first local row of block s whose global id is
 *                  >= j*k, R = ceil(n_rows / k) (int64[B*(R+1)]); it cuts
 *                  each block into the merge ranges of width k.
 * Sizes: call with the output pointers NULL to get B and P only. */
int oracle_partition(int32_t n_rows, int32_t n_cols, const int32_t* rowptr, const int32_t* colidx,
                     const int32_t* w, int32_t W, int32_t k, int64_t* out_B, int64_t* out_P,
                     int64_t* blk_rowoff, int64_t* row_ptr, int32_t* id_map, int32_t* col,
                     int32_t* wout, int64_t* range_ptr) {
  if (n_rows <= 0 || n_cols <= 0 || W <= 0 || k <= 0) return -1;
  const int64_t B = ((int64_t)n_cols + W - 1) / W;
  const int64_t R = ((int64_t)n_rows + k - 1) / k;
  int64_t* rows_in = (int64_t*)calloc((size_t)B, sizeof(int64_t));
  int64_t* arcs_in = (int64_t*)calloc((size_t)B, sizeof(int64_t));
  if (!rows_in || !arcs_in) { free(rows_in); free(arcs_in); return -2; }
  /* count local rows and arcs per block */
  for (int32_t r = 0; r < n_rows; ++r) {
    int64_t last = -1;
    for (int32_t j = rowptr[r]; j < rowptr[r + 1]; ++j) {
      const int64_t s = colidx[j] / W;
      if (s != last) { rows_in[s]++; last = s; }
      arcs_in[s]++;
    }
  }
  int64_t P = 0;
  for (int64_t s = 0; s < B; ++s) P += rows_in[s];
  *out_B = B;
  *out_P = P;
  if (!blk_rowoff) { free(rows_in); free(arcs_in); return 0; }

  int64_t* row_cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)B);
  int64_t* arc_cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)B);
  if (!row_cur || !arc_cur) { free(rows_in); free(arcs_in); free(row_cur); free(arc_cur); return -2; }
  blk_rowoff[0] = 0;
  int64_t arcs_before = 0;
  for (int64_t s = 0; s < B; ++s) {
    blk_rowoff[s + 1] = blk_rowoff[s] + rows_in[s];
    row_cur[s] = blk_rowoff[s];
    arc_cur[s] = arcs_before;
    arcs_before += arcs_in[s];
  }
  /* rows are visited in ascending global id, so local ids come out ascending */
  for (int32_t r = 0; r < n_rows; ++r) {
    int64_t last = -1;
    for (int32_t j = rowptr[r]; j < rowptr[r + 1]; ++j) {
      const int64_t s = colidx[j] / W;
      if (s != last) {
        const int64_t l = row_cur[s]++;
        id_map[l] = r;
        row_ptr[l] = arc_cur[s];
        last = s;
      }
      col[arc_cur[s]] = colidx[j];
      if (w && wout) wout[arc_cur[s]] = w[j];
      arc_cur[s]++;
    }
  }
  row_ptr[P] = arcs_before;
  /* merge-range cuts: lower bound of j*k in each block's id_map */
  for (int64_t s = 0; s < B; ++s) {
    int64_t l = blk_rowoff[s];
    for (int64_t j = 0; j <= R; ++j) {
      const int64_t lo = j * (int64_t)k;
      while (l < blk_rowoff[s + 1] && (int64_t)id_map[l] < lo) ++l;
      range_ptr[s * (R + 1) + j] = l;
    }
  }
  free(rows_in);
  free(arcs_in);
  free(row_cur);
  free(arc_cur);
  return 0;
}
