/* Multithreaded CPU performance baseline (OpenMP): what the host's cores do
 * with the same workloads, timed beside the GPU path. It is neither the
 * oracle (single-threaded FP64, test infrastructure) nor part of the GPU
 * library, and shares no code with either.
 *
 *   cpub_transpose       in-arc CSR from the out-arc CSR (counting sort,
 *                        rows ascending by source); untimed preprocessing
 *   cpub_pagerank_pull   FP32 PageRank by pulling over in-arcs (Algorithm 1
 *                        with the uniform dangling redistribution), one
 *                        thread team over destination vertices
 *   cpub_bfs             direction-optimising BFS (Beamer et al., alpha 14,
 *                        beta 24): top-down levels expand the frontier queue
 *                        with a compare-and-swap per discovered vertex,
 *                        bottom-up levels scan the in-arcs of unvisited
 *                        vertices against a frontier bitmap
 * Each timed entry returns its wall time in seconds (CLOCK_MONOTONIC). */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int cpub_threads(void) { return omp_get_max_threads(); }

/* t_rowptr[n+1], t_colidx[m]: in-arcs of every vertex, sources ascending
 * (out-rows are visited in source order by one thread per destination
 * range, so each in-row is filled in ascending source order). */
int cpub_transpose(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx, int32_t* t_rowptr,
                   int32_t* t_colidx) {
  int64_t* cnt = calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -1;
  for (int64_t i = 0; i < m; ++i) cnt[colidx[i] + 1]++;
  for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  for (int32_t v = 0; v <= n; ++v) t_rowptr[v] = (int32_t)cnt[v];
  const int nt = omp_get_max_threads();
#pragma omp parallel num_threads(nt)
  {
    /* thread k owns destinations [lo, hi): it walks every source in order
     * and appends the arcs that land in its range */
    const int k = omp_get_thread_num();
    const int32_t lo = (int32_t)((int64_t)n * k / nt), hi = (int32_t)((int64_t)n * (k + 1) / nt);
    for (int32_t u = 0; u < n; ++u)
      for (int32_t i = rowptr[u]; i < rowptr[u + 1]; ++i) {
        const int32_t v = colidx[i];
        if (v >= lo && v < hi) t_colidx[cnt[v]++] = u;
      }
  }
  free(cnt);
  (void)m;
  return 0;
}

/* `iters` iterations from r = 1/n: c[u] = r[u] / outdeg(u) (0 when
 * dangling), D = sum of dangling ranks, r'[v] = (1 - d)/n + d (sum of c
 * over in-arcs + D/n). FP32 values, FP32 row sums (the usual CPU choice). */
double cpub_pagerank_pull(int32_t n, const int32_t* rowptr, const int32_t* t_rowptr, const int32_t* t_colidx,
                          float d, int32_t iters, float* r_out) {
  float* c = malloc(sizeof(float) * (size_t)n);
  float* r = r_out;
  if (!c) return -1.0;
  const float base = (1.0f - d) / (float)n;
#pragma omp parallel for schedule(static)
  for (int32_t v = 0; v < n; ++v) r[v] = 1.0f / (float)n;
  const double t0 = now_s();
  for (int32_t it = 0; it < iters; ++it) {
    double dang = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : dang)
    for (int32_t u = 0; u < n; ++u) {
      const int32_t deg = rowptr[u + 1] - rowptr[u];
      c[u] = deg ? r[u] / (float)deg : 0.0f;
      if (!deg) dang += r[u];
    }
    const float dn = (float)(dang / n);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; ++v) {
      float s = 0.0f;
      for (int32_t i = t_rowptr[v]; i < t_rowptr[v + 1]; ++i) s += c[t_colidx[i]];
      r[v] = base + d * (s + dn);
    }
  }
  const double t = now_s() - t0;
  free(c);
  return t;
}

/* depth[n] out (INT32_MAX when unreachable). */
double cpub_bfs(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx, const int32_t* t_rowptr,
                const int32_t* t_colidx, int32_t source, int32_t* depth) {
  const int32_t kInf = INT32_MAX;
  int32_t* q = malloc(sizeof(int32_t) * (size_t)n);
  int32_t* qn = malloc(sizeof(int32_t) * (size_t)n);
  const int64_t words = ((int64_t)n + 63) / 64;
  uint64_t* front = calloc((size_t)words, sizeof(uint64_t));
  uint64_t* next = calloc((size_t)words, sizeof(uint64_t));
  if (!q || !qn || !front || !next) {
    free(q), free(qn), free(front), free(next);
    return -1.0;
  }
  const double t0 = now_s();
#pragma omp parallel for schedule(static)
  for (int32_t v = 0; v < n; ++v) depth[v] = kInf;
  depth[source] = 0;
  q[0] = source;
  int64_t nq = 1;
  int64_t mf = rowptr[source + 1] - rowptr[source];
  int64_t mu = m - mf;
  int bottom_up = 0;
  for (int32_t level = 0; nq > 0; ++level) {
    if (!bottom_up && (double)mf > (double)mu / 14.0) bottom_up = 1;
    else if (bottom_up && (double)nq < (double)n / 24.0) bottom_up = 0;
    int64_t nn = 0, nmf = 0;
    if (bottom_up) {
      memset(front, 0, sizeof(uint64_t) * (size_t)words);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < nq; ++i) __atomic_fetch_or(&front[q[i] >> 6], 1ull << (q[i] & 63), __ATOMIC_RELAXED);
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : nn, nmf)
      for (int32_t v = 0; v < n; ++v) {
        if (depth[v] != kInf) continue;
        for (int32_t i = t_rowptr[v]; i < t_rowptr[v + 1]; ++i) {
          const int32_t u = t_colidx[i];
          if ((front[u >> 6] >> (u & 63)) & 1) {
            depth[v] = level + 1;
            ++nn;
            nmf += rowptr[v + 1] - rowptr[v];
            break;
          }
        }
      }
      /* the next frontier as a queue, in vertex order */
      int64_t w = 0;
      for (int32_t v = 0; v < n; ++v)
        if (depth[v] == level + 1) qn[w++] = v;
      nn = w;
    } else {
#pragma omp parallel reduction(+ : nmf)
      {
        int32_t local[1024];
        int nl = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < nq; ++i) {
          const int32_t u = q[i];
          for (int32_t j = rowptr[u]; j < rowptr[u + 1]; ++j) {
            const int32_t v = colidx[j];
            int32_t expect = kInf;
            if (depth[v] == kInf &&
                __atomic_compare_exchange_n(&depth[v], &expect, level + 1, 0, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
              local[nl++] = v;
              nmf += rowptr[v + 1] - rowptr[v];
              if (nl == 1024) {
                const int64_t at = __atomic_fetch_add(&nn, (int64_t)nl, __ATOMIC_RELAXED);
                memcpy(qn + at, local, sizeof(int32_t) * (size_t)nl);
                nl = 0;
              }
            }
          }
        }
        if (nl) {
          const int64_t at = __atomic_fetch_add(&nn, (int64_t)nl, __ATOMIC_RELAXED);
          memcpy(qn + at, local, sizeof(int32_t) * (size_t)nl);
        }
      }
    }
    int32_t* tq = q;
    q = qn;
    qn = tq;
    nq = nn;
    mu -= nmf;
    mf = nmf;
  }
  const double t = now_s() - t0;
  free(q), free(qn), free(front), free(next);
  return t;
}
