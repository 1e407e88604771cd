// Seeded synthetic graph generators and the edge-list -> CSR builder.
//
// This module only manufactures inputs. It holds none of the graph method's
// arithmetic (no ranks, no traversal, no blocking) and is shared by the CPU
// oracle and the GPU path alike, which both consume the out-edge CSR it emits.
//
// Randomness is counter based: draw(seed, i) is the i-th output of the
// SplitMix64 generator (Steele, Lea & Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014) started from state `seed`, i.e.
//   z = seed + (i + 1) * 0x9E3779B97F4A7C15, followed by its output mix.
// Every random choice is a pure function of (seed, index), so the output is
// identical for any thread count.
//
// Build: g++ -O3 -fopenmp -shared -fPIC (see graphgen/build.py).

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include <omp.h>

namespace {

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline uint64_t draw(uint64_t seed, uint64_t i) {
  return mix64(seed + (i + 1) * 0x9E3779B97F4A7C15ull);
}

struct Csr {
  int32_t n = 0;
  int64_t m = 0;
  std::vector<int32_t> rowptr;  // n + 1 (int32: m must stay below 2^31)
  std::vector<int32_t> colidx;  // m
};

// Builds a deduplicated, self-loop-free CSR with rows sorted ascending from an
// edge source that is a pure function of the edge index:
//   edge(e, &u, &v) -> false if the edge is dropped.
// Two passes regenerate the edges instead of storing the edge list.
template <class EdgeFn>
Csr build_csr(int32_t n, int64_t num_edges, bool symmetrize, EdgeFn edge) {
  Csr g;
  g.n = n;
  std::vector<std::atomic<int64_t>> cnt(static_cast<size_t>(n) + 1);
  for (auto& c : cnt) c.store(0, std::memory_order_relaxed);

#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < num_edges; ++e) {
    int32_t u, v;
    if (!edge(e, u, v) || u == v) continue;
    cnt[u].fetch_add(1, std::memory_order_relaxed);
    if (symmetrize) cnt[v].fetch_add(1, std::memory_order_relaxed);
  }
  std::vector<int64_t> start(static_cast<size_t>(n) + 1, 0);
  for (int32_t i = 0; i < n; ++i) start[i + 1] = start[i] + cnt[i].load();
  const int64_t raw = start[n];
  std::vector<int32_t> tmp(static_cast<size_t>(raw));
  for (int32_t i = 0; i < n; ++i) cnt[i].store(start[i], std::memory_order_relaxed);

#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < num_edges; ++e) {
    int32_t u, v;
    if (!edge(e, u, v) || u == v) continue;
    tmp[cnt[u].fetch_add(1, std::memory_order_relaxed)] = v;
    if (symmetrize) tmp[cnt[v].fetch_add(1, std::memory_order_relaxed)] = u;
  }

  // Sort and deduplicate each row; the result no longer depends on the
  // (racy) order in which the scatter above filled a row.
  std::vector<int64_t> kept(static_cast<size_t>(n) + 1, 0);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t i = 0; i < n; ++i) {
    int32_t* b = tmp.data() + start[i];
    int32_t* e = tmp.data() + start[i + 1];
    std::sort(b, e);
    kept[i + 1] = std::unique(b, e) - b;
  }
  for (int32_t i = 0; i < n; ++i) kept[i + 1] += kept[i];
  g.m = kept[n];
  g.rowptr.resize(static_cast<size_t>(n) + 1);
  g.colidx.resize(static_cast<size_t>(g.m));
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t i = 0; i < n; ++i) {
    const int64_t len = kept[i + 1] - kept[i];
    // (an empty row copies nothing: with no arcs at all colidx has no storage)
    if (len) std::memcpy(g.colidx.data() + kept[i], tmp.data() + start[i], len * sizeof(int32_t));
  }
  for (int32_t i = 0; i <= n; ++i) g.rowptr[i] = static_cast<int32_t>(kept[i]);
  return g;
}

// Seeded uniform random permutation of [0, n) by Fisher-Yates (Knuth,
// TAOCP vol. 2, Algorithm P) fed by the counter-based stream.
std::vector<int32_t> permutation(int32_t n, uint64_t seed) {
  std::vector<int32_t> p(n);
  for (int32_t i = 0; i < n; ++i) p[i] = i;
  for (int64_t i = n - 1; i > 0; --i) {
    const int64_t j = static_cast<int64_t>(draw(seed, static_cast<uint64_t>(i)) %
                                           static_cast<uint64_t>(i + 1));
    std::swap(p[i], p[j]);
  }
  return p;
}

}  // namespace

extern "C" {

struct gg_csr {
  Csr g;
};

// Recursive-matrix (R-MAT) generator (Chakrabarti, Zhan & Faloutsos, SDM
// 2004): 2^scale vertices, edge_factor * 2^scale generated arcs. For every arc
// and every one of the `scale` recursion levels a quadrant is drawn with
// probabilities (a, b, c, 1-a-b-c); the quadrant supplies one bit of the
// source (row) and one of the destination (column). No parameter noise.
// Labels are then relabelled by a seeded random permutation when `permute`
// is set; self-loops and duplicate arcs are dropped. Directed.
gg_csr* gg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c,
                uint64_t seed, int32_t permute) {
  if (scale < 1 || scale > 30 || edge_factor < 1) return nullptr;
  const int32_t n = int32_t(1) << scale;
  const int64_t m = static_cast<int64_t>(edge_factor) << scale;
  const double two32 = 4294967296.0;
  const uint64_t ta = static_cast<uint64_t>(a * two32);
  const uint64_t tab = static_cast<uint64_t>((a + b) * two32);
  const uint64_t tabc = static_cast<uint64_t>((a + b + c) * two32);
  std::vector<int32_t> perm;
  const uint64_t edge_seed = draw(seed, 0);
  if (permute) perm = permutation(n, draw(seed, 1));
  const int32_t* pm = permute ? perm.data() : nullptr;
  auto edge = [=](int64_t e, int32_t& u, int32_t& v) {
    uint32_t su = 0, sv = 0;
    uint64_t h = 0;
    for (int32_t lvl = 0; lvl < scale; ++lvl) {
      if ((lvl & 1) == 0) h = draw(edge_seed, (static_cast<uint64_t>(e) << 4) | (lvl >> 1));
      const uint64_t r = (lvl & 1) ? (h >> 32) : (h & 0xFFFFFFFFull);
      // quadrants in order a: (0,0), b: (0,1), c: (1,0), d: (1,1); written
      // without branches since the draw is unpredictable by construction
      const uint32_t bu = static_cast<uint32_t>(r >= tab);
      const uint32_t bv = static_cast<uint32_t>((r >= ta) & (r < tab)) |
                          static_cast<uint32_t>(r >= tabc);
      su = (su << 1) | bu;
      sv = (sv << 1) | bv;
    }
    u = pm ? pm[su] : static_cast<int32_t>(su);
    v = pm ? pm[sv] : static_cast<int32_t>(sv);
    return true;
  };
  gg_csr* out = new (std::nothrow) gg_csr;
  if (!out) return nullptr;
  out->g = build_csr(n, m, false, edge);
  return out;
}

// rows x cols 4-neighbour lattice without wrap-around, vertex (r, c) has id
// r * cols + c. Every undirected lattice edge independently (probability
// p_rewire) has its second endpoint replaced by a uniform random vertex.
// Stored symmetrically (both arcs); self-loops and duplicates dropped.
gg_csr* gg_grid(int32_t rows, int32_t cols, double p_rewire, uint64_t seed) {
  if (rows < 1 || cols < 1) return nullptr;
  const int64_t n64 = static_cast<int64_t>(rows) * cols;
  if (n64 >= (int64_t(1) << 31)) return nullptr;
  const int32_t n = static_cast<int32_t>(n64);
  const int64_t horiz = static_cast<int64_t>(rows) * (cols - 1);
  const int64_t vert = static_cast<int64_t>(rows - 1) * cols;
  const uint64_t thr = static_cast<uint64_t>(p_rewire * 18446744073709551616.0);
  const bool always = p_rewire >= 1.0;
  auto edge = [=](int64_t e, int32_t& u, int32_t& v) {
    int64_t x, y;
    if (e < horiz) {
      const int64_t r = e / (cols - 1), c = e % (cols - 1);
      x = r * cols + c;
      y = x + 1;
    } else {
      const int64_t f = e - horiz;
      const int64_t r = f / cols, c = f % cols;
      x = r * cols + c;
      y = x + cols;
    }
    const uint64_t d = draw(seed, 2 * static_cast<uint64_t>(e));
    if (always || d < thr) y = static_cast<int64_t>(draw(seed, 2 * static_cast<uint64_t>(e) + 1) % n);
    u = static_cast<int32_t>(x);
    v = static_cast<int32_t>(y);
    return true;
  };
  gg_csr* out = new (std::nothrow) gg_csr;
  if (!out) return nullptr;
  out->g = build_csr(n, horiz + vert, true, edge);
  return out;
}

// Uniform random graph: m undirected edges with independent uniform
// endpoints over n vertices, stored symmetrically; self-loops and duplicates
// dropped.
gg_csr* gg_uniform(int32_t n, int64_t m, uint64_t seed) {
  if (n < 1 || m < 0) return nullptr;
  auto edge = [=](int64_t e, int32_t& u, int32_t& v) {
    u = static_cast<int32_t>(draw(seed, 2 * static_cast<uint64_t>(e)) % static_cast<uint64_t>(n));
    v = static_cast<int32_t>(draw(seed, 2 * static_cast<uint64_t>(e) + 1) % static_cast<uint64_t>(n));
    return true;
  };
  gg_csr* out = new (std::nothrow) gg_csr;
  if (!out) return nullptr;
  out->g = build_csr(n, m, true, edge);
  return out;
}

// CSR from an explicit edge list (test fixtures). Arcs u -> v; with
// `symmetrize` both directions are stored. Out-of-range endpoints are an
// error (returns NULL).
gg_csr* gg_from_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                      int32_t symmetrize) {
  if (n < 1 || m < 0) return nullptr;
  for (int64_t e = 0; e < m; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return nullptr;
  auto edge = [=](int64_t e, int32_t& u, int32_t& v) {
    u = src[e];
    v = dst[e];
    return true;
  };
  gg_csr* out = new (std::nothrow) gg_csr;
  if (!out) return nullptr;
  out->g = build_csr(n, m, symmetrize != 0, edge);
  return out;
}

int32_t gg_n(const gg_csr* g) { return g->g.n; }
int64_t gg_m(const gg_csr* g) { return g->g.m; }

void gg_export(const gg_csr* g, int32_t* rowptr, int32_t* colidx) {
  std::memcpy(rowptr, g->g.rowptr.data(), (static_cast<size_t>(g->g.n) + 1) * sizeof(int32_t));
  if (g->g.m) std::memcpy(colidx, g->g.colidx.data(), static_cast<size_t>(g->g.m) * sizeof(int32_t));
}

void gg_free(gg_csr* g) { delete g; }

// Arc weights in [1, 255]: w(u, v) = 1 + draw(seed, key) mod 255 with
// key = (min(u,v) << 32) | max(u,v) when `undirected` (both arcs of an edge
// get the same weight) and key = (u << 32) | v otherwise. Written in the
// order of the given CSR's arcs.
void gg_weights(int32_t n, const int32_t* rowptr, const int32_t* colidx, uint64_t seed,
                int32_t undirected, int32_t* w) {
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t u = 0; u < n; ++u) {
    for (int64_t j = rowptr[u]; j < rowptr[u + 1]; ++j) {
      const uint64_t v = static_cast<uint32_t>(colidx[j]);
      uint64_t lo = static_cast<uint32_t>(u), hi = v;
      if (undirected && lo > hi) std::swap(lo, hi);
      const uint64_t key = undirected ? ((lo << 32) | hi) : ((static_cast<uint64_t>(u) << 32) | v);
      w[j] = 1 + static_cast<int32_t>(draw(seed, key) % 255u);
    }
  }
}

// `count` distinct traversal sources drawn uniformly among vertices with at
// least one out-arc (candidates draw(seed, 0), draw(seed, 1), ... mod n).
// Returns how many were found (fewer only if the graph has too few).
int32_t gg_sources(int32_t n, const int32_t* rowptr, uint64_t seed, int32_t count, int32_t* out) {
  int32_t found = 0;
  const uint64_t limit = 64ull * static_cast<uint64_t>(n) + 1024;
  for (uint64_t i = 0; i < limit && found < count; ++i) {
    const int32_t v = static_cast<int32_t>(draw(seed, i) % static_cast<uint64_t>(n));
    if (rowptr[v + 1] == rowptr[v]) continue;
    bool dup = false;
    for (int32_t k = 0; k < found; ++k) dup = dup || out[k] == v;
    if (!dup) out[found++] = v;
  }
  return found;
}

// First `count` outputs of the counter-based stream (for tests).
void gg_draw(uint64_t seed, int64_t count, uint64_t* out) {
  for (int64_t i = 0; i < count; ++i) out[i] = draw(seed, static_cast<uint64_t>(i));
}

int32_t gg_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
