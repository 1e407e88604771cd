// Batched persistent form: PageRank on many graphs of uneven size (each with
// its own TOCAB pull partition) and personalised PageRank for up to 64
// one-hot seed vectors on one graph, all iterations in ONE kernel launch.
//
// The grid holds at most as many work-groups as the GPU keeps resident, and
// every phase hands out work items (pull tiles, merge ranges, PPR row
// groups, dangling reductions) by striding over one flat item space built
// from per-graph prefix tables. Phases are separated by a grid barrier
// (atomic arrival counter + generation word, agent-scope fences around it so
// writes of one XCD are visible to the others); a barrier that waits longer
// than a spin limit sets an error flag that makes every work-group leave,
// so the launch always ends. Nothing is allocated and no host
// synchronisation happens inside batch_run, so it can be captured into a
// HIP graph (batch_capture / batch_launch).

#include <algorithm>
#include <vector>

#include "gc_internal.h"
#include "gc_pr_device.h"

namespace {

constexpr int kBatchK = 1024;   // merge range of batched partitions
constexpr int kPprLanes = 64;   // one lane per seed vector
constexpr int kPprRows = 32;    // rows per PPR start item (8 per wave)
constexpr int32_t kPprChunk = 2048;  // in-arcs per PPR chunk (one wave each, kWaves chunks per item)
constexpr int kWaves = kThreads / kWave;
constexpr int kPprBatch = 16;   // 256-byte row gathers a wave keeps in flight
constexpr unsigned long long kSpinLimit = 1ull << 21;

struct BGraph {
  int32_t n, n_tiles, R, B;
  const int32_t* rowptr;     // out-arc CSR offsets (out-degrees)
  const int32_t* row_ptr;    // partition
  const int32_t* col;
  const int32_t* tile_row;
  const int32_t* range_ptr;
  const uint16_t* id16;
  float* partial;
  float* contrib;
  double* dpart;             // >= max(ceil(n/256), R) slots
  double* dtotal;            // [2]
  int64_t rank_off;
};

// Personalised PageRank of up to 64 seeds, lane q of a wave = seed q. An
// iteration gathers, per in-arc u -> v, the 256-byte row c[u][0..64) of the
// current contributions. The in-arcs are cut into chunks of kPprChunk arcs
// (one wave each) rather than handed out by rows, so every wave keeps
// kPprBatch gathers in flight and a hub row's arcs spread over many waves:
// a row whose arcs lie in one chunk is finished by that chunk's wave; a row
// whose arcs span chunks leaves one FP64 piece per chunk (the sum of its
// arcs there: piece_tail of the chunk it starts in, piece_head of the
// others), and the next phase adds the pieces and finishes it.
struct BPpr {
  int32_t n, S;
  int64_t m;
  int32_t init_items;        // start items: kPprRows rows each
  int32_t n_chunks, items;   // iteration items: kWaves chunks each
  int32_t n_split, fix_items;  // rows spanning chunks; finishing items: kWaves rows each
  const int32_t* t_rowptr;
  const int32_t* t_col;
  const int32_t* rowptr;
  const int32_t* seeds;      // [S]
  const int32_t* split;      // [n_split] rows spanning chunks
  float* c[2];               // [n][64]
  double* piece_head;        // [n_chunks][64]
  double* piece_tail;        // [n_chunks][64]
  double* dpart;             // [max(init_items, items + fix_items)][64]
  double* dtotal;            // [2][64]
};

struct BatchArgs {
  const BGraph* graphs;
  int32_t G;
  const int32_t* tile_pre;   // [G+1] prefix of tiles
  const int32_t* range_pre;  // [G+1] prefix of merge ranges
  const int32_t* vert_pre;   // [G+1] prefix of 256-vertex init items
  BPpr ppr;
  int32_t has_ppr;
  double damping;
  int32_t iters;
  const float* rank_in;
  float* rank_out;
  float* ppr_out;            // [n][S]
  unsigned* bar_count;
  unsigned* bar_gen;
  int32_t* err;
};

// Item -> (graph, local index) by binary search in a prefix table.
__device__ __forceinline__ int32_t which(const int32_t* pre, int32_t G, int32_t item) {
  int32_t lo = 0, hi = G - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ bool grid_sync(const BatchArgs& a) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned gen = __hip_atomic_load(a.bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned arrived = atomicAdd(a.bar_count, 1u);
    if (arrived == gridDim.x - 1) {
      __hip_atomic_store(a.bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      atomicAdd(a.bar_gen, 1u);
    } else {
      unsigned long long spins = 0;
      while (__hip_atomic_load(a.bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (++spins > kSpinLimit || __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          atomicExch(a.err, 1);
          break;
        }
        __builtin_amdgcn_s_sleep(4);
      }
    }
    __threadfence();
    ok = __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
  }
  __syncthreads();
  return ok;
}

__device__ __forceinline__ Update make_update(const BGraph& g, double d, const double* dtotal_in, float* rank_out) {
  Update u;
  u.base = (1.0 - d) / g.n;
  u.d = d;
  u.inv_n = 1.0 / g.n;
  u.dtotal_in = dtotal_in;
  u.dpart = g.dpart;
  u.rowptr = g.rowptr;
  u.contrib = g.contrib;
  u.rank_out = rank_out;
  u.n = g.n;
  return u;
}

// Sum over a work-group of double partials of `count` slots, index order.
__device__ __forceinline__ double sum_slots(const double* p, int32_t count, int32_t stride) {
  double acc = 0.0;
  for (int32_t i = threadIdx.x; i < count; i += kThreads) acc += p[static_cast<int64_t>(i) * stride];
  return wg_sum(acc);
}

// Finishes row v of an iteration from its in-arc sum s (lane = seed):
// writes its next contribution and, on the last iteration, its rank; returns
// its dangling mass (its rank when it has no out-arc).
__device__ __forceinline__ double ppr_finish(const BPpr& p, int32_t v, double s, int32_t it, double d, double D,
                                             int32_t seed, float* out) {
  const int lane = threadIdx.x & (kWave - 1);
  const double pv = (v == seed) ? 1.0 : 0.0;
  const double r = (1.0 - d) * pv + d * (s + D * pv);
  const float r32 = static_cast<float>(r);
  const int32_t deg = p.rowptr[v + 1] - p.rowptr[v];
  p.c[(it + 1) & 1][static_cast<int64_t>(v) * kPprLanes + lane] =
      deg ? static_cast<float>(static_cast<double>(r32) / deg) : 0.0f;
  if (out && lane < p.S) out[static_cast<int64_t>(v) * p.S + lane] = r32;
  return deg ? 0.0 : static_cast<double>(r32);
}

// One wave walks in-arc chunk c: arcs [c L, min(m, (c + 1) L)). It finishes
// every row whose arcs all lie in the chunk (and the empty rows that start
// in it; the last chunk also takes those starting at m), and leaves pieces
// for rows that cross its ends. Returns the wave's dangling mass.
__device__ double ppr_chunk(const BPpr& p, int32_t c, int32_t it, double d, double D, int32_t seed, float* out) {
  const int lane = threadIdx.x & (kWave - 1);
  const float* cur = p.c[it & 1];
  const int64_t A0 = static_cast<int64_t>(c) * kPprChunk;
  const int64_t A1 = min(p.m, A0 + kPprChunk);
  const bool last_chunk = c == p.n_chunks - 1;
  // rows starting in the chunk: [lo_row, hi_row); the row holding arc A0,
  // if it started before A0, is the chunk's head row
  const int32_t lo_row = gcd::lower_bound(p.t_rowptr, 0, p.n, static_cast<int32_t>(A0));
  const int32_t hi_row = last_chunk ? p.n : gcd::lower_bound(p.t_rowptr, lo_row, p.n, static_cast<int32_t>(A1));
  const bool head_split = A0 < A1 && lo_row > 0 && p.t_rowptr[lo_row] > A0;
  int32_t v = head_split ? lo_row - 1 : lo_row;  // current row
  // ends of rows base .. base + 63, one per lane
  int32_t base = v;
  int32_t ends = p.t_rowptr[min(base + 1 + lane, p.n)];
  auto row_end = [&](int32_t r) {
    if (r - base >= kWave) {
      base = r;
      ends = p.t_rowptr[min(base + 1 + lane, p.n)];
    }
    return __builtin_amdgcn_readlane(ends, r - base);
  };
  double s = 0.0, dang = 0.0;
  int32_t vend = v < hi_row || head_split ? row_end(v) : 0;
  // rows that end at or before arc a (empty ones included) are finished
  auto flush_to = [&](int64_t a) {
    while (v < hi_row && vend <= a) {
      if (head_split && v == lo_row - 1) {
        p.piece_head[static_cast<int64_t>(c) * kPprLanes + lane] = s;
      } else {
        dang += ppr_finish(p, v, s, it, d, D, seed, out);
      }
      s = 0.0;
      ++v;
      if (v < hi_row) vend = row_end(v);
    }
  };
  for (int64_t a = A0; a < A1; a += kPprBatch) {
    const int32_t nb = static_cast<int32_t>(min<int64_t>(kPprBatch, A1 - a));
    const int32_t u = p.t_col[a + min(lane, nb - 1)];
    float x[kPprBatch];
#pragma unroll
    for (int k = 0; k < kPprBatch; ++k)
      x[k] = cur[static_cast<int64_t>(__builtin_amdgcn_readlane(u, min(k, nb - 1))) * kPprLanes + lane];
#pragma unroll
    for (int k = 0; k < kPprBatch; ++k) {
      if (k < nb) {
        flush_to(a + k);
        s += static_cast<double>(x[k]);
      }
    }
  }
  flush_to(A1);
  // what is left open crosses the chunk's end: the head row (when the whole
  // chunk lies inside it) or the last row that started here
  if (A0 < A1 && v < p.n && (v < hi_row || (head_split && v == lo_row - 1)) && vend > A1) {
    if (head_split && v == lo_row - 1) p.piece_head[static_cast<int64_t>(c) * kPprLanes + lane] = s;
    else p.piece_tail[static_cast<int64_t>(c) * kPprLanes + lane] = s;
  }
  return dang;
}

// Writes the work-group's dangling partial of item `slot` (one per seed).
__device__ __forceinline__ void ppr_dangling(const BPpr& p, int32_t slot, double mine) {
  __shared__ double dp[kWaves][kPprLanes];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  dp[wid][lane] = mine;
  __syncthreads();
  if (wid == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += dp[w][lane];
    p.dpart[static_cast<int64_t>(slot) * kPprLanes + lane] = t;
  }
  __syncthreads();
}

// Iteration item: chunks kWaves * item + wave.
__device__ void ppr_chunks(const BPpr& p, int32_t item, int32_t it, double d, float* out) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const double D = p.dtotal[(it & 1) * kPprLanes + lane];
  const int32_t seed = lane < p.S ? p.seeds[lane] : -1;
  const int32_t c = item * kWaves + wid;
  double mine = 0.0;
  if (c < p.n_chunks) mine = ppr_chunk(p, c, it, d, D, seed, out);
  ppr_dangling(p, item, mine);
}

// Finishing item (the phase after the chunks): rows that span chunks,
// kWaves * item + wave, from their pieces.
__device__ void ppr_split_rows(const BPpr& p, int32_t item, int32_t it, double d, float* out) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const double D = p.dtotal[(it & 1) * kPprLanes + lane];
  const int32_t seed = lane < p.S ? p.seeds[lane] : -1;
  const int32_t i = item * kWaves + wid;
  double mine = 0.0;
  if (i < p.n_split) {
    const int32_t v = p.split[i];
    const int32_t c0 = p.t_rowptr[v] / kPprChunk, c1 = (p.t_rowptr[v + 1] - 1) / kPprChunk;
    double s = p.piece_tail[static_cast<int64_t>(c0) * kPprLanes + lane];
    for (int32_t c = c0 + 1; c <= c1; ++c) s += p.piece_head[static_cast<int64_t>(c) * kPprLanes + lane];
    mine = ppr_finish(p, v, s, it, d, D, seed, out);
  }
  ppr_dangling(p, p.items + item, mine);
}

// PPR start: r0 = p (one-hot per seed), c0 = r0 / outdeg, dangling partials.
__device__ void ppr_init_rows(const BPpr& p, int32_t item) {
  __shared__ double dp[kThreads / kWave][kPprLanes];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int32_t seed = lane < p.S ? p.seeds[lane] : -1;
  double mine = 0.0;
  const int32_t r0 = item * kPprRows;
  for (int32_t v = r0 + wid; v < min(p.n, r0 + kPprRows); v += kThreads / kWave) {
    const int32_t deg = p.rowptr[v + 1] - p.rowptr[v];
    const float r = (v == seed) ? 1.0f : 0.0f;
    p.c[0][static_cast<int64_t>(v) * kPprLanes + lane] = deg ? r / static_cast<float>(deg) : 0.0f;
    if (!deg) mine += r;
  }
  dp[wid][lane] = mine;
  __syncthreads();
  if (wid == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / kWave; ++w) t += dp[w][lane];
    p.dpart[static_cast<int64_t>(item) * kPprLanes + lane] = t;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_batch_reset(unsigned* count, int32_t* err) {
  *count = 0u;
  *err = 0;
}

__global__ __launch_bounds__(kThreads) void k_batch(BatchArgs a) {
  __shared__ float vals[kStageCap];
  __shared__ double acc[kBatchK];
  const int32_t G = a.G;
  const int32_t tiles = G ? a.tile_pre[G] : 0, ranges = G ? a.range_pre[G] : 0, verts = G ? a.vert_pre[G] : 0;
  const int32_t init_items = a.has_ppr ? a.ppr.init_items : 0;
  const int32_t pitems = a.has_ppr ? a.ppr.items : 0;
  const int32_t fitems = a.has_ppr ? a.ppr.fix_items : 0;
  const int32_t red_items = G + (a.has_ppr ? kPprLanes : 0);

  // ---- start: contributions of the start vectors and their dangling mass
  for (int32_t item = blockIdx.x; item < verts + init_items; item += gridDim.x) {
    if (item < verts) {
      const int32_t gi = which(a.vert_pre, G, item);
      const BGraph& g = a.graphs[gi];
      const int32_t v = (item - a.vert_pre[gi]) * kThreads + threadIdx.x;
      double mine = 0.0;
      if (v < g.n) {
        const float r = a.rank_in[g.rank_off + v];
        const int32_t deg = g.rowptr[v + 1] - g.rowptr[v];
        g.contrib[v] = deg ? static_cast<float>(static_cast<double>(r) / deg) : 0.0f;
        mine = deg ? 0.0 : static_cast<double>(r);
      }
      const double t = wg_sum(mine);
      if (threadIdx.x == 0) g.dpart[item - a.vert_pre[gi]] = t;
    } else {
      ppr_init_rows(a.ppr, item - verts);
    }
  }
  if (!grid_sync(a)) return;
  for (int32_t item = blockIdx.x; item < red_items; item += gridDim.x) {
    if (item < G) {
      const BGraph& g = a.graphs[item];
      const double t = sum_slots(g.dpart, a.vert_pre[item + 1] - a.vert_pre[item], 1);
      if (threadIdx.x == 0) g.dtotal[0] = t;
    } else {
      const int32_t q = item - G;
      const double t = sum_slots(a.ppr.dpart + q, init_items, kPprLanes);
      if (threadIdx.x == 0) a.ppr.dtotal[q] = t;
    }
  }
  if (!grid_sync(a)) return;

  for (int32_t it = 0; it < a.iters; ++it) {
    const bool last = it == a.iters - 1;
    // ---- pull tiles of every graph (Algorithm 4) and PPR row groups
    for (int32_t item = blockIdx.x; item < tiles + pitems; item += gridDim.x) {
      if (item < tiles) {
        const int32_t gi = which(a.tile_pre, G, item);
        const BGraph& g = a.graphs[gi];
        const int32_t t = item - a.tile_pre[gi];
        const int32_t r0 = g.tile_row[t], r1 = g.tile_row[t + 1];
        if (r0 < r1)
          pull_tile(g.row_ptr, g.col, g.contrib, r0, r1, vals,
                    [&](int32_t r, double s) { g.partial[r] = static_cast<float>(s); });
        __syncthreads();  // vals is reused by the next item
      } else {
        ppr_chunks(a.ppr, item - tiles, it, a.damping, last ? a.ppr_out : nullptr);
      }
    }
    if (!grid_sync(a)) return;
    // ---- merge ranges fused with the update (Figure 5), and the PPR rows
    // whose arcs span chunks
    for (int32_t item = blockIdx.x; item < ranges + fitems; item += gridDim.x) {
      if (item >= ranges) {
        ppr_split_rows(a.ppr, item - ranges, it, a.damping, last ? a.ppr_out : nullptr);
        continue;
      }
      const int32_t gi = which(a.range_pre, G, item);
      const BGraph& g = a.graphs[gi];
      const int32_t j = item - a.range_pre[gi];
      merge_accumulate<kBatchK, true>(g.range_ptr, g.B, g.id16, g.partial, j, acc);
      const Update u = make_update(g, a.damping, g.dtotal + (it & 1), last ? a.rank_out + g.rank_off : nullptr);
      const double D = g.dtotal[it & 1];
      double mine = 0.0;
      for (int i = threadIdx.x; i < kBatchK; i += kThreads) {
        const int32_t v = j * kBatchK + i;
        if (v < g.n) mine += update_vertex(u, v, acc[i], D);
      }
      const double t = wg_sum(mine);
      if (threadIdx.x == 0) g.dpart[j] = t;
      __syncthreads();  // acc is reused by the next item
    }
    if (!grid_sync(a)) return;
    // ---- next dangling totals
    for (int32_t item = blockIdx.x; item < red_items; item += gridDim.x) {
      if (item < G) {
        const BGraph& g = a.graphs[item];
        const double t = sum_slots(g.dpart, g.R, 1);
        if (threadIdx.x == 0) g.dtotal[(it + 1) & 1] = t;
      } else {
        const int32_t q = item - G;
        const double t = sum_slots(a.ppr.dpart + q, pitems + fitems, kPprLanes);
        if (threadIdx.x == 0) a.ppr.dtotal[((it + 1) & 1) * kPprLanes + q] = t;
      }
    }
    if (!last && !grid_sync(a)) return;
  }
}

}  // namespace

struct gc_batch_s {
  std::vector<gc_graph> graphs;
  std::vector<gc_tocab> parts;
  std::vector<int64_t> rank_off;
  std::vector<int32_t> widths;
  gc_graph ppr_graph = nullptr;
  int32_t n_seeds = 0;
  BatchArgs args{};
  int32_t grid = 0;
  int64_t bytes = 0;
  std::vector<void*> owned;
  int32_t* err_host = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int bfail(int code, const char* fmt, const char* what = "") {
  gcx::set_error(fmt, what);
  return code;
}

void* own(gc_batch b, size_t bytes) {
  void* p = gcx::dev_alloc(bytes, nullptr);
  if (p) {
    b->owned.push_back(p);
    b->bytes += static_cast<int64_t>(bytes);
  }
  return p;
}

void destroy(gc_batch b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (gc_tocab t : b->parts) tocab_free(t);
  for (void* p : b->owned) gcx::dev_free(p, nullptr);
  if (b->err_host) (void)hipHostFree(b->err_host);
  delete b;
}

}  // namespace

extern "C" {

int batch_create(const gc_graph* graphs, int32_t n_graphs, const int32_t* block_widths, gc_graph ppr_graph,
                 const int32_t* seeds, int32_t n_seeds, hipStream_t stream, gc_batch* out) {
  if (!out) return bfail(GC_EINVAL, "batch_create: out is NULL");
  *out = nullptr;
  if (n_graphs < 0 || (n_graphs > 0 && !graphs)) return bfail(GC_EINVAL, "batch_create: bad graph list");
  if (n_seeds < 0 || n_seeds > kPprLanes || (n_seeds > 0 && (!ppr_graph || !seeds)))
    return bfail(GC_EINVAL, "batch_create: 0..64 seeds on a graph");
  if (n_graphs == 0 && n_seeds == 0) return bfail(GC_EINVAL, "batch_create: nothing to run");
  for (int32_t i = 0; i < n_graphs; ++i)
    if (!graphs[i]) return bfail(GC_EINVAL, "batch_create: NULL graph");
  for (int32_t q = 0; q < n_seeds; ++q)
    if (seeds[q] < 0 || seeds[q] >= ppr_graph->n) return bfail(GC_EINVAL, "batch_create: seed out of range");
  gc_batch b = new (std::nothrow) gc_batch_s;
  if (!b) return bfail(GC_ENOMEM, "batch_create: host allocation failed");
  std::vector<BGraph> hg(n_graphs);
  std::vector<int32_t> tile_pre(n_graphs + 1, 0), range_pre(n_graphs + 1, 0), vert_pre(n_graphs + 1, 0);
  int64_t off = 0;
  for (int32_t i = 0; i < n_graphs; ++i) {
    gc_graph g = graphs[i];
    int32_t W = block_widths ? block_widths[i] : 0;
    if (W == 0) {  // autotuned among widths whose slices stay in the last-level cache
      int32_t k = 0;
      float ms = 0.0f;
      if (gcx::autotune(g, GC_PULL, 1 << 16, &W, &k, &ms, stream) != hipSuccess) {
        destroy(b);
        return bfail(GC_EHIP, "batch_create: autotune failed");
      }
    }
    gc_tocab t = nullptr;
    const int rc = tocab_partition(g, GC_PULL, W, kBatchK, stream, &t);
    if (rc != GC_OK) {
      destroy(b);
      return rc;
    }
    if (t->B > kFlatB || t->col16) {
      tocab_free(t);
      destroy(b);
      return bfail(GC_EUNSUPPORTED, "batch_create: widths below 2^16 or above 1024 blocks are not batched");
    }
    b->parts.push_back(t);
    b->graphs.push_back(g);
    b->widths.push_back(W);
    BGraph& d = hg[i];
    d.n = g->n;
    d.n_tiles = t->n_tiles;
    d.R = t->R;
    d.B = t->B;
    d.rowptr = g->rowptr;
    d.row_ptr = t->row_ptr;
    d.col = t->col;
    d.tile_row = t->tile_row;
    d.range_ptr = t->range_ptr;
    d.id16 = t->id16;
    d.partial = t->partial;
    const int32_t vgrid = (g->n + kThreads - 1) / kThreads;
    d.contrib = static_cast<float*>(own(b, sizeof(float) * g->n));
    d.dpart = static_cast<double*>(own(b, sizeof(double) * std::max(vgrid, t->R)));
    d.dtotal = static_cast<double*>(own(b, sizeof(double) * 2));
    d.rank_off = off;
    if (!d.contrib || !d.dpart || !d.dtotal) {
      destroy(b);
      return bfail(GC_ENOMEM, "batch_create: allocation failed");
    }
    b->rank_off.push_back(off);
    off += g->n;
    tile_pre[i + 1] = tile_pre[i] + t->n_tiles;
    range_pre[i + 1] = range_pre[i] + t->R;
    vert_pre[i + 1] = vert_pre[i] + vgrid;
  }
  b->rank_off.push_back(off);
  BatchArgs& a = b->args;
  a.G = n_graphs;
  a.has_ppr = n_seeds > 0;
  if (n_seeds > 0) {
    gc_graph pg = ppr_graph;
    b->ppr_graph = pg;
    b->n_seeds = n_seeds;
    BPpr& p = a.ppr;
    p.n = pg->n;
    p.m = pg->m;
    p.S = n_seeds;
    p.init_items = (pg->n + kPprRows - 1) / kPprRows;
    p.n_chunks = static_cast<int32_t>(std::max<int64_t>(1, (pg->m + kPprChunk - 1) / kPprChunk));
    p.items = (p.n_chunks + kWaves - 1) / kWaves;
    p.t_rowptr = pg->t_rowptr;
    p.t_col = pg->t_colidx;
    p.rowptr = pg->rowptr;
    // rows whose in-arcs span chunks (finished from their pieces)
    std::vector<int32_t> trp(static_cast<size_t>(pg->n) + 1), split;
    if (hipMemcpy(trp.data(), pg->t_rowptr, sizeof(int32_t) * trp.size(), hipMemcpyDeviceToHost) != hipSuccess) {
      destroy(b);
      return bfail(GC_EHIP, "batch_create: copy failed");
    }
    for (int32_t v = 0; v < pg->n; ++v)
      if (trp[v + 1] > trp[v] && trp[v] / kPprChunk != (trp[v + 1] - 1) / kPprChunk) split.push_back(v);
    p.n_split = static_cast<int32_t>(split.size());
    p.fix_items = (p.n_split + kWaves - 1) / kWaves;
    const size_t lanes = kPprLanes;
    int32_t* ds = static_cast<int32_t*>(own(b, sizeof(int32_t) * n_seeds));
    int32_t* sp = static_cast<int32_t*>(own(b, sizeof(int32_t) * std::max<size_t>(split.size(), 1)));
    p.c[0] = static_cast<float*>(own(b, sizeof(float) * lanes * static_cast<size_t>(pg->n)));
    p.c[1] = static_cast<float*>(own(b, sizeof(float) * lanes * static_cast<size_t>(pg->n)));
    p.piece_head = static_cast<double*>(own(b, sizeof(double) * lanes * static_cast<size_t>(p.n_chunks)));
    p.piece_tail = static_cast<double*>(own(b, sizeof(double) * lanes * static_cast<size_t>(p.n_chunks)));
    const size_t slots = static_cast<size_t>(std::max(p.init_items, p.items + p.fix_items));
    p.dpart = static_cast<double*>(own(b, sizeof(double) * lanes * slots));
    p.dtotal = static_cast<double*>(own(b, sizeof(double) * 2 * lanes));
    if (!ds || !sp || !p.c[0] || !p.c[1] || !p.piece_head || !p.piece_tail || !p.dpart || !p.dtotal) {
      destroy(b);
      return bfail(GC_ENOMEM, "batch_create: allocation failed");
    }
    if (hipMemcpy(ds, seeds, sizeof(int32_t) * n_seeds, hipMemcpyDefault) != hipSuccess ||
        (!split.empty() && hipMemcpy(sp, split.data(), sizeof(int32_t) * split.size(), hipMemcpyHostToDevice) !=
                               hipSuccess)) {
      destroy(b);
      return bfail(GC_EHIP, "batch_create: copy failed");
    }
    p.seeds = ds;
    p.split = sp;
  }
  BGraph* dg = static_cast<BGraph*>(own(b, sizeof(BGraph) * std::max(1, n_graphs)));
  int32_t* pre = static_cast<int32_t*>(own(b, sizeof(int32_t) * 3 * (n_graphs + 1)));
  a.bar_count = static_cast<unsigned*>(own(b, sizeof(unsigned) * 2));
  a.err = static_cast<int32_t*>(own(b, sizeof(int32_t)));
  if (!dg || !pre || !a.bar_count || !a.err ||
      hipHostMalloc(reinterpret_cast<void**>(&b->err_host), sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    destroy(b);
    return bfail(GC_ENOMEM, "batch_create: allocation failed");
  }
  a.bar_gen = a.bar_count + 1;
  hipError_t e = hipSuccess;
  if (n_graphs > 0) e = hipMemcpy(dg, hg.data(), sizeof(BGraph) * n_graphs, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pre, tile_pre.data(), sizeof(int32_t) * (n_graphs + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pre + n_graphs + 1, range_pre.data(), sizeof(int32_t) * (n_graphs + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pre + 2 * (n_graphs + 1), vert_pre.data(), sizeof(int32_t) * (n_graphs + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(a.bar_count, 0, sizeof(unsigned) * 2);
  // co-resident grid: every work-group must be live for the grid barrier
  int per_cu = 0, dev = 0;
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_batch), kThreads, 0);
  if (e != hipSuccess || per_cu < 1) {
    destroy(b);
    return bfail(GC_EHIP, "batch_create: device query failed");
  }
  b->grid = per_cu * prop.multiProcessorCount;
  a.graphs = dg;
  a.tile_pre = pre;
  a.range_pre = pre + n_graphs + 1;
  a.vert_pre = pre + 2 * (n_graphs + 1);
  *out = b;
  return GC_OK;
}

int batch_info(gc_batch b, int64_t* rank_offsets, int32_t* block_widths, int32_t* grid, int64_t* bytes) {
  if (!b) return bfail(GC_EINVAL, "batch_info: NULL batch");
  for (size_t i = 0; i < b->rank_off.size() && rank_offsets; ++i) rank_offsets[i] = b->rank_off[i];
  for (size_t i = 0; i < b->widths.size() && block_widths; ++i) block_widths[i] = b->widths[i];
  if (grid) *grid = b->grid;
  if (bytes) *bytes = b->bytes;
  return GC_OK;
}

int batch_run(gc_batch b, float damping, int32_t iters, const float* ranks_in, float* ranks_out, float* ppr_out,
              hipStream_t stream) {
  if (!b) return bfail(GC_EINVAL, "batch_run: NULL batch");
  if (!(damping >= 0.0f && damping <= 1.0f) || iters < 1) return bfail(GC_EINVAL, "batch_run: bad damping or iters");
  if (!b->graphs.empty() && (!ranks_in || !ranks_out)) return bfail(GC_EINVAL, "batch_run: NULL rank buffers");
  if (b->n_seeds > 0 && !ppr_out) return bfail(GC_EINVAL, "batch_run: NULL ppr output");
  BatchArgs a = b->args;
  a.damping = damping;
  a.iters = iters;
  a.rank_in = ranks_in;
  a.rank_out = ranks_out;
  a.ppr_out = ppr_out;
  gcx::ProfScope prof("batch", stream);
  k_batch_reset<<<1, 1, 0, stream>>>(a.bar_count, a.err);
  k_batch<<<b->grid, kThreads, 0, stream>>>(a);
  return hipGetLastError() == hipSuccess ? GC_OK : bfail(GC_EHIP, "batch_run: launch failed");
}

int batch_capture(gc_batch b, float damping, int32_t iters, const float* ranks_in, float* ranks_out, float* ppr_out) {
  if (!b) return bfail(GC_EINVAL, "batch_capture: NULL batch");
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  hipStream_t cs;
  if (hipStreamCreate(&cs) != hipSuccess) return bfail(GC_EHIP, "batch_capture: stream");
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  int rc = GC_OK;
  if (e == hipSuccess) rc = batch_run(b, damping, iters, ranks_in, ranks_out, ppr_out, cs);
  const hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess && rc == GC_OK) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (rc != GC_OK) return rc;
  return e == hipSuccess ? GC_OK : bfail(GC_EHIP, "batch_capture: capture failed");
}

int batch_launch(gc_batch b, hipStream_t stream) {
  if (!b || !b->exec) return bfail(GC_EINVAL, "batch_launch: nothing captured");
  gcx::ProfScope prof("batch_graph", stream);
  return hipGraphLaunch(b->exec, stream) == hipSuccess ? GC_OK : bfail(GC_EHIP, "batch_launch: launch failed");
}

int batch_status(gc_batch b, hipStream_t stream, int32_t* barrier_timeout) {
  if (!b || !barrier_timeout) return bfail(GC_EINVAL, "batch_status: bad argument");
  hipError_t e = hipMemcpyAsync(b->err_host, b->args.err, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return bfail(GC_EHIP, "batch_status: %s", hipGetErrorString(e));
  *barrier_timeout = *b->err_host;
  return GC_OK;
}

int batch_free(gc_batch b) {
  if (!b) return bfail(GC_EINVAL, "batch_free: NULL batch");
  (void)hipDeviceSynchronize();
  destroy(b);
  return GC_OK;
}

}  // extern "C"
