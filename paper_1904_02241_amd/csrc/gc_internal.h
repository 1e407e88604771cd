// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "graphcage.h"

// ---------------------------------------------------------------------------
// Handles

struct gc_graph_s {
  int32_t n = 0;
  int64_t m = 0;
  bool weighted = false;
  // out-arc CSR (row = source), as loaded
  int32_t* rowptr = nullptr;
  int32_t* colidx = nullptr;
  int32_t* w = nullptr;
  // transposed CSR (row = destination, columns ascending)
  int32_t* t_rowptr = nullptr;
  int32_t* t_colidx = nullptr;
  int32_t* t_w = nullptr;
  // PageRank scratch: contributions (two buffers for the fused plain pull),
  // push accumulators, FP64 dangling partials / totals and a done counter
  float* contrib[2] = {nullptr, nullptr};
  double* sums = nullptr;     // push accumulators (FP64 atomics)
  int32_t* tile_row_in = nullptr;  // pull tiles over the transposed graph
  int32_t n_tiles_in = 0;
  double* dpart = nullptr;    // one slot per apply work-group
  double* dtotal = nullptr;   // [2] ping-pong dangling totals
  unsigned* counter = nullptr;
  int32_t dpart_slots = 0;
  bool values_f32 = false;  // the weight arrays hold FP32 values (GC_VALUES_F32)
  // convergence mode (allocated by the first pagerank_converge call): FP64
  // partials of the L1 change per update work-group, their total, and a
  // second FP32 iterate
  double* lpart = nullptr;
  double* ltotal = nullptr;
  float* rank_tmp = nullptr;
  // traversal scratch
  uint32_t* front = nullptr;  // status arrays (Section 3.3), one bit per vertex
  uint32_t* next = nullptr;
  int32_t* queue[2] = {nullptr, nullptr};
  uint32_t* visited = nullptr;  // BFS: bitmap of vertices with a final depth
  int32_t* mark = nullptr;      // SSSP push: round in which a vertex was queued
  int32_t* arc_deg = nullptr;   // out-degrees of a vertex list (arc-balanced push, BC backward)
  int32_t* arc_pre = nullptr;   // [n+1] their exclusive scan
  int32_t max_out_deg = -1;     // largest out-degree (-1: not found yet; set by the first traversal)
  // betweenness centrality (allocated by the first bc_accumulate call):
  // path counts, two alternating arrays of (1 + delta) / sigma, BFS depths
  // and the vertices in level order of the current source
  double* bc_sigma = nullptr;
  double* bc_coef = nullptr;  // [2n]
  int32_t* bc_depth = nullptr;
  int32_t* bc_order = nullptr;
  int32_t* stats = nullptr;     // device counters read back once per level (kStatSlots)
  int32_t* stats_host = nullptr;  // pinned mirror
  int32_t clock_khz = 100000;   // rate of the device wall clock stamped into stats
  int64_t bytes = 0;
  // learned level scheduler attached to this graph (sched_attach)
  gc_sched sched = nullptr;
  gc_sched sched_kind[3] = {nullptr, nullptr, nullptr};  // per kind (BFS, SSSP, PageRank); null: sched
  std::vector<gc_tocab> sched_parts;
  int32_t pr_learned_action = -1;  // pagerank_learned's form for the attached network (-1: not chosen yet)
  // per-level record of the last traversal: action and wall time (ms)
  std::vector<int32_t> trace_action;
  std::vector<float> trace_ms;
};

// Row structure of 64 consecutive arcs of a stream-layout partition: bit i
// set when arc 64w + i is the first arc of its local row, the number of
// local rows that start before arc 64w (the index of the first row whose
// head lies at or after the word), and bit 0 of the next word.
struct alignas(16) gc_head_word {
  uint64_t bits;
  int32_t row;
  int32_t next;
};

struct gc_tocab_s {
  gc_graph g = nullptr;
  int32_t dir = GC_PULL;
  int32_t W = 0, log2W = 0, k = 0, log2k = 0, B = 0, R = 0;
  int32_t n_rows = 0, n_cols = 0;
  int64_t P = 0;
  int64_t m = 0;
  bool weighted = false;
  int32_t* blk_rowoff = nullptr;  // [B+1]
  int32_t* row_ptr = nullptr;     // [P+1]
  int32_t* id_map = nullptr;      // [P]
  int32_t* col = nullptr;         // [m]
  int32_t* w = nullptr;           // [m] or null
  int32_t* range_ptr = nullptr;   // [(R+1)*B], j-major
  float* partial = nullptr;       // [P] pull partial sums (Algorithm 4)
  uint16_t* id16 = nullptr;       // [P] id_map mod k: position inside the merge range
  int32_t* tile_row = nullptr;    // [n_tiles+1] first local row of each pull tile
  int32_t n_tiles = 0;
  // Stream layout of an LDS-resident pull partition (W <= kLdsMaxWidth):
  // 16-bit columns inside the block, one head bit per arc marking the first
  // arc of every local row, and partial sums stored range-major (all blocks'
  // partials of merge range j contiguous) so the merge reads one stream.
  uint16_t* col16 = nullptr;      // [m_pad], zero past m
  gc_head_word* heads = nullptr;  // [m_pad/64 + 1], bits at and past m set
  int64_t m_pad = 0;              // multiple of wave_tile_arcs(), >= m + wave_tile_arcs()
  int32_t* wtile_row = nullptr;   // unused by the stream layout
  int32_t n_wtiles = 0;
  int2* seg = nullptr;            // [B][R+1]: first local row of block b in range j, shift to range-major index
  int32_t* rstart = nullptr;      // [R+1] range-major start of merge range j
  uint16_t* id16s = nullptr;      // [P] id16 in range-major order
  int32_t* chunk_beg = nullptr;   // [n_chunks] first local row
  int32_t* chunk_end = nullptr;   // [n_chunks] one past the last local row
  int32_t* chunk_blk = nullptr;   // [n_chunks] block
  int32_t* chunk_j0 = nullptr;    // [n_chunks] first merge range the chunk's rows fall in
  int32_t* chunk_ns = nullptr;    // [n_chunks] number of merge ranges the chunk's rows span
  int32_t n_chunks = 0;
  int32_t seg_max = 0;            // largest chunk_ns (sizes the work-group's LDS table)
  int32_t* pmin = nullptr;        // [P + 8] traversal partials (next flags / min; range-major for SSSP over the stream layout)
  double* bc_part = nullptr;      // [P] BC path-count partials (allocated on first use)
  float* val32 = nullptr;         // [m_pad] FP32 arc values in stream order (first valued SpMV)
  int32_t* w_pad = nullptr;       // [m_pad] integer weights in stream order, 0 past m (first SSSP over the stream layout)
  uint8_t* w8 = nullptr;          // [m_pad] the same as bytes, instead of w_pad when every weight lies in [0, 255]
  // Expanded contributions of a GC_PUSH partition with block sums in LDS
  // (W <= kPushLdsMaxWidth, B <= kPushExpandMaxBlocks): the work-group that
  // updates source block s writes the new contribution of each local row
  // whose source lies in it (block b's rows [range_ptr[j0 B + b],
  // range_ptr[j1 B + b]) for the merge ranges j0 .. j1 of the block) to xc.
  uint16_t* xid16 = nullptr;      // [P + 8] source of each local row (source-major when xperm is set), offset inside its source block
  int32_t* xperm = nullptr;       // [P] short runs only: the local row at each source-major position
  int32_t* xstart = nullptr;      // [n_sblk + 1] short runs only: first source-major position of each source block
  float* xc = nullptr;            // [2P] contribution of each local row's source, two iterates in turn
  int32_t n_sblk = 0;             // source blocks (ceil(rows / W)); 0 without the expanded form
  // ... and its arcs as streams: destination offsets inside the block (16
  // bits) and one head bit per arc marking the first arc of each local row
  // (the head word layout of the pull's stream layout), padded to whole
  // 512-arc tiles.
  uint16_t* pcol16 = nullptr;     // [pm_pad], zero past m
  gc_head_word* pheads = nullptr; // [pm_pad/64 + 1], bits at and past m set
  int64_t pm_pad = 0;
  int64_t bytes = 0;
};

// ---------------------------------------------------------------------------
// Runtime helpers (gc_runtime.hip)

namespace gcx {

void set_error(const char* fmt, ...);
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);

// RAII buffer from the library allocator
struct Buf {
  void* p = nullptr;
  hipStream_t s = nullptr;
  Buf() = default;
  Buf(size_t bytes, hipStream_t st) : p(dev_alloc(bytes, st)), s(st) {}
  ~Buf() { if (p) dev_free(p, s); }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  template <class T> T* as() const { return static_cast<T*>(p); }
  void* release() { void* q = p; p = nullptr; return q; }
};

// ---- construction kernels (gc_build.hip) ----
// Device-side structural check of an out-arc CSR; *bad_out != 0 if broken.
hipError_t check_csr(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx, int32_t* bad_out,
                     hipStream_t s);
// Exclusive scan of int32 `in[0..n)` into `out[0..n]` (out[n] = total).
hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);
// Transposed CSR with rows sorted by column; weights carried (w may be null).
hipError_t build_transpose(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx,
                           const int32_t* w, int32_t* t_rowptr, int32_t* t_colidx, int32_t* t_w,
                           hipStream_t s);
// Pull tile table: tile i owns the rows whose first arc lies in
// [i*tile_arcs, (i+1)*tile_arcs); out[i] = first such row, out[n_tiles] = rows.
hipError_t build_tiles(const int32_t* row_ptr, int64_t rows, int64_t arcs, int32_t tile_arcs,
                       int32_t** out, int32_t* n_tiles, hipStream_t s);
// TOCAB partition of CSR A (see tocab_partition); fills t's arrays.
hipError_t build_partition(gc_tocab t, const int32_t* a_rowptr, const int32_t* a_col,
                           const int32_t* a_w, hipStream_t s);

// ---- PageRank (gc_pagerank.hip) ----
int32_t pull_tile_arcs();
int32_t wave_tile_arcs();
// Largest block width whose FP32 contribution slice is staged in LDS.
constexpr int32_t kLdsMaxWidth = 1 << 15;
// Largest block width of a TOCAB push whose block sums (FP64) sit in LDS.
constexpr int32_t kPushLdsMaxWidth = 1 << 14;
// Most blocks of a push partition with expanded contributions (a work-group
// keeps two run bounds per block in LDS).
constexpr int32_t kPushExpandMaxBlocks = 4096;
// Average run length (local rows per (source block, block) pair) from which
// the expanded push walks its runs in place rather than through a
// source-major list.
constexpr int64_t kPushLongRun = 128;
// Offset of the second buffer of expanded contributions (16-byte aligned).
inline int64_t push_xc_stride(int64_t P) { return (std::max<int64_t>(P, 1) + 3) & ~int64_t(3); }
// Smallest number of arcs per chunk of an LDS-resident block (one work-group each).
constexpr int32_t kLdsChunkArcs = 1 << 16;
// LDS bytes one work-group of the LDS-resident pull may use: half a CU's
// 160 KB (two resident work-groups) for slices up to 2^13 floats, all of it
// for wider ones.
inline int32_t lds_budget(int32_t W) { return W >= (1 << 14) ? 160 * 1024 - 512 : 80 * 1024 - 512; }
// LDS bytes of the pull's per-wave output staging (16 waves x (384 rows +
// 16 spare slots) floats).
constexpr int32_t kLdsStageBytes = 16 * (384 + 16) * 4;
// Largest range table (entries) that fits beside a W-float slice and the
// staging (with 8 entries of padding).
inline int32_t lds_seg_cap(int32_t W) { return ((lds_budget(W) - 4 * W - kLdsStageBytes) / 4 - 8) / 2; }
// ---- SpMV (gc_spmv.hip; the stream-layout form in gc_pagerank.hip) ----
hipError_t spmv_run(gc_graph g, gc_tocab t, const float* x, float* y, hipStream_t s);
hipError_t spmv_stream(gc_graph g, gc_tocab t, const float* x, const float* vals, float* y, hipStream_t s);
hipError_t stream_values(gc_graph g, gc_tocab t, hipStream_t s);

// Convergence mode of pagerank_run: iterate until the L1 change between
// consecutive iterates is at most tol (or max_iters); iters / delta report
// the iterations run and the last change.
struct Converge {
  double tol = 0.0;
  int32_t max_iters = 0;
  int32_t iters = 0;
  double delta = 0.0;
};
// Device buffers an iteration writes besides rank_out: contributions (two,
// used in turn by the forms that read one while writing the next), FP64
// push sums (n), FP64 dangling partials (one per update work-group, at most
// the graph's dpart_slots) and their two totals, and the pull partition's
// partial sums (P + 8). By default the graph's and the partition's own.
struct PrBuffers {
  float* contrib[2];
  double* sums;
  double* dpart;
  double* dtotal;
  float* partial;
};
hipError_t pagerank_run(gc_graph g, gc_tocab t, int32_t dir, float damping, int32_t dangling,
                        const float* rank_in, float* rank_out, int32_t iters, hipStream_t s,
                        Converge* cv = nullptr, int32_t ladder = -1, const PrBuffers* bufs = nullptr);

// PageRank's working-set action among 0 push, 1 pull, 2 + i TOCAB over parts[i].
int32_t pagerank_fallback_action(const gc_tocab* parts, int32_t n_parts);
// Scheduler training rows for PageRank (see sched_collect, kind 2).
hipError_t collect_pagerank(gc_graph g, gc_tocab* parts, int32_t n_parts, int32_t n_rows, float* features,
                            float* times, int32_t max_rows, int32_t* rows, hipStream_t s);

// ---- autotuner (gc_autotune.hip) ----
// Candidate widths start at max(2^12, min_W).
hipError_t autotune(gc_graph g, int32_t dir, int32_t min_W, int32_t* W_out, int32_t* k_out, float* ms_out,
                    hipStream_t s);

// ---- traversal (gc_traverse.hip) ----
hipError_t bfs_run(gc_graph g, gc_tocab t, int32_t source, int32_t* depth, int32_t* levels,
                   uint32_t policy, hipStream_t s);
hipError_t sssp_run(gc_graph g, gc_tocab t, int32_t source, int32_t* dist, int32_t* rounds,
                    uint32_t policy, hipStream_t s, bool* overflow);
hipError_t bc_run(gc_graph g, gc_tocab t, const int32_t* sources, int32_t n_src, double* bc, uint32_t policy,
                  hipStream_t s);
hipError_t collect(gc_graph g, gc_tocab* parts, int32_t n_parts, bool bfs, const int32_t* sources, int32_t n_src,
                   float* features, float* times, int32_t max_rows, int32_t* rows, hipStream_t s);
void sched_features(int64_t n, int64_t m, int64_t n_f, int64_t m_f, int32_t level, double prior_ms,
                    int64_t prior_arcs, float* f);

// The scheduler's 6 inputs for a level (the same arithmetic on the host and
// in the device-side decision): log1p(frontier vertices), log1p(frontier
// out-arcs), log1p(m / n), log2(ceil(n / 2^18) + 1), level / 16, and
// log1p(the previous level's time per out-arc of its frontier, in ns), 0
// before the first level.
__host__ __device__ inline void level_features(int64_t n, int64_t m, int64_t n_f, int64_t m_f, int32_t level,
                                               double prior_ms, int64_t prior_arcs, float* f) {
  f[0] = static_cast<float>(log1p(static_cast<double>(n_f)));
  f[1] = static_cast<float>(log1p(static_cast<double>(m_f)));
  f[2] = static_cast<float>(log1p(static_cast<double>(m) / static_cast<double>(n > 1 ? n : 1)));
  f[3] = static_cast<float>(log2(static_cast<double>((n + (1 << 18) - 1) >> 18) + 1.0));
  f[4] = static_cast<float>(level) / 16.0f;
  f[5] = static_cast<float>(log1p(prior_ms * 1e6 / static_cast<double>(prior_arcs > 1 ? prior_arcs : 1)));
}

// Device counters of one traversal level (int32 slots), copied once per
// level to a pinned host mirror.
constexpr int kStatQLen = 0;      // vertices appended to the next queue
constexpr int kStatOverflow = 1;  // SSSP: a path length reached INT32_MAX
constexpr int kStatDegLo = 2;     // out-arcs of the next frontier (64-bit: lo, hi)
constexpr int kStatT0 = 4;        // device wall clock at the level's start (64-bit)
constexpr int kStatT1 = 6;        // device wall clock when its relaxation kernels have finished (64-bit)
constexpr int kStatChoice = 8;    // learned scheduler: action for the next level (-1: no finite output)
constexpr int kStatInDegLo = 10;  // in-arcs of the next frontier (64-bit: lo, hi)
constexpr int kStatOut = 16;      // learned scheduler: its K outputs (FP32 bit patterns)
constexpr int kStatSlots = kStatOut + GC_SCHED_HIDDEN;

// Learned policy: the working-set rule's choice is kept unless the network
// predicts its own pick faster by more than this margin (its outputs are
// log times relative to the fastest action, so 0.3 is about 35 %: the
// network overrides the rule only where it expects a clear win).
constexpr float kLearnedGate = 0.3f;

// ---- scheduler network (gc_sched.hip) ----
int32_t sched_actions(gc_sched m);
// The network deciding for one kind of work on g (0 BFS, 1 SSSP, 2
// PageRank): the one attached for that kind, else the shared one (or null).
inline gc_sched sched_for(gc_graph g, int kind) { return g->sched_kind[kind] ? g->sched_kind[kind] : g->sched; }
// Device pointer to the network's parameters (layout in gc_mlp.h).
const float* sched_params(gc_sched m);
// Device pointer to the training range of its inputs (null before training).
const float* sched_range(gc_sched m);
// Decision from host features: action (-1 when an output is not finite)
// and, when out is given, the K outputs. Synchronises s.
hipError_t sched_decide(gc_sched m, const float* features, hipStream_t s, int32_t* action, float* out = nullptr);

// Records HIP events around the launches made in its scope while
// profiling is on (gc_profile); a no-op otherwise.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  hipEvent_t start_ = nullptr, stop_ = nullptr;
};

}  // namespace gcx

#define GC_HIP_TRY(expr)                    \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return e_;        \
  } while (0)
