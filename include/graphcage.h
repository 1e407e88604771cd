/*
 * graphcage.h - C ABI of the MI355X (gfx950) GraphCage / TOCAB library.
 *
 * GraphCage (Chen, "GraphCage: Cache Aware Graph Processing on GPUs", 2019)
 * runs vertex programs over a CSR graph in the pull direction (Algorithm 1)
 * or the push direction (Algorithm 2) and adds throughput-oriented cache
 * blocking (TOCAB, Section 3.1): a static 1D partition into subgraphs whose
 * vertex values fit in the last-level cache, processed one block after the
 * other (Algorithms 4 and 5) and merged range by range (Figure 5).
 *
 * Conventions shared by every call:
 *  - Every function returns a gc_status. Arguments are checked before any
 *    work is queued: on a non-zero return nothing was queued and no output
 *    was touched; gc_last_error() then holds a message (per thread).
 *  - Work is queued on the caller's HIP stream `stream` (NULL = the null
 *    stream). Calls return before the GPU finishes unless stated otherwise;
 *    device faults surface as GC_EHIP from a later synchronising call.
 *  - A graph or partition handle keeps per-iteration scratch inside it, so
 *    one handle must not be used from two streams at the same time.
 *  - Vertex ids are int32 in [0, n); arc counts m < 2^31.
 *  - Device buffers the caller passes stay owned by the caller.
 *  - Memory the library needs comes from the allocator set with
 *    gc_set_allocator (default: hipMalloc / hipFree).
 */
#ifndef GRAPHCAGE_H
#define GRAPHCAGE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GC_OK = 0,
  GC_EINVAL = -1,       /* bad argument or malformed graph                    */
  GC_ENOMEM = -2,       /* the allocator returned NULL                        */
  GC_EHIP = -3,         /* a HIP runtime call failed                          */
  GC_EUNSUPPORTED = -4, /* valid request the library does not handle         */
  GC_EOVERFLOW = -5     /* a result would not fit its integer type            */
} gc_status;

#define GC_UNREACHED INT32_MAX /* depth / distance of a vertex not reached     */

/* graph_load_csr flags */
#define GC_DEVICE_PTRS 1u /* rowptr/colidx/weight are device pointers          */
#define GC_VALIDATE 2u    /* check monotone rowptr, column range, sorted rows,  */
                          /* no self-loops and no duplicate arcs (host check)   */
#define GC_VALUES_F32 4u  /* weight holds FP32 arc values (bit patterns) for   */
                          /* spmv; such a graph has no integer weights          */

/* directions */
#define GC_PULL 0 /* gather over in-arcs (transposed graph); blocks by source  */
#define GC_PUSH 1 /* scatter over out-arcs; blocks by destination              */

/* PageRank treatment of vertices without out-arcs (the paper leaves it open) */
#define GC_DANGLING_UNIFORM 0 /* their rank is spread evenly (sum stays 1)     */
#define GC_DANGLING_LEAK 1    /* their rank leaves the system                   */

/* PageRank baselines of the paper's comparison (Section 4), pagerank_ladder */
#define GC_LADDER_BASE 0  /* pull, one lane per destination, serial in-arcs     */
#define GC_LADDER_VWC 1   /* pull, a virtual warp of 8 lanes per destination     */
#define GC_LADDER_VWC64 2 /* pull, a whole 64-lane wave per destination          */
#define GC_LADDER_CB 3    /* conventional column blocking: block after block,   */
                          /* row sums added straight into global FP64 sums      */

/* traversal policies (bfs_pull / sssp_pull) */
#define GC_POLICY_PULL 0      /* every level: topology-driven pull             */
#define GC_POLICY_PUSH 1      /* every level: data-driven push with a queue    */
#define GC_POLICY_HEURISTIC 2 /* per level: working-set rule of Section 3.3    */
#define GC_POLICY_LEARNED 3   /* per level: attached scheduler network (below), */
                              /* gated by and falling back to the heuristic     */

typedef struct gc_graph_s* gc_graph;
typedef struct gc_tocab_s* gc_tocab;
typedef struct gc_sched_s* gc_sched;

/* Message of the last failed call on this thread ("" if none). */
const char* gc_last_error(void);

/* Replaces the device allocator used for every buffer the library owns.
 * alloc(bytes, stream, ctx) returns device memory or NULL; release(ptr,
 * stream, ctx) gives it back. Both NULL restores hipMalloc / hipFree. Must
 * not be called while handles made with the previous allocator are alive. */
int gc_set_allocator(void* (*alloc)(size_t bytes, hipStream_t stream, void* ctx),
                     void (*release)(void* ptr, hipStream_t stream, void* ctx), void* ctx);

/* Loads a graph given as out-arc CSR (row = source; Section 2.1, "CSR
 * format"): rowptr int32[n+1], colidx int32[m], optional weight int32[m]
 * (NULL: unweighted). With GC_DEVICE_PTRS the arrays are device memory,
 * else host memory. The library copies them and builds on the GPU the
 * transposed CSR the pull direction reads (row = destination, columns sorted
 * ascending, weights carried along; Algorithm 1 takes G^T). Rows of the input
 * must be sorted ascending without duplicates or self-loops (checked with
 * GC_VALIDATE). Synchronises `stream` once. Free with graph_free. */
int graph_load_csr(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx,
                   const int32_t* weight, uint32_t flags, hipStream_t stream, gc_graph* out);

int graph_info(gc_graph g, int32_t* n, int64_t* m, int32_t* weighted);

/* Copies the transposed CSR (row = destination) into caller buffers (device
 * or host, any mix): t_rowptr int32[n+1], t_colidx int32[m], t_weight
 * int32[m] (may be NULL). Queued on `stream`. */
int graph_export_transpose(gc_graph g, int32_t* t_rowptr, int32_t* t_colidx, int32_t* t_weight,
                           hipStream_t stream);

int graph_free(gc_graph g);

/* TOCAB preprocessing (Section 3.1; Figures 3 and 4). dir = GC_PULL blocks
 * the transposed graph by source (column blocking), GC_PUSH blocks the graph
 * itself by destination (row blocking); the same code does both.
 * block_width W: power of two in [2^10, 2^26]; B = ceil(n / W) <= 32768;
 * 0 = chosen by tocab_autotune (with its merge range unless one is given).
 * merge_range k: power of two in [256, 16384], width of the merge ranges of
 * Figure 5 (0 = 4096, or the autotuned value when W = 0). Inside block s only rows with at least one arc there
 * get a local id, in ascending global order; id_map maps local to global.
 * A GC_PUSH partition with W <= 2^14 and k <= W (its block sums fit in LDS)
 * also holds the expanded-contribution form its PageRank iterations use:
 * the local rows in source-major order (int32 + uint16 per row), two FP32
 * buffers of one contribution per local row (written each iteration by the
 * work-group that updates the row's source), and the arcs as streams (16-bit
 * destination offsets, one head bit per arc): about 14P + 2.25m more bytes.
 * Synchronises `stream` once (it sizes its buffers). Free with tocab_free. */
int tocab_partition(gc_graph g, int32_t dir, int32_t block_width, int32_t merge_range,
                    hipStream_t stream, gc_tocab* out);

/* Chooses W and k for `dir` on this graph (the paper picks its subgraph
 * size with a sweep, Section 4.3): candidate widths 2^12 .. min(2^22, n)
 * are timed on PageRank iterations of the graph itself with successive
 * halving (2, 4, 8, ... iterations; the faster half survives each round),
 * then merge ranges 2048 / 4096 / 8192 are compared for the winner. Builds
 * and frees candidate partitions (needs room for one at a time), allocates
 * two rank vectors, synchronises `stream`. The result is cached per graph
 * signature (n, m, sampled offsets) for the life of the process.
 * ms_per_iter (nullable) receives the winner's time per iteration. */
int tocab_autotune(gc_graph g, int32_t dir, int32_t* block_width, int32_t* merge_range, float* ms_per_iter,
                   hipStream_t stream);

/* B, P (number of local rows over all blocks), W, k, direction and the
 * device bytes the partition holds. Any pointer may be NULL. */
int tocab_info(gc_tocab t, int32_t* B, int64_t* P, int32_t* W, int32_t* k, int32_t* dir,
               int64_t* bytes);

/* Pull layout of partition t: *stream_layout = 1 when its blocks are small
 * enough for the LDS-resident stream layout (16-bit columns, one head bit per
 * arc, range-major partial sums), else 0; *chunks = work-groups of its pull
 * kernel (0 without the stream layout); *table_bytes = bytes of its
 * range-major position table. Any output may be NULL. Returns GC_EINVAL for a
 * NULL partition. */
int tocab_layout(gc_tocab t, int32_t* stream_layout, int32_t* chunks, int64_t* table_bytes);

/* Copies the partition into caller buffers (device or host). Layout, blocks
 * concatenated in block order:
 *   blk_rowoff int32[B+1]   first local row of each block
 *   row_ptr    int32[P+1]   first arc of each local row
 *   id_map     int32[P]     global row of each local row (ascending per block)
 *   col        int32[m]     global column of each arc (ascending per row)
 *   weight     int32[m]     arc weights (NULL to skip; unweighted: ignored)
 *   range_ptr  int32[(R+1)*B], R = ceil(n / k): entry [j*B + s] is the first
 *              local row of block s whose global id is >= j*k.
 * Queued on `stream`. */
int tocab_export(gc_tocab t, int32_t* blk_rowoff, int32_t* row_ptr, int32_t* id_map, int32_t* col,
                 int32_t* weight, int32_t* range_ptr, hipStream_t stream);

int tocab_free(gc_tocab t);

/* PageRank iterations (Algorithm 1 pull, Algorithm 2 push; with t != NULL
 * Algorithm 4 + Figure 5 merge for a GC_PULL partition, Algorithm 5 for a
 * GC_PUSH partition). One iteration:
 *   c[u] = r[u] / outdeg(u) (0 if outdeg(u) = 0), s[v] = sum_{u->v} c[u],
 *   r'[v] = (1 - d)/n + d * (s[v] + D/n)   (UNIFORM, D = rank on vertices
 *                                          without out-arcs; LEAK: no D/n)
 * rank_in, rank_out: device float[n], must not overlap; after the call
 * rank_out holds iterate k + iters given iterate k in rank_in (iters = 0
 * copies). dir_if_plain selects pull or push when t == NULL. Precision:
 * ranks and contributions are stored as FP32. Plain pull, plain push, the
 * wide-block TOCAB pull (block width above 2^15) and TOCAB push accumulate
 * every row sum in FP64. The LDS-resident TOCAB pull (a GC_PULL partition
 * with block width at most 2^15, the stream layout) sums in FP32 within one
 * 512-arc tile (a lane's 8 arcs, then a wave-wide segmented scan), in FP64
 * for the part of a row carried from one tile to the next, and stores each
 * (row, block) partial sum as FP32; its merge adds the partials in FP64.
 * Queues work only: no host synchronisation and no allocation. */
int pagerank_iter(gc_graph g, gc_tocab t, int32_t dir_if_plain, float damping, int32_t dangling,
                  const float* rank_in, float* rank_out, int32_t iters, hipStream_t stream);

/* pagerank_iter for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results, but the per-call scratch
 * (contributions, dangling partials and totals, push accumulators, pull
 * partial sums) lives in a static device array of the library, 64 MiB per
 * GPU, held from library load until the process ends, instead of the
 * graph's and the partition's buffers. Needs, in bytes, each term rounded up
 * to 256:
 *   4n + 4n + 8 * max(ceil(n / 256), m / 2048 + 2) + 16
 *   + 8n               (push: plain push or a GC_PUSH partition)
 *   + 4(P + 520)       (a GC_PULL partition with P local rows)
 * and returns GC_EINVAL, queueing nothing, when that exceeds 64 MiB (a
 * plain pull of a graph with 16 arcs per vertex fits up to about 8.3
 * million vertices). Calls no allocator (hipMalloc, the gc_set_allocator
 * hook, or any library routine that allocates). Every call on one GPU shares that GPU's array, and the
 * array keeps the last call's contents: calls that overlap on one GPU (on
 * different streams or from different host threads) race and give wrong
 * results; serialise them. A GC_PUSH partition's expanded contributions
 * (see tocab_partition) stay in the partition, which holds them from its
 * construction: calls over one partition also race with each other.
 * Errors otherwise as pagerank_iter. */
int pagerank_iter_noalloc(gc_graph g, gc_tocab t, int32_t dir_if_plain, float damping, int32_t dangling,
                          const float* rank_in, float* rank_out, int32_t iters, hipStream_t stream);

/* PageRank until the change between consecutive iterates is small (the
 * "run until converged" protocol of Section 4; the paper leaves the test
 * unstated, the reading taken is the L1 norm): iterates exactly like
 * pagerank_iter and after iteration k computes
 *   delta_k = sum_v |r_k[v] - r_{k-1}[v]|   (FP64 over the FP32 iterates,
 *                                           fused into the update kernels)
 * stopping after the first k with delta_k <= tol, or after max_iters.
 * rank_in, rank_out: device float[n], must not overlap; rank_out receives
 * the last iterate. *iters_out (host) = iterations run; *delta_out (host,
 * NULL to skip) = the last delta. Synchronises `stream` once per iteration
 * to read delta_k. The first call on a graph allocates its convergence
 * buffers (an FP32 iterate and one FP64 slot per update work-group), freed
 * by graph_free. Errors: GC_EINVAL for bad arguments (tol < 0 or NaN,
 * max_iters < 1, NULL iters_out, plus pagerank_iter's checks), GC_ENOMEM. */
int pagerank_converge(gc_graph g, gc_tocab t, int32_t dir_if_plain, float damping, int32_t dangling,
                      const float* rank_in, float* rank_out, double tol, int32_t max_iters, int32_t* iters_out,
                      double* delta_out, hipStream_t stream);

/* The baselines TOCAB is compared with in Section 4, same iteration and
 * arguments as pagerank_iter: GC_LADDER_BASE (a straightforward pull, one
 * lane per vertex), GC_LADDER_VWC / GC_LADDER_VWC64 (virtual-warp-centric
 * mapping of Section 2.1 with 8 / 64 lanes per vertex), GC_LADDER_CB (the
 * conventional cache blocking Section 3.1 starts from: the column blocks of
 * t, which must be a GC_PULL partition, run one launch after another and
 * add every local row's sum into the global sums; t is ignored otherwise).
 * Sums are FP64 inside a row, ranks FP32. GC_LADDER_CB synchronises `stream` once
 * per call to read the block row offsets; the others only queue work.
 * Errors as pagerank_iter, plus GC_EINVAL for an unknown method or a
 * missing / push partition with GC_LADDER_CB. */
int pagerank_ladder(gc_graph g, gc_tocab t, int32_t method, float damping, int32_t dangling,
                    const float* rank_in, float* rank_out, int32_t iters, hipStream_t stream);

/* Sparse matrix-vector product over the arcs in the pull direction (the
 * SpMV benchmark of Section 4; the generalised SpMV that Algorithm 1
 * follows): y[v] = sum over arcs u -> v of val(u -> v) * x[u], i.e.
 * y = A^T x for the loaded out-arc CSR A. val is the arc's FP32 value for a
 * graph loaded with GC_VALUES_F32, its integer weight converted to FP32 for
 * other weighted graphs, 1 for unweighted ones. t == NULL: plain pull; t, a
 * GC_PULL partition of g: column-blocked pull (Algorithm 4) into partial
 * sums per (row, block), then the Figure 5 merge. Products are FP32 and y
 * is FP32. Sums are FP64 inside a row for plain pull and for blocks wider
 * than 2^15; for the stream layout (block width at most 2^15) they are FP32
 * within one 512-arc tile and FP64 across tiles, the (row, block) partials
 * are FP32, and the merge adds them in FP64. x, y: device float[n], must
 * not overlap. Queues work only.
 * Errors: GC_EINVAL for bad arguments (NULL or overlapping vectors, host
 * memory, a partition of another graph or a GC_PUSH partition). */
int spmv(gc_graph g, gc_tocab t, const float* x, float* y, hipStream_t stream);

/* Breadth-first search from `source` over out-arcs. depth: device
 * int32[n] out, depth[source] = 0, GC_UNREACHED when unreachable. The pull
 * levels are topology driven with status arrays (Section 3.3): with a
 * GC_PULL partition t they run blocked, each block writing a local `next`
 * that the merge reduces; t == NULL pulls over the whole transposed graph.
 * policy chooses pull, data-driven push, or the working-set heuristic per
 * level (direction by the direction-optimising test; the form of a pull
 * level by the working-set test, except over a partition with the LDS
 * stream layout (blocks up to 2^15), where a pull level runs as TOCAB on
 * graphs with at most 10 arcs per vertex while at least 1/64 of the arcs
 * end at unvisited vertices, as plain pull otherwise). levels (host,
 * nullable) receives the number of levels run. Synchronises `stream` once
 * per level to read the frontier size. */
int bfs_pull(gc_graph g, gc_tocab t, int32_t source, int32_t* depth, int32_t* levels,
             uint32_t policy, hipStream_t stream);

/* Single-source shortest paths from `source` over out-arcs with the graph's
 * positive weights: synchronous Bellman-Ford rounds that relax the in-arcs
 * of every vertex from the vertices changed in the previous round (min-merge
 * over blocks with a GC_PULL partition), or data-driven push rounds, chosen
 * by `policy` as for bfs_pull. dist: device int32[n] out, GC_UNREACHED when
 * unreachable. Requires a weighted graph (GC_EINVAL otherwise). Distances
 * are int32: if a finite distance would reach INT32_MAX the call returns
 * GC_EOVERFLOW (dist is then not meaningful). rounds (host, nullable)
 * receives the number of rounds. Synchronises once per round. */
int sssp_pull(gc_graph g, gc_tocab t, int32_t source, int32_t* dist, int32_t* rounds,
              uint32_t policy, hipStream_t stream);

/* Betweenness centrality restricted to a source set (the BC benchmark of
 * Section 4, Brandes' accumulation): for every source s in `sources` (host
 * int32[n_sources], each in [0, n)), a BFS over out-arcs counts shortest
 * paths sigma_s (a vertex one level down adds sigma_s of each in-neighbour on
 * the level above, Algorithm 3's update), then the dependencies
 * delta_s(v) = sum over arcs v -> w with depth(w) = depth(v) + 1 of
 * sigma_s(v) / sigma_s(w) * (1 + delta_s(w)) are formed deepest level first
 * and delta_s(v) is ADDED to bc[v] for every v != s. bc: device double[n],
 * accumulated into (clear it first for a fresh sum). Path counts and
 * dependencies are FP64; path counts stay exact below 2^53. Forward levels
 * run as chosen by `policy` (GC_POLICY_PULL: TOCAB pull over the GC_PULL
 * partition t with FP64 per-block partials and the Figure 5 merge, or plain
 * pull with t == NULL; GC_POLICY_PUSH; GC_POLICY_HEURISTIC); GC_POLICY_LEARNED
 * is refused. The first call allocates 20 bytes per vertex on g (and 8 per
 * local row on t), freed with them. Synchronises `stream` once per level;
 * returns after the last source's work is complete. The per-level record of
 * traversal_trace covers the forward levels of every source in turn.
 * Errors: GC_EINVAL for bad arguments (NULL or host bc, a source out of
 * range, a partition of another graph or a GC_PUSH one, the learned policy). */
int bc_accumulate(gc_graph g, gc_tocab t, const int32_t* sources, int32_t n_sources, double* bc,
                  uint32_t policy, hipStream_t stream);

/* Per-level record of the last bfs_pull / sssp_pull on g: actions[i] is the
 * way level i ran (0 push, 1 plain pull, 2 TOCAB pull with the call's
 * partition, or 2 + j for the j-th partition attached with sched_attach) and
 * ms[i] its wall time including the level's synchronisation. Up to `max`
 * entries are written; *count receives the number of levels. */
int traversal_trace(gc_graph g, int32_t* actions, float* ms, int32_t max, int32_t* count);

/* ---- learned level scheduler ---------------------------------------------
 * Not in the paper: a small network that picks, per traversal level, among
 * data-driven push, plain topology-driven pull and TOCAB pull over one of
 * several block widths, trained on per-level timings the traversal itself
 * produces. Network: GC_SCHED_INPUTS -> GC_SCHED_HIDDEN -> GC_SCHED_HIDDEN ->
 * K, ReLU after the hidden layers, FP32; output k scores action k (lower is
 * faster: a predicted log time, or log time over the level's fastest action,
 * as the training targets define). On a traversal level the working-set
 * heuristic keeps the direction (push or pull); on a pull level the
 * network's arg-min over the pull forms (plain pull, TOCAB pull per attached
 * width) replaces the heuristic's form only when its output is lower than
 * that form's output by more than 0.3 (about 35 % predicted gain with
 * relative log-time targets); the heuristic alone decides when an output is
 * not finite. A trained network clamps each input into the range it saw in
 * training (sched_train records it), so a level outside that range is
 * decided as the nearest trained one. For every traversal level after the
 * first, the network runs on the device in a one-work-group kernel queued
 * right after the previous level (it stops at once when the rule's
 * direction for the next level is push), on counters that never leave the
 * device, and its answer returns with the level's counters (no
 * synchronisation of its own). Parameters, row-major:
 *   W1[64][6], b1[64], W2[64][64], b2[64], W3[K][64], b3[K].
 * Features of a level (sched_features): log1p(frontier size), log1p(frontier
 * out-arcs), log1p(m / n), log2(ceil(n / 2^18) + 1), level / 16,
 * log1p(previous level's time per out-arc of its frontier, in ns; 0 at the
 * first level). Level times are the device's own clock from a level's start
 * to the end of its relaxation kernels. */
#define GC_SCHED_INPUTS 6
#define GC_SCHED_HIDDEN 64

int sched_param_count(int32_t n_actions, int64_t* count);
/* New network with K = n_actions outputs (1..64) from initial parameters
 * (host or device, sched_param_count floats; the caller draws them). */
int sched_create(int32_t n_actions, const float* params, gc_sched* out);
int sched_get_params(gc_sched m, float* params, hipStream_t stream);
/* y[batch][K] = network(x[batch][6]); device buffers. */
int sched_forward(gc_sched m, const float* x, int32_t batch, float* y, hipStream_t stream);
/* Masked mean squared error sum(mask (y - t)^2) / sum(mask) of the outputs
 * against targets t (log ms), and its gradient with respect to the
 * parameters (same layout); device buffers; deterministic. */
int sched_loss_grad(gc_sched m, const float* x, const float* t, const float* mask, int32_t batch, float* loss,
                    float* grad, hipStream_t stream);
/* `steps` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8) at rate
 * lr; loss_hist (device, nullable) receives the loss before each step. */
int sched_train(gc_sched m, const float* x, const float* t, const float* mask, int32_t batch, int32_t steps, float lr,
                float* loss_hist, hipStream_t stream);
int sched_free(gc_sched m);
/* The 6 features of a level (the library computes the same on the device
 * for its per-level decisions). prior_ms = time of the previous level,
 * prior_arcs = out-arcs of that level's frontier (both 0 at the first level). */
int sched_features(int32_t n, int64_t m, int32_t frontier, int64_t frontier_arcs, int32_t level, float prior_ms,
                   int64_t prior_arcs, float* features);
/* Training rows for a network with K = 2 + n_parts actions: traverses from
 * each source (kind 0 = BFS, 1 = SSSP) and at every level runs every action
 * from the same saved state, timing each with HIP events, then continues with
 * the fastest. kind 2 = PageRank: every vertex is active at every iteration,
 * so a row is one all-active level: each action (0 plain push, 1 plain
 * pull, 2 + i TOCAB pull over parts[i]) runs 4 iterations from the same
 * ranks and times_ms holds its time per iteration; the row's features are
 * those pagerank_learned uses (level 1, prior time = the working-set form's
 * time per iteration); n_sources rows are collected (sources is unused and
 * may be NULL), each from the previous row's fastest result. BFS / SSSP
 * rows give the prior-level input from the device clock stamps, as the
 * learned traversal does. Writes host features[rows][6] and times_ms[rows][K]
 * (up to max_rows) and *rows. parts must be GC_PULL partitions of g. */
int sched_collect(gc_graph g, const gc_tocab* parts, int32_t n_parts, int32_t kind, const int32_t* sources,
                  int32_t n_sources, float* features, float* times_ms, int32_t max_rows, int32_t* rows,
                  hipStream_t stream);
/* Attaches network m (K = 2 + n_parts) and its TOCAB partitions to g for
 * GC_POLICY_LEARNED and pagerank_learned; m = NULL detaches. The handles
 * must outlive the use. */
int sched_attach(gc_graph g, gc_sched m, const gc_tocab* parts, int32_t n_parts);
/* Attaches network m for one kind of work only (kind 0 = BFS, 1 = SSSP,
 * 2 = PageRank) over the partitions of the last sched_attach (m must have
 * the same K = 2 + n_parts); m = NULL returns that kind to the network of
 * sched_attach, which also clears every per-kind network. The six level
 * inputs do not say which operation runs, and the fastest action for the
 * same frontier differs between them (a BFS pull gathers status bits, an
 * SSSP pull 4-byte distances), so a network per kind can learn each one's
 * choices. GC_EINVAL before any sched_attach or on a K mismatch. */
int sched_attach_kind(gc_graph g, int32_t kind, gc_sched m);
/* PageRank (as pagerank_iter, `iters` iterations) in the form chosen for
 * g: 0 plain push, 1 plain pull, 2 + j TOCAB pull over the j-th attached
 * partition. The working-set rule's form for an all-active level is TOCAB
 * pull over the attached partition whose width is nearest 2^18 (plain pull
 * when none is attached). Every iteration is alike, so the choice is made
 * once per attached network, by the first call: it runs that form for 3
 * iterations from rank_in (1 warm-up, 2 timed with HIP events; their result
 * is discarded), feeds the network an all-active level (frontier n vertices
 * and m arcs, level 1, prior time = the timed iteration), times the same way
 * the (at most two) forms the network predicts faster than the rule's by
 * more than the gate above, and keeps the fastest measured form (the rule's
 * form when an output is not finite). That first call synchronises `stream`
 * up to four times; later calls only queue work.
 * *action (host, nullable) receives the form run. Errors as pagerank_iter,
 * plus GC_EINVAL when no network is attached. */
int pagerank_learned(gc_graph g, float damping, int32_t dangling, const float* rank_in, float* rank_out,
                     int32_t iters, int32_t* action, hipStream_t stream);

/* ---- batched persistent form ----------------------------------------------
 * Not in the paper: PageRank on many graphs of uneven size, each over its
 * own TOCAB pull partition (merge range 1024; widths[i] = 0 lets the
 * autotuner choose among widths >= 2^16, whose slices stay in the
 * last-level cache), together with personalised PageRank
 *   r'[v] = (1 - d) p[v] + d (s[v] + D p[v]),  r0 = p = one-hot(seed)
 * for up to 64 seeds on one graph (one lane per seed, an N x 64 FP32 state),
 * all iterations in ONE persistent kernel launch whose phases are separated
 * by grid barriers. The grid holds as many work-groups as stay resident; a
 * barrier that waits too long sets a flag (batch_status) and every
 * work-group leaves, so the launch always ends. */
typedef struct gc_batch_s* gc_batch;

/* Builds partitions and per-graph state (synchronises). The graph handles
 * must outlive the batch. n_graphs may be 0 (PPR only) and n_seeds 0. */
int batch_create(const gc_graph* graphs, int32_t n_graphs, const int32_t* block_widths, gc_graph ppr_graph,
                 const int32_t* seeds, int32_t n_seeds, hipStream_t stream, gc_batch* out);
/* rank_offsets[n_graphs + 1]: each graph's slice of the concatenated rank
 * vectors; block_widths[n_graphs]; grid = persistent work-groups. */
int batch_info(gc_batch b, int64_t* rank_offsets, int32_t* block_widths, int32_t* grid, int64_t* bytes);
/* Queues the launch: `iters` iterations on every graph from ranks_in
 * (device float[total n], concatenated) into ranks_out, and PPR into
 * ppr_out (device float[n][n_seeds]). No allocation, no host sync. */
int batch_run(gc_batch b, float damping, int32_t iters, const float* ranks_in, float* ranks_out, float* ppr_out,
              hipStream_t stream);
/* Captures batch_run with these arguments into a HIP graph (replaces any
 * earlier capture); batch_launch replays it on `stream`. */
int batch_capture(gc_batch b, float damping, int32_t iters, const float* ranks_in, float* ranks_out, float* ppr_out);
int batch_launch(gc_batch b, hipStream_t stream);
/* Synchronises `stream`; *barrier_timeout = 1 if the last launch's barrier
 * gave up waiting (its results are then not valid). */
int batch_status(gc_batch b, hipStream_t stream, int32_t* barrier_timeout);
int batch_free(gc_batch b);

/* Waits for `stream` and reports a pending asynchronous HIP error. */
int gc_sync(hipStream_t stream);

/* Measurement support. While on, every kernel launch is bracketed by a
 * pair of HIP events recorded on the launching stream, so per-kernel device
 * time can be read back without an external profiler. enable = 1 clears
 * old records and starts, 0 stops. gc_profile_count gives the number of
 * distinct kernels recorded; gc_profile_get returns, for index in [0,
 * count), the kernel's name (NUL-terminated, truncated to name_len), its
 * summed event time in ms and its number of launches. Both wait for the
 * recorded events to complete. */
int gc_profile(int32_t enable);
int gc_profile_count(int32_t* count);
int gc_profile_get(int32_t index, char* name, int32_t name_len, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* GRAPHCAGE_H */
