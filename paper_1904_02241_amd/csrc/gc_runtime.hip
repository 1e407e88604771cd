// Host side of the C ABI: error reporting, the device allocator hook,
// argument validation (done before anything is queued), handle lifetime.

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "gc_internal.h"

namespace {

thread_local char g_err[512] = "";

void* (*g_alloc)(size_t, hipStream_t, void*) = nullptr;
void (*g_release)(void*, hipStream_t, void*) = nullptr;
void* g_ctx = nullptr;

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  if (e == hipErrorOutOfMemory) return fail(GC_ENOMEM, "%s: out of device memory", where);
  return fail(GC_EHIP, "%s: %s", where, hipGetErrorString(e));
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int32_t ilog2(int64_t x) {
  int32_t r = 0;
  while ((int64_t(1) << r) < x) ++r;
  return r;
}

// Host-side structural check of an out-arc CSR (GC_VALIDATE).
int validate_host(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx, const int32_t* w) {
  if (rowptr[0] != 0) return fail(GC_EINVAL, "rowptr[0] = %d, expected 0", rowptr[0]);
  if (rowptr[n] != m) return fail(GC_EINVAL, "rowptr[n] = %d but m = %lld", rowptr[n], (long long)m);
  for (int32_t u = 0; u < n; ++u) {
    if (rowptr[u + 1] < rowptr[u]) return fail(GC_EINVAL, "rowptr decreases at row %d", u);
    for (int32_t j = rowptr[u]; j < rowptr[u + 1]; ++j) {
      const int32_t v = colidx[j];
      if (v < 0 || v >= n) return fail(GC_EINVAL, "colidx[%d] = %d out of range [0, %d)", j, v, n);
      if (v == u) return fail(GC_EINVAL, "self-loop at vertex %d", u);
      if (j > rowptr[u] && colidx[j - 1] >= v)
        return fail(GC_EINVAL, "row %d not strictly ascending at arc %d", u, j);
      if (w && w[j] <= 0) return fail(GC_EINVAL, "weight[%d] = %d is not positive", j, w[j]);
    }
  }
  return GC_OK;
}

// True when p is device memory (or managed memory) usable by kernels.
bool is_device_ptr(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

void free_graph(gc_graph g) {
  if (!g) return;
  void* bufs[] = {g->rowptr, g->colidx, g->w, g->t_rowptr, g->t_colidx, g->t_w, g->contrib[0], g->contrib[1],
                  g->sums, g->dpart, g->dtotal, g->counter, g->front, g->next, g->queue[0], g->queue[1],
                  g->stats, g->tile_row_in, g->visited, g->mark, g->lpart, g->ltotal, g->rank_tmp, g->bc_sigma,
                  g->bc_coef, g->bc_depth, g->bc_order, g->arc_deg,
                  g->arc_pre};
  for (void* p : bufs)
    if (p) gcx::dev_free(p, nullptr);
  if (g->stats_host) (void)hipHostFree(g->stats_host);
  delete g;
}

void free_tocab(gc_tocab t) {
  if (!t) return;
  void* bufs[] = {t->blk_rowoff, t->row_ptr, t->id_map, t->col, t->w, t->range_ptr, t->partial, t->pmin,
                  t->tile_row, t->col16, t->chunk_beg, t->chunk_end, t->chunk_blk, t->wtile_row, t->id16,
                  t->heads, t->seg, t->rstart, t->id16s, t->chunk_j0, t->chunk_ns, t->bc_part,
                  t->val32, t->w_pad, t->w8, t->xid16, t->xperm, t->xstart, t->xc, t->pcol16, t->pheads};
  for (void* p : bufs)
    if (p) gcx::dev_free(p, nullptr);
  delete t;
}

}  // namespace

namespace gcx {

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void* dev_alloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 1;
  if (g_alloc) return g_alloc(bytes, s, g_ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  if (g_release) g_release(p, s, g_ctx);
  else (void)hipFree(p);
}

}  // namespace gcx

// ---- pagerank_iter_noalloc: the same iterations with the library's static scratch

namespace {

// Device scratch of pagerank_iter_noalloc (contributions, dangling partials
// and totals, push accumulators, pull partial sums). Each GPU holds its own
// copy for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Address of the current device's scratch (looked up on the first call on
// that device, with it current).
hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of the buffers pagerank_run needs for this graph / form inside
// the scratch; returns the total.
struct NoAllocLayout {
  size_t contrib0, contrib1, dpart, dtotal, sums, partial, total;
};
NoAllocLayout noalloc_layout(gc_graph g, gc_tocab t, int32_t dir_if_plain) {
  const bool push = t ? (t->dir == GC_PUSH) : (dir_if_plain == GC_PUSH);
  const size_t n = static_cast<size_t>(g->n);
  NoAllocLayout l{};
  size_t off = 0;
  l.contrib0 = off;
  off += align256(sizeof(float) * n);
  l.contrib1 = off;
  off += align256(sizeof(float) * n);
  l.dpart = off;
  off += align256(sizeof(double) * static_cast<size_t>(g->dpart_slots));
  l.dtotal = off;
  off += align256(sizeof(double) * 2);
  l.sums = SIZE_MAX;
  if (push) {
    l.sums = off;
    off += align256(sizeof(double) * n);
  }
  l.partial = SIZE_MAX;
  if (t && !push) {  // the same slack as the partition's own partial buffer
    l.partial = off;
    off += align256(sizeof(float) * (static_cast<size_t>(t->P) + 8 + 512));
  }
  l.total = off;
  return l;
}

}  // namespace

extern "C" {

const char* gc_last_error(void) { return g_err; }

int gc_set_allocator(void* (*alloc)(size_t, hipStream_t, void*), void (*release)(void*, hipStream_t, void*),
                     void* ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail(GC_EINVAL, "gc_set_allocator: give both functions or neither");
  g_alloc = alloc;
  g_release = release;
  g_ctx = alloc ? ctx : nullptr;
  return GC_OK;
}

int graph_load_csr(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx, const int32_t* weight,
                   uint32_t flags, hipStream_t stream, gc_graph* out) {
  g_err[0] = '\0';
  if (!out) return fail(GC_EINVAL, "graph_load_csr: out is NULL");
  *out = nullptr;
  if (n <= 0) return fail(GC_EINVAL, "graph_load_csr: n = %d must be positive", n);
  if (n > INT32_MAX - 1) return fail(GC_EINVAL, "graph_load_csr: n too large");
  if (m < 0 || m >= INT32_MAX) return fail(GC_EINVAL, "graph_load_csr: m = %lld outside [0, 2^31)", (long long)m);
  if (!rowptr || (m > 0 && !colidx)) return fail(GC_EINVAL, "graph_load_csr: NULL rowptr or colidx");
  if (flags & ~(GC_DEVICE_PTRS | GC_VALIDATE | GC_VALUES_F32))
    return fail(GC_EINVAL, "graph_load_csr: unknown flags 0x%x", flags);
  if ((flags & GC_VALUES_F32) && !weight) return fail(GC_EINVAL, "graph_load_csr: GC_VALUES_F32 without values");
  const bool dev = (flags & GC_DEVICE_PTRS) != 0;

  if (flags & GC_VALIDATE) {
    std::vector<int32_t> hr, hc, hw;
    const int32_t *pr = rowptr, *pc = colidx, *pw = weight;
    if (dev) {
      hr.resize(static_cast<size_t>(n) + 1);
      hc.resize(static_cast<size_t>(m));
      if (weight) hw.resize(static_cast<size_t>(m));
      hipError_t e = hipMemcpy(hr.data(), rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost);
      if (e == hipSuccess && m > 0) e = hipMemcpy(hc.data(), colidx, sizeof(int32_t) * m, hipMemcpyDeviceToHost);
      if (e == hipSuccess && m > 0 && weight)
        e = hipMemcpy(hw.data(), weight, sizeof(int32_t) * m, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(e, "graph_load_csr (validate copy)");
      pr = hr.data();
      pc = hc.data();
      pw = weight ? hw.data() : nullptr;
    }
    const int rc = validate_host(n, m, pr, pc, (flags & GC_VALUES_F32) ? nullptr : pw);
    if (rc != GC_OK) return rc;
  } else if (!dev) {
    if (rowptr[0] != 0 || rowptr[n] != m)
      return fail(GC_EINVAL, "graph_load_csr: rowptr[0] must be 0 and rowptr[n] must equal m");
  }

  gc_graph g = new (std::nothrow) gc_graph_s;
  if (!g) return fail(GC_ENOMEM, "graph_load_csr: host allocation failed");
  g->n = n;
  g->m = m;
  g->weighted = weight != nullptr;
  g->values_f32 = (flags & GC_VALUES_F32) != 0;
  const size_t nb = sizeof(int32_t) * (static_cast<size_t>(n) + 1);
  const size_t mb = sizeof(int32_t) * static_cast<size_t>(m > 0 ? m : 1);
  g->dpart_slots = static_cast<int32_t>(std::max<int64_t>((n + 255) / 256, m / gcx::pull_tile_arcs() + 2));
  g->rowptr = static_cast<int32_t*>(gcx::dev_alloc(nb, stream));
  g->colidx = static_cast<int32_t*>(gcx::dev_alloc(mb, stream));
  g->t_rowptr = static_cast<int32_t*>(gcx::dev_alloc(nb, stream));
  g->t_colidx = static_cast<int32_t*>(gcx::dev_alloc(mb, stream));
  if (g->weighted) {
    g->w = static_cast<int32_t*>(gcx::dev_alloc(mb, stream));
    g->t_w = static_cast<int32_t*>(gcx::dev_alloc(mb, stream));
  }
  g->contrib[0] = static_cast<float*>(gcx::dev_alloc(sizeof(float) * n, stream));
  g->contrib[1] = static_cast<float*>(gcx::dev_alloc(sizeof(float) * n, stream));
  g->sums = static_cast<double*>(gcx::dev_alloc(sizeof(double) * n, stream));
  g->dpart = static_cast<double*>(gcx::dev_alloc(sizeof(double) * g->dpart_slots, stream));
  g->dtotal = static_cast<double*>(gcx::dev_alloc(sizeof(double) * 2, stream));
  g->counter = static_cast<unsigned*>(gcx::dev_alloc(sizeof(unsigned) * 4, stream));
  const size_t words = (static_cast<size_t>(n) + 31) / 32;
  g->front = static_cast<uint32_t*>(gcx::dev_alloc(sizeof(uint32_t) * words, stream));
  g->next = static_cast<uint32_t*>(gcx::dev_alloc(sizeof(uint32_t) * words, stream));
  g->queue[0] = static_cast<int32_t*>(gcx::dev_alloc(sizeof(int32_t) * n, stream));
  g->queue[1] = static_cast<int32_t*>(gcx::dev_alloc(sizeof(int32_t) * n, stream));
  g->stats = static_cast<int32_t*>(gcx::dev_alloc(sizeof(int32_t) * gcx::kStatSlots, stream));
  g->visited = static_cast<uint32_t*>(gcx::dev_alloc(sizeof(uint32_t) * ((static_cast<size_t>(n) + 31) / 32), stream));
  g->mark = static_cast<int32_t*>(gcx::dev_alloc(sizeof(int32_t) * n, stream));
  g->arc_deg = static_cast<int32_t*>(gcx::dev_alloc(sizeof(int32_t) * n, stream));
  g->arc_pre = static_cast<int32_t*>(gcx::dev_alloc(sizeof(int32_t) * (static_cast<size_t>(n) + 1), stream));
  bool ok = g->visited && g->mark && g->arc_deg && g->arc_pre && g->rowptr && g->colidx && g->t_rowptr && g->t_colidx && (!g->weighted || (g->w && g->t_w)) &&
            g->contrib[0] && g->contrib[1] && g->sums && g->dpart && g->dtotal && g->counter && g->front &&
            g->next && g->queue[0] && g->queue[1] && g->stats;
  if (ok && hipHostMalloc(reinterpret_cast<void**>(&g->stats_host), sizeof(int32_t) * gcx::kStatSlots,
                          hipHostMallocDefault) !=
                hipSuccess) {
    g->stats_host = nullptr;
    ok = false;
  }
  if (!ok) {
    free_graph(g);
    return fail(GC_ENOMEM, "graph_load_csr: device allocation failed");
  }
  {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      g->clock_khz = khz;
    (void)hipGetLastError();
  }
  g->bytes = 2 * static_cast<int64_t>(nb) + 2 * static_cast<int64_t>(mb) * (g->weighted ? 2 : 1) +
             12 * static_cast<int64_t>(n) + 8 * static_cast<int64_t>(words) + 8 * static_cast<int64_t>(n) +
             8 * static_cast<int64_t>(n) + 4;

  const hipMemcpyKind kind = hipMemcpyDefault;  // the runtime resolves host or device sources
  hipError_t e = hipMemcpyAsync(g->rowptr, rowptr, nb, kind, stream);
  if (e == hipSuccess && m > 0) e = hipMemcpyAsync(g->colidx, colidx, sizeof(int32_t) * m, kind, stream);
  if (e == hipSuccess && m > 0 && g->weighted) e = hipMemcpyAsync(g->w, weight, sizeof(int32_t) * m, kind, stream);
  int32_t bad = 0;
  if (e == hipSuccess) e = gcx::check_csr(n, m, g->rowptr, g->colidx, &bad, stream);
  if (e == hipSuccess && bad) {
    free_graph(g);
    return fail(GC_EINVAL, "graph_load_csr: %s", (bad & 1) ? "rowptr is not a valid offset array for m arcs"
                                                            : "a column index is outside [0, n)");
  }
  if (e == hipSuccess) e = hipMemsetAsync(g->counter, 0, sizeof(unsigned) * 4, stream);
  if (e == hipSuccess) e = hipMemsetAsync(g->dtotal, 0, sizeof(double) * 2, stream);
  if (e == hipSuccess)
    e = gcx::build_transpose(n, m, g->rowptr, g->colidx, g->w, g->t_rowptr, g->t_colidx, g->t_w, stream);
  if (e == hipSuccess)
    e = gcx::build_tiles(g->t_rowptr, n, m, gcx::pull_tile_arcs(), &g->tile_row_in, &g->n_tiles_in, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    free_graph(g);
    return hip_fail(e, "graph_load_csr");
  }
  *out = g;
  return GC_OK;
}

int graph_info(gc_graph g, int32_t* n, int64_t* m, int32_t* weighted) {
  if (!g) return fail(GC_EINVAL, "graph_info: NULL graph");
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (weighted) *weighted = g->weighted ? 1 : 0;
  return GC_OK;
}

int graph_export_transpose(gc_graph g, int32_t* t_rowptr, int32_t* t_colidx, int32_t* t_weight,
                           hipStream_t stream) {
  if (!g) return fail(GC_EINVAL, "graph_export_transpose: NULL graph");
  if (!t_rowptr || (g->m > 0 && !t_colidx)) return fail(GC_EINVAL, "graph_export_transpose: NULL output");
  if (t_weight && !g->weighted) return fail(GC_EINVAL, "graph_export_transpose: graph has no weights");
  hipError_t e = hipMemcpyAsync(t_rowptr, g->t_rowptr, sizeof(int32_t) * (g->n + 1), hipMemcpyDefault, stream);
  if (e == hipSuccess && g->m > 0)
    e = hipMemcpyAsync(t_colidx, g->t_colidx, sizeof(int32_t) * g->m, hipMemcpyDefault, stream);
  if (e == hipSuccess && g->m > 0 && t_weight)
    e = hipMemcpyAsync(t_weight, g->t_w, sizeof(int32_t) * g->m, hipMemcpyDefault, stream);
  return e == hipSuccess ? GC_OK : hip_fail(e, "graph_export_transpose");
}

int graph_free(gc_graph g) {
  if (!g) return fail(GC_EINVAL, "graph_free: NULL graph");
  (void)hipDeviceSynchronize();
  free_graph(g);
  return GC_OK;
}

int tocab_partition(gc_graph g, int32_t dir, int32_t block_width, int32_t merge_range, hipStream_t stream,
                    gc_tocab* out) {
  g_err[0] = '\0';
  if (!out) return fail(GC_EINVAL, "tocab_partition: out is NULL");
  *out = nullptr;
  if (!g) return fail(GC_EINVAL, "tocab_partition: NULL graph");
  if (dir != GC_PULL && dir != GC_PUSH) return fail(GC_EINVAL, "tocab_partition: dir must be GC_PULL or GC_PUSH");
  if (block_width == 0) {
    int32_t W = 0, k = 0;
    float ms = 0.0f;
    const int rc = tocab_autotune(g, dir, &W, &k, &ms, stream);
    if (rc != GC_OK) return rc;
    block_width = W;
    if (merge_range == 0) merge_range = k;
  }
  if (!is_pow2(block_width) || block_width < (1 << 10) || block_width > (1 << 26))
    return fail(GC_EINVAL, "tocab_partition: block_width %d is not a power of two in [2^10, 2^26]", block_width);
  if (merge_range == 0) merge_range = 4096;
  if (!is_pow2(merge_range) || merge_range < 256 || merge_range > (1 << 14))
    return fail(GC_EINVAL, "tocab_partition: merge_range %d is not a power of two in [256, 16384]", merge_range);
  const int64_t B = (static_cast<int64_t>(g->n) + block_width - 1) / block_width;
  const int64_t R = (static_cast<int64_t>(g->n) + merge_range - 1) / merge_range;
  if (B > 32768) return fail(GC_EINVAL, "tocab_partition: %lld blocks exceed 32768; use a wider block", (long long)B);
  if (B * (R + 1) > (int64_t(1) << 28))
    return fail(GC_EUNSUPPORTED, "tocab_partition: %lld x %lld range table too large; widen block or merge range",
                (long long)B, (long long)(R + 1));

  gc_tocab t = new (std::nothrow) gc_tocab_s;
  if (!t) return fail(GC_ENOMEM, "tocab_partition: host allocation failed");
  t->g = g;
  t->dir = dir;
  t->W = block_width;
  t->log2W = ilog2(block_width);
  t->k = merge_range;
  t->log2k = ilog2(merge_range);
  t->B = static_cast<int32_t>(B);
  t->R = static_cast<int32_t>(R);
  t->n_rows = g->n;
  t->n_cols = g->n;
  t->m = g->m;
  t->weighted = g->weighted;
  const int32_t* a_rowptr = dir == GC_PULL ? g->t_rowptr : g->rowptr;
  const int32_t* a_col = dir == GC_PULL ? g->t_colidx : g->colidx;
  const int32_t* a_w = dir == GC_PULL ? g->t_w : g->w;
  hipError_t e = gcx::build_partition(t, a_rowptr, a_col, a_w, stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(stream);
    free_tocab(t);
    return hip_fail(e, "tocab_partition");
  }
  *out = t;
  return GC_OK;
}

int tocab_autotune(gc_graph g, int32_t dir, int32_t* block_width, int32_t* merge_range, float* ms_per_iter,
                   hipStream_t stream) {
  if (!g) return fail(GC_EINVAL, "tocab_autotune: NULL graph");
  if (dir != GC_PULL && dir != GC_PUSH) return fail(GC_EINVAL, "tocab_autotune: dir must be GC_PULL or GC_PUSH");
  if (!block_width || !merge_range) return fail(GC_EINVAL, "tocab_autotune: NULL output");
  float ms = 0.0f;
  const hipError_t e = gcx::autotune(g, dir, 0, block_width, merge_range, &ms, stream);
  if (e != hipSuccess) return hip_fail(e, "tocab_autotune");
  if (ms_per_iter) *ms_per_iter = ms;
  return GC_OK;
}

int tocab_info(gc_tocab t, int32_t* B, int64_t* P, int32_t* W, int32_t* k, int32_t* dir, int64_t* bytes) {
  if (!t) return fail(GC_EINVAL, "tocab_info: NULL partition");
  if (B) *B = t->B;
  if (P) *P = t->P;
  if (W) *W = t->W;
  if (k) *k = t->k;
  if (dir) *dir = t->dir;
  if (bytes) *bytes = t->bytes;
  return GC_OK;
}

int tocab_layout(gc_tocab t, int32_t* stream_layout, int32_t* chunks, int64_t* table_bytes) {
  if (!t) return fail(GC_EINVAL, "tocab_layout: NULL partition");
  const bool st = t->col16 != nullptr;
  if (stream_layout) *stream_layout = st ? 1 : 0;
  if (chunks) *chunks = st ? t->n_chunks : 0;
  if (table_bytes) *table_bytes = st ? static_cast<int64_t>(sizeof(int2)) * t->B * (t->R + 1) : 0;
  return GC_OK;
}

int tocab_export(gc_tocab t, int32_t* blk_rowoff, int32_t* row_ptr, int32_t* id_map, int32_t* col,
                 int32_t* weight, int32_t* range_ptr, hipStream_t stream) {
  if (!t) return fail(GC_EINVAL, "tocab_export: NULL partition");
  if (!blk_rowoff || !row_ptr || !id_map || !col || !range_ptr) return fail(GC_EINVAL, "tocab_export: NULL output");
  const hipMemcpyKind k = hipMemcpyDefault;
  hipError_t e = hipMemcpyAsync(blk_rowoff, t->blk_rowoff, sizeof(int32_t) * (t->B + 1), k, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(row_ptr, t->row_ptr, sizeof(int32_t) * (t->P + 1), k, stream);
  if (e == hipSuccess && t->P > 0) e = hipMemcpyAsync(id_map, t->id_map, sizeof(int32_t) * t->P, k, stream);
  if (e == hipSuccess && t->m > 0) e = hipMemcpyAsync(col, t->col, sizeof(int32_t) * t->m, k, stream);
  if (e == hipSuccess && t->m > 0 && weight && t->weighted)
    e = hipMemcpyAsync(weight, t->w, sizeof(int32_t) * t->m, k, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(range_ptr, t->range_ptr, sizeof(int32_t) * (t->R + 1) * static_cast<size_t>(t->B), k, stream);
  return e == hipSuccess ? GC_OK : hip_fail(e, "tocab_export");
}

int tocab_free(gc_tocab t) {
  if (!t) return fail(GC_EINVAL, "tocab_free: NULL partition");
  (void)hipDeviceSynchronize();
  free_tocab(t);
  return GC_OK;
}

namespace {

// Checks shared by pagerank_iter and pagerank_converge (`who` names the call).
static int check_pagerank(const char* who, gc_graph g, gc_tocab t, int32_t dir_if_plain, float damping,
                   int32_t dangling, const float* rank_in, float* rank_out) {
  if (!g) return fail(GC_EINVAL, "%s: NULL graph", who);
  if (t && t->g != g) return fail(GC_EINVAL, "%s: partition belongs to another graph", who);
  if (!t && dir_if_plain != GC_PULL && dir_if_plain != GC_PUSH)
    return fail(GC_EINVAL, "%s: dir_if_plain must be GC_PULL or GC_PUSH", who);
  if (!(damping >= 0.0f && damping <= 1.0f)) return fail(GC_EINVAL, "%s: damping outside [0, 1]", who);
  if (dangling != GC_DANGLING_UNIFORM && dangling != GC_DANGLING_LEAK)
    return fail(GC_EINVAL, "%s: unknown dangling mode %d", who, dangling);
  if (!rank_in || !rank_out) return fail(GC_EINVAL, "%s: NULL rank buffer", who);
  if (!is_device_ptr(rank_in) || !is_device_ptr(rank_out))
    return fail(GC_EINVAL, "%s: rank buffers must be device memory", who);
  const char* a = reinterpret_cast<const char*>(rank_in);
  const char* b = reinterpret_cast<const char*>(rank_out);
  const size_t bytes = sizeof(float) * static_cast<size_t>(g->n);
  if (a < b + bytes && b < a + bytes) return fail(GC_EINVAL, "%s: rank_in and rank_out overlap", who);
  return GC_OK;
}

}  // namespace

int pagerank_iter(gc_graph g, gc_tocab t, int32_t dir_if_plain, float damping, int32_t dangling,
                  const float* rank_in, float* rank_out, int32_t iters, hipStream_t stream) {
  const int rc = check_pagerank("pagerank_iter", g, t, dir_if_plain, damping, dangling, rank_in, rank_out);
  if (rc != GC_OK) return rc;
  if (iters < 0) return fail(GC_EINVAL, "pagerank_iter: iters < 0");
  const hipError_t e = gcx::pagerank_run(g, t, dir_if_plain, damping, dangling, rank_in, rank_out, iters, stream);
  return e == hipSuccess ? GC_OK : hip_fail(e, "pagerank_iter");
}

int pagerank_iter_noalloc(gc_graph g, gc_tocab t, int32_t dir_if_plain, float damping, int32_t dangling,
                          const float* rank_in, float* rank_out, int32_t iters, hipStream_t stream) {
  const int rc = check_pagerank("pagerank_iter_noalloc", g, t, dir_if_plain, damping, dangling, rank_in, rank_out);
  if (rc != GC_OK) return rc;
  if (iters < 0) return fail(GC_EINVAL, "pagerank_iter_noalloc: iters < 0");
  const NoAllocLayout l = noalloc_layout(g, t, dir_if_plain);
  if (l.total > kNoAllocScratchBytes)
    return fail(GC_EINVAL, "pagerank_iter_noalloc: needs %zu bytes of scratch, more than its %zu-byte maximum",
                l.total, kNoAllocScratchBytes);
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return hip_fail(e, "pagerank_iter_noalloc (scratch address)");
  char* b = static_cast<char*>(base);
  gcx::PrBuffers buf;
  buf.contrib[0] = reinterpret_cast<float*>(b + l.contrib0);
  buf.contrib[1] = reinterpret_cast<float*>(b + l.contrib1);
  buf.dpart = reinterpret_cast<double*>(b + l.dpart);
  buf.dtotal = reinterpret_cast<double*>(b + l.dtotal);
  buf.sums = l.sums == SIZE_MAX ? nullptr : reinterpret_cast<double*>(b + l.sums);
  buf.partial = l.partial == SIZE_MAX ? nullptr : reinterpret_cast<float*>(b + l.partial);
  e = gcx::pagerank_run(g, t, dir_if_plain, damping, dangling, rank_in, rank_out, iters, stream, nullptr, -1, &buf);
  return e == hipSuccess ? GC_OK : hip_fail(e, "pagerank_iter_noalloc");
}

int pagerank_learned(gc_graph g, float damping, int32_t dangling, const float* rank_in, float* rank_out,
                     int32_t iters, int32_t* action, hipStream_t stream) {
  const int rc = check_pagerank("pagerank_learned", g, nullptr, GC_PULL, damping, dangling, rank_in, rank_out);
  if (rc != GC_OK) return rc;
  if (iters < 0) return fail(GC_EINVAL, "pagerank_learned: iters < 0");
  const gc_sched net = gcx::sched_for(g, 2);
  if (!net) return fail(GC_EINVAL, "pagerank_learned: no scheduler attached");
  const int32_t np = static_cast<int32_t>(g->sched_parts.size());
  const int32_t K = gcx::sched_actions(net);
  const int32_t fa = gcx::pagerank_fallback_action(g->sched_parts.data(), np);
  hipError_t e = hipSuccess;
  if (g->pr_learned_action < 0) {
    // Every iteration is alike, so the form is chosen once per attached
    // network. The working-set rule's form is timed (one warm-up iteration,
    // then two timed with HIP events), the network gets that time per arc as
    // its prior-level input, and its (at most two) picks predicted faster
    // than the rule's form by more than the gate are timed the same way; the
    // fastest measured form is kept. The network proposes, the clock decides:
    // a wrong prediction costs a few iterations once, never the run.
    auto time_form = [&](int32_t act, float* ms) -> hipError_t {
      gc_tocab ft = act >= 2 ? g->sched_parts[act - 2] : nullptr;
      const int32_t dir = act == 0 ? GC_PUSH : GC_PULL;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      hipError_t err = hipEventCreate(&e0);
      if (err == hipSuccess) err = hipEventCreate(&e1);
      if (err == hipSuccess) err = gcx::pagerank_run(g, ft, dir, damping, dangling, rank_in, rank_out, 1, stream);
      if (err == hipSuccess) err = hipEventRecord(e0, stream);
      if (err == hipSuccess) err = gcx::pagerank_run(g, ft, dir, damping, dangling, rank_in, rank_out, 2, stream);
      if (err == hipSuccess) err = hipEventRecord(e1, stream);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      if (err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      return err;
    };
    float fms = 0.0f;
    e = time_form(fa, &fms);
    if (e != hipSuccess) return hip_fail(e, "pagerank_learned: timing the fallback form");
    float feats[GC_SCHED_INPUTS];
    gcx::sched_features(g->n, g->m, g->n, g->m, 1, fms / 2.0, g->m, feats);
    std::vector<float> out(static_cast<size_t>(K));
    int32_t a = -1;
    e = gcx::sched_decide(net, feats, stream, &a, out.data());
    if (e != hipSuccess) return hip_fail(e, "pagerank_learned");
    int32_t best = fa;
    float best_ms = fms;
    if (a >= 0 && fa < K) {  // finite outputs
      std::vector<int32_t> order;
      for (int32_t c = 0; c < K && c < 2 + np; ++c)
        if (c != fa && out[c] + gcx::kLearnedGate < out[fa]) order.push_back(c);
      std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return out[x] < out[y]; });
      if (order.size() > 2) order.resize(2);
      for (int32_t c : order) {
        float ms = 0.0f;
        e = time_form(c, &ms);
        if (e != hipSuccess) return hip_fail(e, "pagerank_learned: timing a proposed form");
        if (ms < best_ms) {
          best = c;
          best_ms = ms;
        }
      }
    }
    g->pr_learned_action = best;
  }
  const int32_t a = g->pr_learned_action;
  if (action) *action = a;
  gc_tocab t = a >= 2 ? g->sched_parts[a - 2] : nullptr;
  e = gcx::pagerank_run(g, t, a == 0 ? GC_PUSH : GC_PULL, damping, dangling, rank_in, rank_out, iters, stream);
  return e == hipSuccess ? GC_OK : hip_fail(e, "pagerank_learned");
}

int pagerank_ladder(gc_graph g, gc_tocab t, int32_t method, float damping, int32_t dangling,
                    const float* rank_in, float* rank_out, int32_t iters, hipStream_t stream) {
  if (method < GC_LADDER_BASE || method > GC_LADDER_CB)
    return fail(GC_EINVAL, "pagerank_ladder: unknown method %d", method);
  if (method == GC_LADDER_CB && (!t || t->dir != GC_PULL))
    return fail(GC_EINVAL, "pagerank_ladder: GC_LADDER_CB needs a GC_PULL partition");
  const int rc = check_pagerank("pagerank_ladder", g, method == GC_LADDER_CB ? t : nullptr, GC_PULL, damping,
                                dangling, rank_in, rank_out);
  if (rc != GC_OK) return rc;
  if (iters < 0) return fail(GC_EINVAL, "pagerank_ladder: iters < 0");
  const hipError_t e = gcx::pagerank_run(g, t, GC_PULL, damping, dangling, rank_in, rank_out, iters, stream,
                                         nullptr, method);
  return e == hipSuccess ? GC_OK : hip_fail(e, "pagerank_ladder");
}

int spmv(gc_graph g, gc_tocab t, const float* x, float* y, hipStream_t stream) {
  if (!g) return fail(GC_EINVAL, "spmv: NULL graph");
  if (t && t->g != g) return fail(GC_EINVAL, "spmv: partition belongs to another graph");
  if (t && t->dir != GC_PULL) return fail(GC_EINVAL, "spmv: partition must be GC_PULL");
  if (!x || !y) return fail(GC_EINVAL, "spmv: NULL vector");
  if (!is_device_ptr(x) || !is_device_ptr(y)) return fail(GC_EINVAL, "spmv: vectors must be device memory");
  const char* a = reinterpret_cast<const char*>(x);
  const char* b = reinterpret_cast<const char*>(y);
  const size_t bytes = sizeof(float) * static_cast<size_t>(g->n);
  if (a < b + bytes && b < a + bytes) return fail(GC_EINVAL, "spmv: x and y overlap");
  const hipError_t e = gcx::spmv_run(g, t, x, y, stream);
  return e == hipSuccess ? GC_OK : hip_fail(e, "spmv");
}

int pagerank_converge(gc_graph g, gc_tocab t, int32_t dir_if_plain, float damping, int32_t dangling,
                      const float* rank_in, float* rank_out, double tol, int32_t max_iters, int32_t* iters_out,
                      double* delta_out, hipStream_t stream) {
  const int rc = check_pagerank("pagerank_converge", g, t, dir_if_plain, damping, dangling, rank_in, rank_out);
  if (rc != GC_OK) return rc;
  if (!(tol >= 0.0)) return fail(GC_EINVAL, "pagerank_converge: tol must be >= 0");
  if (max_iters < 1) return fail(GC_EINVAL, "pagerank_converge: max_iters < 1");
  if (!iters_out) return fail(GC_EINVAL, "pagerank_converge: NULL iters_out");
  if (!g->lpart) {  // first call on this graph: its convergence buffers
    g->lpart = static_cast<double*>(gcx::dev_alloc(sizeof(double) * g->dpart_slots, stream));
    g->ltotal = static_cast<double*>(gcx::dev_alloc(sizeof(double), stream));
    g->rank_tmp = static_cast<float*>(gcx::dev_alloc(sizeof(float) * std::max<int32_t>(g->n, 1), stream));
    if (!g->lpart || !g->ltotal || !g->rank_tmp) {
      for (void* p : {static_cast<void*>(g->lpart), static_cast<void*>(g->ltotal), static_cast<void*>(g->rank_tmp)})
        if (p) gcx::dev_free(p, stream);
      g->lpart = nullptr;
      g->ltotal = nullptr;
      g->rank_tmp = nullptr;
      return fail(GC_ENOMEM, "pagerank_converge: device allocation failed");
    }
  }
  gcx::Converge cv;
  cv.tol = tol;
  cv.max_iters = max_iters;
  const hipError_t e =
      gcx::pagerank_run(g, t, dir_if_plain, damping, dangling, rank_in, rank_out, max_iters, stream, &cv);
  if (e != hipSuccess) return hip_fail(e, "pagerank_converge");
  *iters_out = cv.iters;
  if (delta_out) *delta_out = cv.delta;
  return GC_OK;
}

int bfs_pull(gc_graph g, gc_tocab t, int32_t source, int32_t* depth, int32_t* levels, uint32_t policy,
             hipStream_t stream) {
  if (!g) return fail(GC_EINVAL, "bfs_pull: NULL graph");
  if (t && t->g != g) return fail(GC_EINVAL, "bfs_pull: partition belongs to another graph");
  if (t && t->dir != GC_PULL) return fail(GC_EINVAL, "bfs_pull: partition must be GC_PULL");
  if (source < 0 || source >= g->n) return fail(GC_EINVAL, "bfs_pull: source %d outside [0, %d)", source, g->n);
  if (!depth) return fail(GC_EINVAL, "bfs_pull: NULL depth");
  if (!is_device_ptr(depth)) return fail(GC_EINVAL, "bfs_pull: depth must be device memory");
  if (policy > GC_POLICY_LEARNED) return fail(GC_EINVAL, "bfs_pull: unknown policy %u", policy);
  if (policy == GC_POLICY_LEARNED && !gcx::sched_for(g, 0))
    return fail(GC_EINVAL, "bfs_pull: no scheduler attached");
  const hipError_t e = gcx::bfs_run(g, t, source, depth, levels, policy, stream);
  return e == hipSuccess ? GC_OK : hip_fail(e, "bfs_pull");
}

int sssp_pull(gc_graph g, gc_tocab t, int32_t source, int32_t* dist, int32_t* rounds, uint32_t policy,
              hipStream_t stream) {
  if (!g) return fail(GC_EINVAL, "sssp_pull: NULL graph");
  if (!g->weighted || g->values_f32) return fail(GC_EINVAL, "sssp_pull: graph has no integer weights");
  if (t && t->g != g) return fail(GC_EINVAL, "sssp_pull: partition belongs to another graph");
  if (t && t->dir != GC_PULL) return fail(GC_EINVAL, "sssp_pull: partition must be GC_PULL");
  if (source < 0 || source >= g->n) return fail(GC_EINVAL, "sssp_pull: source %d outside [0, %d)", source, g->n);
  if (!dist) return fail(GC_EINVAL, "sssp_pull: NULL dist");
  if (!is_device_ptr(dist)) return fail(GC_EINVAL, "sssp_pull: dist must be device memory");
  if (policy > GC_POLICY_LEARNED) return fail(GC_EINVAL, "sssp_pull: unknown policy %u", policy);
  if (policy == GC_POLICY_LEARNED && !gcx::sched_for(g, 1))
    return fail(GC_EINVAL, "sssp_pull: no scheduler attached");
  bool overflow = false;
  const hipError_t e = gcx::sssp_run(g, t, source, dist, rounds, policy, stream, &overflow);
  if (e != hipSuccess) return hip_fail(e, "sssp_pull");
  if (overflow) return fail(GC_EOVERFLOW, "sssp_pull: a distance reached INT32_MAX");
  return GC_OK;
}

int bc_accumulate(gc_graph g, gc_tocab t, const int32_t* sources, int32_t n_sources, double* bc, uint32_t policy,
                  hipStream_t stream) {
  if (!g) return fail(GC_EINVAL, "bc_accumulate: NULL graph");
  if (t && t->g != g) return fail(GC_EINVAL, "bc_accumulate: partition belongs to another graph");
  if (t && t->dir != GC_PULL) return fail(GC_EINVAL, "bc_accumulate: partition must be GC_PULL");
  if (n_sources < 0 || (n_sources > 0 && !sources))
    return fail(GC_EINVAL, "bc_accumulate: bad source list (%d sources)", n_sources);
  for (int32_t i = 0; i < n_sources; ++i)
    if (sources[i] < 0 || sources[i] >= g->n)
      return fail(GC_EINVAL, "bc_accumulate: source %d outside [0, %d)", sources[i], g->n);
  if (!bc) return fail(GC_EINVAL, "bc_accumulate: NULL bc");
  if (!is_device_ptr(bc)) return fail(GC_EINVAL, "bc_accumulate: bc must be device memory");
  if (policy > GC_POLICY_HEURISTIC) return fail(GC_EINVAL, "bc_accumulate: policy %u not supported", policy);
  const hipError_t e = gcx::bc_run(g, t, sources, n_sources, bc, policy, stream);
  return e == hipSuccess ? GC_OK : hip_fail(e, "bc_accumulate");
}

int traversal_trace(gc_graph g, int32_t* actions, float* ms, int32_t max, int32_t* count) {
  if (!g || !count || max < 0) return fail(GC_EINVAL, "traversal_trace: bad argument");
  const int32_t nl = static_cast<int32_t>(g->trace_action.size());
  for (int32_t i = 0; i < std::min(nl, max); ++i) {
    if (actions) actions[i] = g->trace_action[i];
    if (ms) ms[i] = g->trace_ms[i];
  }
  *count = nl;
  return GC_OK;
}

int sched_features(int32_t n, int64_t m, int32_t frontier, int64_t frontier_arcs, int32_t level, float prior_ms,
                   int64_t prior_arcs, float* features) {
  if (n <= 0 || m < 0 || frontier < 0 || frontier_arcs < 0 || level < 0 || prior_arcs < 0 || !(prior_ms >= 0.0f) ||
      !features)
    return fail(GC_EINVAL, "sched_features: bad argument");
  gcx::sched_features(n, m, frontier, frontier_arcs, level, prior_ms, prior_arcs, features);
  return GC_OK;
}

int sched_collect(gc_graph g, const gc_tocab* parts, int32_t n_parts, int32_t kind, const int32_t* sources,
                  int32_t n_sources, float* features, float* times_ms, int32_t max_rows, int32_t* rows,
                  hipStream_t stream) {
  if (!g || (n_parts > 0 && !parts) || n_parts < 0 || n_parts > 62 || (kind != 2 && !sources) || n_sources < 0 ||
      !features || !times_ms || max_rows < 0 || !rows)
    return fail(GC_EINVAL, "sched_collect: bad argument");
  if (kind < 0 || kind > 2) return fail(GC_EINVAL, "sched_collect: kind must be 0 (BFS), 1 (SSSP) or 2 (PageRank)");
  if (kind == 1 && !g->weighted) return fail(GC_EINVAL, "sched_collect: SSSP needs a weighted graph");
  for (int32_t i = 0; i < n_parts; ++i)
    if (!parts[i] || parts[i]->g != g || parts[i]->dir != GC_PULL)
      return fail(GC_EINVAL, "sched_collect: partition %d is not a GC_PULL partition of this graph", i);
  std::vector<gc_tocab> ps(parts, parts + n_parts);
  if (kind == 2) {  // PageRank: n_sources rows, sources unused
    const hipError_t e = gcx::collect_pagerank(g, ps.data(), n_parts, n_sources, features, times_ms, max_rows, rows,
                                               stream);
    return e == hipSuccess ? GC_OK : hip_fail(e, "sched_collect");
  }
  for (int32_t i = 0; i < n_sources; ++i)
    if (sources[i] < 0 || sources[i] >= g->n) return fail(GC_EINVAL, "sched_collect: source %d out of range", i);
  const hipError_t e = gcx::collect(g, ps.data(), n_parts, kind == 0, sources, n_sources, features, times_ms,
                                    max_rows, rows, stream);
  return e == hipSuccess ? GC_OK : hip_fail(e, "sched_collect");
}

int sched_attach(gc_graph g, gc_sched m, const gc_tocab* parts, int32_t n_parts) {
  if (!g) return fail(GC_EINVAL, "sched_attach: NULL graph");
  g->pr_learned_action = -1;  // pagerank_learned decides again for the new network
  if (!m) {
    g->sched = nullptr;
    for (gc_sched& k : g->sched_kind) k = nullptr;
    g->sched_parts.clear();
    return GC_OK;
  }
  if (n_parts < 0 || (n_parts > 0 && !parts)) return fail(GC_EINVAL, "sched_attach: bad partitions");
  if (gcx::sched_actions(m) != 2 + n_parts)
    return fail(GC_EINVAL, "sched_attach: network has %d outputs, needs 2 + %d", gcx::sched_actions(m), n_parts);
  for (int32_t i = 0; i < n_parts; ++i)
    if (!parts[i] || parts[i]->g != g || parts[i]->dir != GC_PULL)
      return fail(GC_EINVAL, "sched_attach: partition %d is not a GC_PULL partition of this graph", i);
  g->sched = m;
  for (gc_sched& k : g->sched_kind) k = nullptr;
  g->sched_parts.assign(parts, parts + n_parts);
  return GC_OK;
}

int sched_attach_kind(gc_graph g, int32_t kind, gc_sched m) {
  if (!g) return fail(GC_EINVAL, "sched_attach_kind: NULL graph");
  if (kind < 0 || kind > 2) return fail(GC_EINVAL, "sched_attach_kind: kind %d is not 0, 1 or 2", kind);
  if (m && !g->sched)
    return fail(GC_EINVAL, "sched_attach_kind: attach a network and its partitions with sched_attach first");
  if (m && gcx::sched_actions(m) != 2 + static_cast<int32_t>(g->sched_parts.size()))
    return fail(GC_EINVAL, "sched_attach_kind: network has %d outputs, needs 2 + %d", gcx::sched_actions(m),
                static_cast<int32_t>(g->sched_parts.size()));
  g->sched_kind[kind] = m;
  if (kind == 2) g->pr_learned_action = -1;
  return GC_OK;
}

int gc_sync(hipStream_t stream) {
  const hipError_t e = hipStreamSynchronize(stream);
  return e == hipSuccess ? GC_OK : hip_fail(e, "gc_sync");
}

}  // extern "C"
