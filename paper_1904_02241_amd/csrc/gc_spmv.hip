// Sparse matrix-vector product over the graph's arcs in the pull direction
// (the SpMV benchmark of Section 4): y[v] = sum over arcs u -> v of
// val(u -> v) * x[u]. Plain: the pull tiles of the transposed graph.
// Blocked: Algorithm 4's column-blocked pull over a GC_PULL partition into
// per-(row, block) partial sums, then the Figure 5 merge writing y; blocks
// of at most 2^15 vertices go through the stream-layout kernels of PageRank
// (x's slice in LDS, values streamed beside the 16-bit columns). Products
// are FP32 (x times the arc's value), row and merge sums FP64 (inside a
// stream-layout tile FP32, as for PageRank), y FP32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gc_device.h"
#include "gc_internal.h"

#include "gc_pr_device.h"

namespace {

// Plain pull: one tile of the transposed graph per work-group.
__global__ __launch_bounds__(kThreads) void k_spmv_plain(const int32_t* __restrict__ t_rowptr,
                                                         const int32_t* __restrict__ t_col,
                                                         const int32_t* __restrict__ tile_row,
                                                         const float* __restrict__ x, ValuedArc arc,
                                                         float* __restrict__ y) {
  __shared__ float vals[kStageCap];
  const int32_t r0 = tile_row[blockIdx.x], r1 = tile_row[blockIdx.x + 1];
  if (r0 >= r1) return;
  pull_tile(t_rowptr, t_col, x, r0, r1, vals, [&](int32_t v, double s) { y[v] = static_cast<float>(s); }, arc);
}

// (Every vertex is a row of the transposed graph and the tile table covers
// all rows, so plain pull writes every y[v]; the merge ranges of the blocked
// form cover [0, n) as well.)

// Blocked pull (Algorithm 4): partial[l] = sum over the block's arcs of
// local row l, tiles block after block.
__global__ __launch_bounds__(kThreads) void k_spmv_tocab(const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col,
                                                         const int32_t* __restrict__ tile_row,
                                                         const float* __restrict__ x, ValuedArc arc,
                                                         float* __restrict__ partial) {
  __shared__ float vals[kStageCap];
  const int32_t r0 = tile_row[blockIdx.x], r1 = tile_row[blockIdx.x + 1];
  if (r0 >= r1) return;
  pull_tile(row_ptr, col, x, r0, r1, vals,
            [&](int32_t r, double s) { gcd::st_stream(partial + r, static_cast<float>(s)); }, arc);
}

// Figure 5 merge for SpMV: work-group j sums every block's partials of
// range [jK, (j+1)K) in LDS and writes y for the range.
template <int K, bool kFlat>
__global__ __launch_bounds__(kThreads) void k_spmv_merge(const int32_t* __restrict__ range_ptr, int32_t B,
                                                         const uint16_t* __restrict__ id16,
                                                         const float* __restrict__ partial, int32_t n,
                                                         float* __restrict__ y) {
  __shared__ double acc[K];
  merge_accumulate<K, kFlat>(range_ptr, B, id16, partial, blockIdx.x, acc);
  const int32_t v0 = blockIdx.x * K;
  for (int i = threadIdx.x; i < K; i += kThreads)
    if (v0 + i < n) y[v0 + i] = static_cast<float>(acc[i]);
}

template <int K>
void launch_spmv_merge(int32_t R, hipStream_t s, const int32_t* rp, int32_t B, const uint16_t* id16,
                       const float* partial, int32_t n, float* y) {
  if (B <= kFlatB) k_spmv_merge<K, true><<<R, kThreads, 0, s>>>(rp, B, id16, partial, n, y);
  else k_spmv_merge<K, false><<<R, kThreads, 0, s>>>(rp, B, id16, partial, n, y);
}

}  // namespace

namespace gcx {

hipError_t spmv_run(gc_graph g, gc_tocab t, const float* x, float* y, hipStream_t s) {
  if (!t) {
    ProfScope prof("spmv_plain", s);
    ValuedArc arc{g->weighted ? g->t_w : nullptr, g->values_f32};
    if (g->n_tiles_in > 0)
      k_spmv_plain<<<g->n_tiles_in, kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, g->tile_row_in, x, arc, y);
    return hipGetLastError();
  }
  if (t->col16) {  // stream layout: the LDS-resident pull of the PageRank kernels, valued
    const float* vals = nullptr;
    if (t->weighted) {
      GC_HIP_TRY(stream_values(g, t, s));
      vals = t->val32;
    }
    return spmv_stream(g, t, x, vals, y, s);
  }
  ValuedArc arc{t->weighted ? t->w : nullptr, g->values_f32};
  {
    ProfScope prof("spmv_tocab", s);
    if (t->n_tiles > 0) k_spmv_tocab<<<t->n_tiles, kThreads, 0, s>>>(t->row_ptr, t->col, t->tile_row, x, arc, t->partial);
  }
  ProfScope prof("spmv_merge", s);
  switch (t->k) {
    case 256: launch_spmv_merge<256>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, g->n, y); break;
    case 512: launch_spmv_merge<512>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, g->n, y); break;
    case 1024: launch_spmv_merge<1024>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, g->n, y); break;
    case 2048: launch_spmv_merge<2048>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, g->n, y); break;
    case 4096: launch_spmv_merge<4096>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, g->n, y); break;
    case 8192: launch_spmv_merge<8192>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, g->n, y); break;
    case 16384: launch_spmv_merge<16384>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, g->n, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gcx
