// PageRank iterations on gfx950: plain pull (Algorithm 1), plain push
// (Algorithm 2), TOCAB pull (Algorithm 4 + the Figure 5 merge) and TOCAB push
// (Algorithm 5), all with the same FP64 in-row accumulation and the same
// fused update, so the comparison between them isolates the blocking.
//
// Per iteration t (uniform dangling mode):
//   c[u]  = r[u] / outdeg(u) (0 when outdeg(u) = 0)      [contributions]
//   D     = sum of r[u] over outdeg(u) = 0                 [dangling mass]
//   s[v]  = sum over arcs u -> v of c[u]
//   r'[v] = (1 - d)/n + d * (s[v] + D/n)
// The update kernel of iteration t writes c for iteration t+1 and each of
// its work-groups a partial of the next D; the last work-group to finish
// adds the partials in a fixed order, so D is reproducible.

#include <climits>

#include "gc_device.h"
#include "gc_internal.h"

#include "gc_pr_device.h"

namespace {

// D for the next iteration: the partials summed in index order by one
// work-group (deterministic).
__global__ __launch_bounds__(1024) void k_reduce_dangling(const double* __restrict__ dpart, int32_t count,
                                                          double* __restrict__ dtotal) {
  __shared__ double part[1024 / kWave];
  double acc = 0.0;
  for (int32_t i = threadIdx.x; i < count; i += 1024) acc += dpart[i];
  acc = gcd::wave_sum(acc);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 1024 / kWave; ++w) t += part[w];
    *dtotal = t;
  }
}

// Contributions of the starting vector and its dangling mass; zeroes the
// push accumulators when given.
__global__ __launch_bounds__(kThreads) void k_pr_init(const float* __restrict__ rank_in, Update u,
                                                      double* __restrict__ sums) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  double mine = 0.0;
  if (v < u.n) {
    const float r = rank_in[v];
    const int32_t deg = u.rowptr[v + 1] - u.rowptr[v];
    u.contrib[v] = deg ? static_cast<float>(static_cast<double>(r) / deg) : 0.0f;
    mine = deg ? 0.0 : static_cast<double>(r);
    if (sums) sums[v] = 0.0;
  }
  publish_dangling(u, mine);
}

// Algorithm 4 over every subgraph in one launch. Local rows are stored block
// after block, so consecutive tiles stay inside one block and its slice of
// c stays cache resident: partial[l] = sum of c over local row l, written
// densely by local id.
__global__ __launch_bounds__(kThreads) void k_pr_tocab_pull(const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col,
                                                            const int32_t* __restrict__ tile_row,
                                                            const float* __restrict__ c,
                                                            float* __restrict__ partial) {
  __shared__ float vals[kStageCap];
  const int32_t r0 = tile_row[blockIdx.x], r1 = tile_row[blockIdx.x + 1];
  if (r0 >= r1) return;
  pull_tile(row_ptr, col, c, r0, r1, vals,
            [&](int32_t r, double s) { gcd::st_stream(partial + r, static_cast<float>(s)); });
}

// Algorithm 4 with the block's slice of c resident in LDS (block widths up
// to kLdsMaxWidth): gfx950 serves random 4-byte reads from LDS about ten
// times faster than from L2, so on this GPU the block is sized for the
// 160 KB LDS of a compute unit rather than for the last-level cache. One
// work-group takes a chunk of one block's local rows and loads the slice
// c[sW, sW + W) into LDS once (coalesced). Its waves then work
// independently on the kWaveTile-arc tiles covering the chunk: a wave
// stages the tile's gathered values (16-bit column offsets read as one
// 8-byte load per lane, values read from the LDS slice) in its own LDS
// strip, each lane sums whole rows that start in the tile, and the one row
// that may run past the tile's end is finished by the whole wave.
constexpr int kLdsThreads = 1024;
constexpr int kLdsWaves = kLdsThreads / kWave;
constexpr int kWaveTile = 4 * kWave;  // 4 arcs per lane

__global__ __launch_bounds__(kLdsThreads) void k_pr_tocab_pull_lds(
    const int32_t* __restrict__ row_ptr, const uint16_t* __restrict__ col16, const int32_t* __restrict__ wtile_row,
    const int32_t* __restrict__ chunk_beg, const int32_t* __restrict__ chunk_end, const int32_t* __restrict__ chunk_blk,
    int32_t log2W, int32_t n, int32_t m, const float* __restrict__ c, float* __restrict__ partial) {
  extern __shared__ float lds[];
  const int32_t W = 1 << log2W;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  float* slice = lds;
  float* stage = lds + W + wid * kWaveTile;
  const int32_t r0 = chunk_beg[blockIdx.x], r1 = chunk_end[blockIdx.x];
  if (r0 >= r1) return;
  const int32_t v0 = chunk_blk[blockIdx.x] << log2W;
  const int32_t cnt = min(W, n - v0);
  for (int32_t i = threadIdx.x; i < cnt; i += kLdsThreads) slice[i] = c[v0 + i];
  __syncthreads();
  const int32_t q0 = row_ptr[r0] / kWaveTile, q1 = (row_ptr[r1] - 1) / kWaveTile;
  for (int32_t q = q0 + wid; q <= q1; q += kLdsWaves) {
    const int32_t rb = max(r0, wtile_row[q]), re = min(r1, wtile_row[q + 1]);
    if (rb >= re) continue;  // no chunk row starts here (middle of a long row)
    const int32_t tb = q * kWaveTile;
    const int32_t te = min(tb + kWaveTile, m);
    uint16_t u[4];
    if (tb + kWaveTile <= m) {
      const uint64_t four = gcd::ld_stream(reinterpret_cast<const uint64_t*>(col16 + tb) + lane);
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = static_cast<uint16_t>(four >> (16 * j));
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = col16[min(tb + 4 * lane + j, m - 1)];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) stage[4 * lane + j] = slice[u[j]];
    wave_lds_fence();
    bool over = false;
    int32_t over_row = 0, over_end = 0;
    double over_sum = 0.0;
    for (int32_t r = rb + lane; r < re; r += kWave) {
      const int32_t b = row_ptr[r], e = row_ptr[r + 1];
      const int32_t ee = min(e, te);
      double sum = 0.0;
      for (int32_t i = b; i < ee; ++i) sum += static_cast<double>(stage[i - tb]);
      if (e > te) {  // only the tile's last row can run past its end
        over = true;
        over_row = r;
        over_end = e;
        over_sum = sum;
      } else {
        gcd::st_stream(partial + r, static_cast<float>(sum));
      }
    }
    const uint64_t ob = __ballot(over);
    if (ob) {
      const int owner = __ffsll(static_cast<long long>(ob)) - 1;
      const int32_t oe = __shfl(over_end, owner, kWave);
      double acc = 0.0;
      for (int32_t i = te + lane; i < oe; i += kWave) acc += static_cast<double>(slice[col16[i]]);
      acc = gcd::wave_sum(acc);
      if (lane == owner) partial[over_row] = static_cast<float>(over_sum + acc);
    }
    wave_lds_fence();  // the strip is rewritten by the next tile
  }
}

// Algorithm 1 with the update fused (same tiles over the transposed graph):
// reads c from one buffer and writes the next iteration's c into the other.
__global__ __launch_bounds__(kThreads) void k_pr_plain_pull(const int32_t* __restrict__ t_rowptr,
                                                            const int32_t* __restrict__ t_col,
                                                            const int32_t* __restrict__ tile_row,
                                                            const float* __restrict__ c_in, Update u) {
  __shared__ float vals[kStageCap];
  const int32_t r0 = tile_row[blockIdx.x], r1 = tile_row[blockIdx.x + 1];
  double mine = 0.0;
  if (r0 < r1) {
    const double D = *u.dtotal_in;
    pull_tile(t_rowptr, t_col, c_in, r0, r1, vals,
              [&](int32_t v, double s) { mine += update_vertex(u, v, s, D); });
  }
  publish_dangling(u, mine);
}

// Figure 5 merge fused with the update: work-group j owns vertices
// [j*K, (j+1)*K); it accumulates every block's partial sums for the range
// in LDS (merge_accumulate), then updates its vertices with coalesced writes.
template <int K, bool kFlat>
__global__ __launch_bounds__(kThreads) void k_pr_merge(const int32_t* __restrict__ range_ptr, int32_t B,
                                                       const uint16_t* __restrict__ id16,
                                                       const float* __restrict__ partial, Update u) {
  __shared__ double acc[K];
  merge_accumulate<K, kFlat>(range_ptr, B, id16, partial, blockIdx.x, acc);
  const int32_t v0 = blockIdx.x * K;
  const double D = *u.dtotal_in;
  double mine = 0.0;
  for (int i = threadIdx.x; i < K; i += kThreads) {
    const int32_t v = v0 + i;
    if (v < u.n) mine += update_vertex(u, v, acc[i], D);
  }
  publish_dangling(u, mine);
}

// Push with thread+warp+CTA style fine-grained balancing (Section 2.1,
// applied to push in Section 3.2): the work-group's 256 rows are laid end to
// end by an exclusive scan of their lengths and every lane takes one arc at
// a time, locating its row by binary search; each arc is an FP64 atomic add
// into sums[dst]. With id_map (Algorithm 5) rows are a push partition's
// local sources and the destinations of one block stay inside a W-wide
// slice of sums.
__global__ __launch_bounds__(kThreads) void k_pr_push(const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ id_map,
                                                      const int32_t* __restrict__ col,
                                                      const float* __restrict__ c, double* __restrict__ sums,
                                                      int64_t rows) {
  __shared__ int32_t start[kThreads];
  __shared__ int32_t first[kThreads];
  __shared__ float val[kThreads];
  __shared__ int32_t wave_tot[kThreads / kWave];
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  int32_t b = 0, len = 0;
  float cu = 0.0f;
  if (r < rows) {
    b = row_ptr[r];
    len = row_ptr[r + 1] - b;
    cu = c[id_map ? id_map[r] : static_cast<int32_t>(r)];
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int incl = gcd::wave_incl_scan(len);
  if (lane == kWave - 1) wave_tot[wid] = incl;
  __syncthreads();
  int off = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kThreads / kWave; ++w) {
    off += (w < wid) ? wave_tot[w] : 0;
    total += wave_tot[w];
  }
  start[threadIdx.x] = off + incl - len;
  first[threadIdx.x] = b;
  val[threadIdx.x] = cu;
  __syncthreads();
  for (int32_t a = threadIdx.x; a < total; a += kThreads) {
    int lo = 0, hi = kThreads - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (start[mid] <= a) lo = mid;
      else hi = mid - 1;
    }
    const int32_t e = first[lo] + (a - start[lo]);
    atomicAdd(&sums[col[e]], static_cast<double>(val[lo]));
  }
}

// Update after a push pass; clears sums for the next pass.
__global__ __launch_bounds__(kThreads) void k_pr_apply(double* __restrict__ sums, Update u) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  const double D = *u.dtotal_in;
  double mine = 0.0;
  if (v < u.n) {
    const double s = sums[v];
    sums[v] = 0.0;
    mine = update_vertex(u, v, s, D);
  }
  publish_dangling(u, mine);
}

template <int K>
void launch_merge(int32_t R, hipStream_t s, const int32_t* rp, int32_t B, const uint16_t* id16,
                  const float* partial, const Update& u) {
  if (B <= kFlatB) k_pr_merge<K, true><<<R, kThreads, 0, s>>>(rp, B, id16, partial, u);
  else k_pr_merge<K, false><<<R, kThreads, 0, s>>>(rp, B, id16, partial, u);
}

}  // namespace

namespace gcx {

int32_t pull_tile_arcs() { return kTileArcs; }

int32_t wave_tile_arcs() { return kWaveTile; }

hipError_t pagerank_setup() {
  // the LDS-resident pull holds a slice of up to kLdsMaxWidth floats plus one strip per wave
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pr_tocab_pull_lds),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(sizeof(float) * (kLdsMaxWidth + kLdsThreads * 4)));
}

hipError_t pagerank_run(gc_graph g, gc_tocab t, int32_t dir, float damping, int32_t dangling,
                        const float* rank_in, float* rank_out, int32_t iters, hipStream_t s) {
  const int32_t n = g->n;
  if (iters == 0)
    return hipMemcpyAsync(rank_out, rank_in, sizeof(float) * n, hipMemcpyDeviceToDevice, s);
  static const hipError_t setup = pagerank_setup();
  GC_HIP_TRY(setup);
  const bool push = t ? (t->dir == GC_PUSH) : (dir == GC_PUSH);
  Update u;
  u.d = damping;
  u.base = (1.0 - static_cast<double>(damping)) / n;
  u.inv_n = dangling == GC_DANGLING_UNIFORM ? 1.0 / n : 0.0;
  u.dpart = g->dpart;
  u.rowptr = g->rowptr;
  u.n = n;
  u.rank_out = nullptr;
  const int vgrid = (n + kThreads - 1) / kThreads;

  // contributions of rank_in and D of iteration 0 -> dtotal[0]
  u.dtotal_in = nullptr;
  u.contrib = g->contrib[0];
  {
    ProfScope prof("pr_init", s);
    k_pr_init<<<vgrid, kThreads, 0, s>>>(rank_in, u, push ? g->sums : nullptr);
  }
  k_reduce_dangling<<<1, 1024, 0, s>>>(g->dpart, vgrid, g->dtotal);
  GC_HIP_TRY(hipGetLastError());

  int cur = 0;
  for (int32_t it = 0; it < iters; ++it) {
    u.dtotal_in = g->dtotal + (it & 1);
    double* dtotal_out = g->dtotal + ((it + 1) & 1);
    u.rank_out = (it == iters - 1) ? rank_out : nullptr;
    int32_t parts = vgrid;  // work-groups of the update kernel
    if (t && !push) {
      if (t->col16) {
        ProfScope prof("pr_tocab_pull", s);
        const size_t lds = sizeof(float) * (static_cast<size_t>(t->W) + kLdsThreads * 4);
        k_pr_tocab_pull_lds<<<t->n_chunks, kLdsThreads, lds, s>>>(
            t->row_ptr, t->col16, t->wtile_row, t->chunk_beg, t->chunk_end, t->chunk_blk, t->log2W, n,
            static_cast<int32_t>(t->m), g->contrib[0], t->partial);
      } else {
        ProfScope prof("pr_tocab_pull", s);
        k_pr_tocab_pull<<<t->n_tiles, kThreads, 0, s>>>(t->row_ptr, t->col, t->tile_row, g->contrib[0],
                                                        t->partial);
      }
      u.contrib = g->contrib[0];  // safe in place: the pull pass has finished reading c
      parts = t->R;
      ProfScope prof("pr_merge", s);
      switch (t->k) {
        case 256: launch_merge<256>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, u); break;
        case 512: launch_merge<512>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, u); break;
        case 1024: launch_merge<1024>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, u); break;
        case 2048: launch_merge<2048>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, u); break;
        case 4096: launch_merge<4096>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, u); break;
        case 8192: launch_merge<8192>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, u); break;
        case 16384: launch_merge<16384>(t->R, s, t->range_ptr, t->B, t->id16, t->partial, u); break;
        default: return hipErrorInvalidValue;
      }
    } else if (!push) {
      u.contrib = g->contrib[cur ^ 1];
      parts = g->n_tiles_in;
      ProfScope prof("pr_plain_pull", s);
      k_pr_plain_pull<<<g->n_tiles_in, kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, g->tile_row_in,
                                                         g->contrib[cur], u);
      cur ^= 1;
    } else {
      if (t) {
        const int64_t P = t->P;
        if (P > 0) {
          ProfScope prof("pr_tocab_push", s);
          k_pr_push<<<static_cast<uint32_t>((P + kThreads - 1) / kThreads), kThreads, 0, s>>>(
              t->row_ptr, t->id_map, t->col, g->contrib[0], g->sums, P);
        }
      } else {
        ProfScope prof("pr_plain_push", s);
        k_pr_push<<<vgrid, kThreads, 0, s>>>(g->rowptr, nullptr, g->colidx, g->contrib[0], g->sums, n);
      }
      u.contrib = g->contrib[0];
      ProfScope prof("pr_apply", s);
      k_pr_apply<<<vgrid, kThreads, 0, s>>>(g->sums, u);
    }
    {
      ProfScope prof("pr_dangling", s);
      k_reduce_dangling<<<1, 1024, 0, s>>>(g->dpart, parts, dtotal_out);
    }
    GC_HIP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

}  // namespace gcx
