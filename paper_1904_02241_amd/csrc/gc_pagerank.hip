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

namespace {

using gcd::kWave;

constexpr int kThreads = 256;
constexpr int kHeavyRow = 32;  // longer rows are summed by a whole wave

struct Update {
  double base;      // (1 - d) / n
  double d;         // damping
  double inv_n;     // 1 / n, applied to D in uniform mode (0 in leak mode)
  const double* dtotal_in;
  double* dtotal_out;
  double* dpart;
  unsigned* counter;
  const int32_t* rowptr;  // out-arc CSR: outdeg(v) = rowptr[v+1] - rowptr[v]
  float* contrib;         // written for the next iteration
  float* rank_out;        // written on the last iteration only (else null)
  int32_t n;
};

// r'[v] from the neighbour sum; writes c'[v] (and r'[v] on the last pass),
// returns r'[v] when v has no out-arcs (its share of the next D), else 0.
__device__ __forceinline__ double update_vertex(const Update& u, int32_t v, double sum, double D) {
  const double r = u.base + u.d * (sum + D * u.inv_n);
  const float r32 = static_cast<float>(r);
  const int32_t deg = u.rowptr[v + 1] - u.rowptr[v];
  u.contrib[v] = deg ? static_cast<float>(static_cast<double>(r32) / deg) : 0.0f;
  if (u.rank_out) u.rank_out[v] = r32;
  return deg ? 0.0 : static_cast<double>(r32);
}

// Work-group sum of one double per thread (fixed reduction tree).
__device__ __forceinline__ double wg_sum(double x) {
  __shared__ double part[kThreads / kWave];
  x = gcd::wave_sum(x);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kThreads / kWave; ++w) t += part[w];
  __syncthreads();
  return t;
}

// Publishes this work-group's dangling partial; the last work-group to
// arrive sums all partials in index order into *dtotal_out and resets the
// arrival counter for the next launch.
__device__ void finish_dangling(const Update& u, double mine) {
  __shared__ bool last;
  const double total_mine = wg_sum(mine);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&u.dpart[blockIdx.x], total_mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned prev = atomicAdd(u.counter, 1u);
    last = prev == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < gridDim.x; i += kThreads)
    acc += __hip_atomic_load(&u.dpart[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double total = wg_sum(acc);
  if (threadIdx.x == 0) {
    *u.dtotal_out = total;
    __hip_atomic_store(u.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Contributions of the starting vector and its dangling mass; zeroes the
// push accumulators when given.
__global__ __launch_bounds__(kThreads) void k_pr_init(const float* __restrict__ rank_in, Update u,
                                                      float* __restrict__ sums) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  double mine = 0.0;
  if (v < u.n) {
    const float r = rank_in[v];
    const int32_t deg = u.rowptr[v + 1] - u.rowptr[v];
    u.contrib[v] = deg ? static_cast<float>(static_cast<double>(r) / deg) : 0.0f;
    mine = deg ? 0.0 : static_cast<double>(r);
    if (sums) sums[v] = 0.0f;
  }
  finish_dangling(u, mine);
}

// Sum of c over one row's columns [b, e), four loads in flight per step.
__device__ __forceinline__ double row_sum(const int32_t* __restrict__ col, const float* __restrict__ c,
                                          int32_t b, int32_t e) {
  double s = 0.0;
  int32_t i = b;
  for (; i + 4 <= e; i += 4) {
    const int32_t c0 = gcd::ld_stream(col + i), c1 = gcd::ld_stream(col + i + 1);
    const int32_t c2 = gcd::ld_stream(col + i + 2), c3 = gcd::ld_stream(col + i + 3);
    const float x0 = c[c0], x1 = c[c1], x2 = c[c2], x3 = c[c3];
    s += static_cast<double>(x0) + static_cast<double>(x1) + static_cast<double>(x2) + static_cast<double>(x3);
  }
  for (; i < e; ++i) s += static_cast<double>(c[gcd::ld_stream(col + i)]);
  return s;
}

// Coarse-grained load balancing of the pull direction (Section 3.2): one
// lane per row serially; rows longer than kHeavyRow are taken by the whole
// wave, which reduces its lanes' partial sums. No atomics.
__device__ __forceinline__ double pull_row(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                           const float* __restrict__ c, int64_t row, int64_t rows) {
  const int lane = threadIdx.x & (kWave - 1);
  int32_t b = 0, e = 0;
  if (row < rows) {
    b = gcd::ld_stream(ptr + row);
    e = gcd::ld_stream(ptr + row + 1);
  }
  const bool heavy = (e - b) > kHeavyRow;
  double sum = heavy ? 0.0 : row_sum(col, c, b, e);
  uint64_t pending = __ballot(heavy);
  while (pending) {
    const int owner = __ffsll(static_cast<long long>(pending)) - 1;
    pending &= pending - 1;
    const int32_t hb = __shfl(b, owner, kWave), he = __shfl(e, owner, kWave);
    double acc = 0.0;
    for (int32_t i = hb + lane; i < he; i += kWave) acc += static_cast<double>(c[gcd::ld_stream(col + i)]);
    acc = gcd::wave_sum(acc);
    if (lane == owner) sum = acc;
  }
  return sum;
}

// Algorithm 4 over every subgraph in one launch (local rows are stored
// block after block, so consecutive work-groups stay inside one block and
// its slice of c stays cache resident): partial[l] = sum of c over the
// local row's columns, written densely by local id.
__global__ __launch_bounds__(kThreads) void k_pr_tocab_pull(const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col,
                                                            const float* __restrict__ c,
                                                            float* __restrict__ partial, int64_t P) {
  const int64_t l = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const double s = pull_row(row_ptr, col, c, l, P);
  if (l < P) gcd::st_stream(partial + l, static_cast<float>(s));
}

// Figure 5 merge fused with the update: work-group j owns vertices
// [j*K, (j+1)*K). For every block s it reads the slice of partial sums whose
// local rows map into that range (contiguous, since local ids ascend with
// global ids), accumulates them in LDS (FP64), then updates its vertices
// with coalesced writes.
template <int K>
__global__ __launch_bounds__(kThreads) void k_pr_merge(const int32_t* __restrict__ range_ptr, int32_t B,
                                                       const int32_t* __restrict__ id_map,
                                                       const float* __restrict__ partial, Update u) {
  __shared__ double acc[K];
  const int32_t v0 = blockIdx.x * K;
  for (int i = threadIdx.x; i < K; i += kThreads) acc[i] = 0.0;
  __syncthreads();
  const int32_t* lo = range_ptr + static_cast<int64_t>(blockIdx.x) * B;
  const int32_t* hi = lo + B;
  for (int32_t s = 0; s < B; ++s) {
    const int32_t a = lo[s], z = hi[s];
    for (int32_t l = a + threadIdx.x; l < z; l += kThreads) {
      const int32_t v = gcd::ld_stream(id_map + l);
      const float p = gcd::ld_stream(partial + l);
      atomicAdd(&acc[v - v0], static_cast<double>(p));
    }
  }
  __syncthreads();
  const double D = *u.dtotal_in;
  double mine = 0.0;
  for (int i = threadIdx.x; i < K; i += kThreads) {
    const int32_t v = v0 + i;
    if (v < u.n) mine += update_vertex(u, v, acc[i], D);
  }
  finish_dangling(u, mine);
}

// Algorithm 1 with the update fused: reads c from one buffer and writes the
// next iteration's c into the other.
__global__ __launch_bounds__(kThreads) void k_pr_plain_pull(const int32_t* __restrict__ t_rowptr,
                                                            const int32_t* __restrict__ t_col,
                                                            const float* __restrict__ c_in, Update u) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  const double s = pull_row(t_rowptr, t_col, c_in, v, u.n);
  const double D = *u.dtotal_in;
  double mine = 0.0;
  if (v < u.n) mine = update_vertex(u, v, s, D);
  finish_dangling(u, mine);
}

// Push with thread+warp+CTA style fine-grained balancing (Section 2.1,
// applied to push in Section 3.2): the work-group's 256 rows are laid end to
// end by an exclusive scan of their lengths and every lane takes one arc at
// a time, locating its row by binary search; each arc is an FP32 atomic add
// into sums[dst]. With id_map (Algorithm 5) rows are a push partition's
// local sources and the destinations of one block stay inside a W-wide
// slice of sums.
__global__ __launch_bounds__(kThreads) void k_pr_push(const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ id_map,
                                                      const int32_t* __restrict__ col,
                                                      const float* __restrict__ c, float* __restrict__ sums,
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
    atomicAdd(&sums[col[e]], val[lo]);
  }
}

// Update after a push pass; clears sums for the next pass.
__global__ __launch_bounds__(kThreads) void k_pr_apply(float* __restrict__ sums, Update u) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  const double D = *u.dtotal_in;
  double mine = 0.0;
  if (v < u.n) {
    const float s = sums[v];
    sums[v] = 0.0f;
    mine = update_vertex(u, v, static_cast<double>(s), D);
  }
  finish_dangling(u, mine);
}

template <int K>
void launch_merge(int32_t R, hipStream_t s, const int32_t* rp, int32_t B, const int32_t* id_map,
                  const float* partial, const Update& u) {
  k_pr_merge<K><<<R, kThreads, 0, s>>>(rp, B, id_map, partial, u);
}

}  // namespace

namespace gcx {

hipError_t pagerank_run(gc_graph g, gc_tocab t, int32_t dir, float damping, int32_t dangling,
                        const float* rank_in, float* rank_out, int32_t iters, hipStream_t s) {
  const int32_t n = g->n;
  if (iters == 0)
    return hipMemcpyAsync(rank_out, rank_in, sizeof(float) * n, hipMemcpyDeviceToDevice, s);
  const bool push = t ? (t->dir == GC_PUSH) : (dir == GC_PUSH);
  Update u;
  u.d = damping;
  u.base = (1.0 - static_cast<double>(damping)) / n;
  u.inv_n = dangling == GC_DANGLING_UNIFORM ? 1.0 / n : 0.0;
  u.dpart = g->dpart;
  u.counter = g->counter;
  u.rowptr = g->rowptr;
  u.n = n;
  u.rank_out = nullptr;
  const int vgrid = (n + kThreads - 1) / kThreads;

  // contributions of rank_in and D of iteration 0 -> dtotal[0]
  u.dtotal_in = nullptr;
  u.dtotal_out = g->dtotal;
  u.contrib = g->contrib[0];
  {
    ProfScope prof("pr_init", s);
    k_pr_init<<<vgrid, kThreads, 0, s>>>(rank_in, u, push ? g->sums : nullptr);
  }
  GC_HIP_TRY(hipGetLastError());

  int cur = 0;
  for (int32_t it = 0; it < iters; ++it) {
    u.dtotal_in = g->dtotal + (it & 1);
    u.dtotal_out = g->dtotal + ((it + 1) & 1);
    u.rank_out = (it == iters - 1) ? rank_out : nullptr;
    if (t && !push) {
      const int64_t P = t->P;
      if (P > 0) {
        ProfScope prof("pr_tocab_pull", s);
        k_pr_tocab_pull<<<static_cast<uint32_t>((P + kThreads - 1) / kThreads), kThreads, 0, s>>>(
            t->row_ptr, t->col, g->contrib[0], t->partial, P);
      }
      u.contrib = g->contrib[0];  // safe in place: the pull pass has finished reading c
      ProfScope prof("pr_merge", s);
      switch (t->k) {
        case 256: launch_merge<256>(t->R, s, t->range_ptr, t->B, t->id_map, t->partial, u); break;
        case 512: launch_merge<512>(t->R, s, t->range_ptr, t->B, t->id_map, t->partial, u); break;
        case 1024: launch_merge<1024>(t->R, s, t->range_ptr, t->B, t->id_map, t->partial, u); break;
        case 2048: launch_merge<2048>(t->R, s, t->range_ptr, t->B, t->id_map, t->partial, u); break;
        case 4096: launch_merge<4096>(t->R, s, t->range_ptr, t->B, t->id_map, t->partial, u); break;
        case 8192: launch_merge<8192>(t->R, s, t->range_ptr, t->B, t->id_map, t->partial, u); break;
        case 16384: launch_merge<16384>(t->R, s, t->range_ptr, t->B, t->id_map, t->partial, u); break;
        default: return hipErrorInvalidValue;
      }
    } else if (!push) {
      u.contrib = g->contrib[cur ^ 1];
      {
        ProfScope prof("pr_plain_pull", s);
        k_pr_plain_pull<<<vgrid, kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, g->contrib[cur], u);
      }
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
    GC_HIP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

}  // namespace gcx
