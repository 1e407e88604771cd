// Traversal on gfx950: BFS and SSSP level by level (Section 3.3).
//
// Frontier state kept by the library, per graph handle:
//   front      status of the current frontier, one bit per vertex (the
//              paper's status array, at n/8 bytes: 2 MB at 2^24 vertices,
//              so the random tests of a pull level stay in one XCD's L2)
//   next       the same for the next level; all zero when a level starts
//              (cleared through the old frontier's queue)
//   queue      list of the current frontier (size n_f), and the list being
//              filled for the next level
//   visited    bitmap of vertices with a final depth (BFS)
// A level runs in one of three ways:
//   pull  topology-driven over the transposed graph: every unvisited vertex
//         scans its in-arcs for an active source (BFS stops at the first);
//   tocab the same over a GC_PULL partition: each block writes a flag (BFS)
//         or a minimum (SSSP) per local row, and a merge over vertex ranges
//         reduces them, updates depth / dist and builds the next frontier;
//   push  data-driven from the queue: every frontier vertex relaxes its
//         out-arcs with atomics (CAS on depth, atomicMin on dist).
// The host reads the frontier size and its out-arc count once per level.

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "gc_device.h"
#include "gc_internal.h"
#include "gc_mlp.h"
#include "gc_merge.h"

namespace {

using gcd::kWave;
using gcx::Buf;
using gcx::ProfScope;

constexpr int kThreads = 256;
constexpr int32_t kInf = INT32_MAX;
constexpr int kHeavy = 32;  // rows longer than this are scanned by the whole wave

// stats slots (device int32[gcx::kStatSlots], copied to the pinned mirror once per level)
constexpr int kQLen = gcx::kStatQLen;
constexpr int kOverflow = gcx::kStatOverflow;
constexpr int kDegLo = gcx::kStatDegLo;

// Appends v to queue for every thread with take set, with one atomic on the
// queue length per work-group (per-wave atomics on the one counter
// serialise in L2 when most waves of a large grid append); positions follow
// the thread order inside the work-group. Synchronises the work-group: every
// thread must reach each call.
template <int NT = kThreads>
__device__ __forceinline__ void block_append(bool take, int32_t v, int32_t* __restrict__ queue,
                                             int32_t* __restrict__ qlen) {
  __shared__ int32_t wave_cnt[NT / kWave];
  __shared__ int32_t wave_off[NT / kWave];
  const uint64_t mask = __ballot(take);
  const int wid = threadIdx.x / kWave;
  if (gcd::lane_id() == 0) wave_cnt[wid] = __popcll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t tot = 0;
    for (int w = 0; w < NT / kWave; ++w) {
      wave_off[w] = tot;
      tot += wave_cnt[w];
    }
    const int32_t base = tot ? atomicAdd(qlen, tot) : 0;
    for (int w = 0; w < NT / kWave; ++w) wave_off[w] += base;
  }
  __syncthreads();
  if (take) queue[wave_off[wid] + __popcll(mask & gcd::lanemask_lt())] = v;
}

// Appends to the queue, with one atomic for the work-group, the vertices
// vbase + u * stride of every thread for the set bits u of took (at most
// 32 per thread). Every thread of the work-group calls it (it synchronises).
template <int NT>
__device__ __forceinline__ void block_append_bits(uint32_t took, int32_t vbase, int32_t stride,
                                                  int32_t* __restrict__ queue, int32_t* __restrict__ qlen) {
  __shared__ int32_t wave_cnt[NT / kWave];
  __shared__ int32_t wave_off[NT / kWave];
  const int lane = gcd::lane_id();
  const int wid = threadIdx.x / kWave;
  const int32_t c = __popc(took);
  int32_t x = c;  // inclusive sum of the counts over the wave's lanes
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wave_cnt[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t tot = 0;
    for (int w = 0; w < NT / kWave; ++w) {
      wave_off[w] = tot;
      tot += wave_cnt[w];
    }
    const int32_t base = tot ? atomicAdd(qlen, tot) : 0;
    for (int w = 0; w < NT / kWave; ++w) wave_off[w] += base;
  }
  __syncthreads();
  int32_t pos = wave_off[wid] + x - c;
  while (took) {
    const int u = __ffs(took) - 1;
    took &= took - 1u;
    queue[pos++] = vbase + u * stride;
  }
}

// Appends to the queue, with one atomic for the work-group, vals[u] of
// every thread for the set bits u of took. Every thread of the work-group
// calls it (it synchronises).
template <int NT, int kN>
__device__ __forceinline__ void block_append_list(uint32_t took, const int32_t (&vals)[kN],
                                                  int32_t* __restrict__ queue, int32_t* __restrict__ qlen) {
  __shared__ int32_t wave_cnt[NT / kWave];
  __shared__ int32_t wave_off[NT / kWave];
  const int lane = gcd::lane_id();
  const int wid = threadIdx.x / kWave;
  const int32_t c = __popc(took);
  int32_t x = c;  // inclusive sum of the counts over the wave's lanes
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wave_cnt[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t tot = 0;
    for (int w = 0; w < NT / kWave; ++w) {
      wave_off[w] = tot;
      tot += wave_cnt[w];
    }
    const int32_t base = tot ? atomicAdd(qlen, tot) : 0;
    for (int w = 0; w < NT / kWave; ++w) wave_off[w] += base;
  }
  __syncthreads();
  int32_t pos = wave_off[wid] + x - c;
#pragma unroll
  for (int u = 0; u < kN; ++u)
    if ((took >> u) & 1u) queue[pos++] = vals[u];
}

__device__ __forceinline__ bool bit_test(const uint32_t* bits, int32_t v) {
  return (bits[v >> 5] >> (v & 31)) & 1u;
}

__device__ __forceinline__ void bit_set(uint32_t* bits, int32_t v) { atomicOr(&bits[v >> 5], 1u << (v & 31)); }

// Sets bit v in `bits` for the lanes where `take` holds, one atomic per
// 32-bit word: every lane of the wave calls it, and lane l holds vertex
// v0 + l for a v0 that is a multiple of 32 (a wave of consecutive
// vertices). Per-vertex atomics on the few words a wave shares serialise in
// L2 on levels that discover millions of vertices.
__device__ __forceinline__ void wave_bits_set(uint32_t* bits, int32_t v, bool take) {
  const uint64_t m = __ballot(take);
  const int lane = gcd::lane_id();
  const uint32_t word = static_cast<uint32_t>(m >> (lane & 32));
  if ((lane & 31) == 0 && word != 0u) atomicOr(&bits[v >> 5], word);
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t x) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = x;
}

__global__ void k_set_source(int32_t src, int32_t* __restrict__ value, uint32_t* __restrict__ front,
                             int32_t* __restrict__ queue, uint32_t* __restrict__ visited) {
  value[src] = 0;
  front[src >> 5] |= 1u << (src & 31);
  queue[0] = src;
  if (visited) visited[src >> 5] |= 1u << (src & 31);
}

// Clears the old frontier's bitmap through its queue: every set bit belongs
// to a queued vertex, so zeroing the words the queue touches clears it all.
__global__ void k_clear_front(uint32_t* __restrict__ front, const int32_t* __restrict__ queue, int32_t qn) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < qn) front[queue[i] >> 5] = 0u;
}

// Start of a level: clears the counters the level accumulates and stamps
// the device wall clock.
__global__ void k_level_begin(int32_t* __restrict__ stats) {
  if (threadIdx.x < gcx::kStatT0) stats[threadIdx.x] = 0;
  if (threadIdx.x < 2) stats[gcx::kStatInDegLo + threadIdx.x] = 0;
  if (threadIdx.x == 0) *reinterpret_cast<uint64_t*>(stats + gcx::kStatT0) = wall_clock64();
}

// What the learned scheduler needs to decide the next level on the device:
// its parameters and the graph's and level's counts.
struct LevelDecide {
  const float* params = nullptr;
  const float* frange = nullptr;
  int32_t K = 0;
  int64_t n = 0, m = 0;
  int32_t level = 0;
  int64_t prior_arcs = 0;
  int32_t clock_khz = 1;
  // the working-set rule's direction test for the next level (the network
  // only picks the form of pull levels, so push levels skip it): its state,
  // and the unexplored arcs before the next frontier's are taken off (BFS)
  // or the whole arc count (SSSP)
  bool pulling = false;
  bool sub_next = false;
  int64_t unexplored = 0;
  double alpha = 0.0, beta = 0.0;
};

// Out-arc count of the queued vertices (for the direction heuristic). The
// kernel runs right after the level's relaxation kernels on the same
// stream, so its start stamps the end of the level.
__global__ void k_queue_degree(const int32_t* __restrict__ queue, const int32_t* __restrict__ qlen,
                               const int32_t* __restrict__ rowptr, const int32_t* __restrict__ t_rowptr,
                               int32_t* __restrict__ stats) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *reinterpret_cast<uint64_t*>(stats + gcx::kStatT1) = wall_clock64();
  const int32_t qn = *qlen;
  uint64_t sum = 0, sum_in = 0;  // out-arcs and in-arcs of the queued vertices
  // four queue entries per step, their loads issued together (one
  // dependent pair of round trips per step, not per entry)
  const int32_t stride = static_cast<int32_t>(gridDim.x * blockDim.x);
  int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  for (; static_cast<int64_t>(i) + 3 * static_cast<int64_t>(stride) < qn; i += 4 * stride) {
    int32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = queue[i + k * stride];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sum += static_cast<uint64_t>(rowptr[v[k] + 1] - rowptr[v[k]]);
      if (t_rowptr) sum_in += static_cast<uint64_t>(t_rowptr[v[k] + 1] - t_rowptr[v[k]]);
    }
  }
  for (; i < qn; i += stride) {
    const int32_t v = queue[i];
    sum += static_cast<uint64_t>(rowptr[v + 1] - rowptr[v]);
    if (t_rowptr) sum_in += static_cast<uint64_t>(t_rowptr[v + 1] - t_rowptr[v]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_xor(sum, o, kWave);
    sum_in += __shfl_xor(sum_in, o, kWave);
  }
  // one atomic per work-group (per-wave atomics on the one counter serialise)
  __shared__ uint64_t part[kThreads / kWave], part_in[kThreads / kWave];
  if (gcd::lane_id() == 0) {
    part[threadIdx.x / kWave] = sum;
    part_in[threadIdx.x / kWave] = sum_in;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t total = 0, total_in = 0;
    for (int w = 0; w < kThreads / kWave; ++w) {
      total += part[w];
      total_in += part_in[w];
    }
    if (total) atomicAdd(reinterpret_cast<unsigned long long*>(stats + kDegLo), total);
    if (total_in) atomicAdd(reinterpret_cast<unsigned long long*>(stats + gcx::kStatInDegLo), total_in);
  }
}

// LDS the learned decision needs: the parameters, and W2 again at a pitch
// of one word more than its rows.
size_t level_decide_lds(int32_t K) {
  return sizeof(float) * (static_cast<size_t>(gcmlp::Layout(K).total) + gcmlp::kHid * (gcmlp::kHid + 1));
}

// The learned scheduler's decision for the next level, from the counters of
// the level just ended (read after k_queue_degree): the next frontier's
// size and out-arcs and the level's time from its clock stamps. The
// network only picks the form of pull levels, so the kernel first applies
// the working-set rule's direction test and stops on a push level. Else the
// work-group stages the parameters in LDS (coalesced, all loads in flight
// together; W2 at a pitch of kHid + 1, since each lane reads its own row)
// and its first wave runs the network. Dynamic LDS: level_decide_lds(K).
__global__ __launch_bounds__(kThreads) void k_level_decide(int32_t* __restrict__ stats, LevelDecide dec) {
  extern __shared__ float sp[];
  const int64_t n_f = stats[gcx::kStatQLen];
  const int64_t m_f = static_cast<int64_t>(static_cast<uint32_t>(stats[kDegLo])) |
                      (static_cast<int64_t>(stats[kDegLo + 1]) << 32);
  const double mu = static_cast<double>(dec.sub_next ? dec.unexplored - m_f : dec.unexplored);
  const bool pull_next = dec.pulling ? !(static_cast<double>(n_f) < static_cast<double>(dec.n) / dec.beta)
                                     : static_cast<double>(m_f) > mu / dec.alpha;
  if (!pull_next) {  // uniform
    if (threadIdx.x == 0) stats[gcx::kStatChoice] = -1;  // push: the rule alone
    return;
  }
  const gcmlp::Layout L(dec.K);
  float* w2 = sp + L.total;  // row r at r * (kHid + 1)
  for (int32_t i = threadIdx.x; i < L.total; i += kThreads) {
    const float x = dec.params[i];
    const int32_t r = i - L.W2;
    if (r >= 0 && r < gcmlp::kHid * gcmlp::kHid) w2[r + r / gcmlp::kHid] = x;
    else sp[i] = x;
  }
  __syncthreads();
  if (threadIdx.x >= kWave) return;
  const uint64_t t0 = *reinterpret_cast<const uint64_t*>(stats + gcx::kStatT0);
  const uint64_t t1 = *reinterpret_cast<const uint64_t*>(stats + gcx::kStatT1);
  const double prior_ms = t1 > t0 ? static_cast<double>(t1 - t0) / dec.clock_khz : 0.0;
  float in[GC_SCHED_INPUTS];
  gcx::level_features(dec.n, dec.m, n_f, m_f, dec.level, prior_ms, dec.prior_arcs, in);
  gcmlp::mlp_decide<gcmlp::kHid + 1>(sp, w2, dec.K, in, dec.frange, stats + gcx::kStatChoice,
                                     reinterpret_cast<float*>(stats + gcx::kStatOut));
}

// Largest out-degree of the graph into *out (zero on entry): one atomic
// per work-group.
__global__ __launch_bounds__(kThreads) void k_max_out_degree(const int32_t* __restrict__ rowptr, int32_t n,
                                                             int32_t* __restrict__ out) {
  int32_t mx = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; v < n; v += stride)
    mx = max(mx, rowptr[v + 1] - rowptr[v]);
  for (int o = kWave / 2; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, kWave));
  __shared__ int32_t part[kThreads / kWave];
  if (gcd::lane_id() == 0) part[threadIdx.x / kWave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t top = 0;
    for (int w = 0; w < kThreads / kWave; ++w) top = max(top, part[w]);
    if (top) atomicMax(out, top);
  }
}

// ---------------------------------------------------------------------------
// BFS

// Scans in-arcs [b, e) for an active source; rows longer than kHeavy are
// taken by the whole wave, which stops as soon as any lane hits.
__device__ __forceinline__ bool scan_front(const int32_t* __restrict__ col, const uint32_t* __restrict__ front,
                                           bool active, int32_t b, int32_t e) {
  const int lane = gcd::lane_id();
  const bool heavy = active && (e - b) > kHeavy;
  bool found = false;
  if (active && !heavy) {
    int32_t i = b;
    for (; i + 4 <= e; i += 4) {  // four arcs' loads in flight at a time
      int32_t u[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) u[k] = col[i + k];
      uint32_t any = 0;  // all four tests, no short circuit
#pragma unroll
      for (int k = 0; k < 4; ++k) any |= (front[u[k] >> 5] >> (u[k] & 31)) & 1u;
      if (any) {
        found = true;
        break;
      }
    }
    for (; !found && i < e; ++i) found = bit_test(front, col[i]);
  }
  uint64_t pending = __ballot(heavy);
  while (pending) {
    const int owner = __ffsll(static_cast<long long>(pending)) - 1;
    pending &= pending - 1;
    const int32_t hb = __shfl(b, owner, kWave), he = __shfl(e, owner, kWave);
    bool hit = false;
    for (int32_t base = hb; base < he; base += kWave) {
      const int32_t i = base + lane;
      const bool h = i < he && bit_test(front, col[i]);
      if (__any(h)) {
        hit = true;
        break;
      }
    }
    if (lane == owner) found = hit;
  }
  return found;
}

// Topology-driven pull over the whole transposed graph.
__global__ __launch_bounds__(kThreads) void k_bfs_pull(const int32_t* __restrict__ t_rowptr,
                                                       const int32_t* __restrict__ t_col, int32_t n,
                                                       const uint32_t* __restrict__ front, int32_t* __restrict__ depth,
                                                       int32_t level, uint32_t* __restrict__ next,
                                                       uint32_t* __restrict__ visited, int32_t* __restrict__ queue,
                                                       int32_t* __restrict__ stats) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  // the visited word and the row bounds are loaded together (one memory
  // round trip before the scan, not two)
  uint32_t vw = ~0u;
  int32_t b = 0, e = 0;
  if (v < n) {
    vw = visited[v >> 5];
    b = t_rowptr[v];
    e = t_rowptr[v + 1];
  }
  const bool active = !((vw >> (v & 31)) & 1u);
  const bool found = scan_front(t_col, front, active, b, e);
  if (found) depth[v] = level + 1;
  wave_bits_set(next, v, found);
  wave_bits_set(visited, v, found);
  block_append(found, v, queue, stats + kQLen);
}

// TOCAB pull, per block: flag[l] = 1 when local row l (an unvisited vertex)
// has an in-arc from an active source of this block; a local next array.
__global__ __launch_bounds__(kThreads) void k_bfs_tocab(const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col,
                                                        const int32_t* __restrict__ id_map, int64_t P,
                                                        const uint32_t* __restrict__ visited,
                                                        const uint32_t* __restrict__ front,
                                                        uint8_t* __restrict__ flag) {
  // the stride is uniform over the work-group, so every wave of it runs the
  // same passes and the wave-wide scans inside stay convergent
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kThreads; base < P;
       base += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int64_t l = base + threadIdx.x;
    bool active = false;
    int32_t b = 0, e = 0;
    if (l < P && !bit_test(visited, id_map[l])) {
      active = true;
      b = row_ptr[l];
      e = row_ptr[l + 1];
    }
    const bool found = scan_front(col, front, active, b, e);
    if (l < P) flag[l] = found ? 1 : 0;
  }
}

// Merge of the per-block flags over vertex range j (OR), fused with the
// depth update and the next frontier (Section 3.3: the reduction of next is
// done in the same kernel as that of the partial results).
template <int K, bool kFlat>
__global__ __launch_bounds__(kThreads) void k_bfs_merge(const int32_t* __restrict__ range_ptr, int32_t B,
                                                        const uint16_t* __restrict__ id16,
                                                        const uint8_t* __restrict__ flag, int32_t n,
                                                        int32_t* __restrict__ depth, int32_t level,
                                                        uint32_t* __restrict__ next, uint32_t* __restrict__ visited,
                                                        int32_t* __restrict__ queue, int32_t* __restrict__ stats) {
  __shared__ uint8_t hit[K];
  const int32_t v0 = blockIdx.x * K;
  for (int i = threadIdx.x; i < K; i += kThreads) hit[i] = 0;
  gcm::merge_slices<kFlat, kThreads>(range_ptr, B, id16, flag, blockIdx.x, [&](uint32_t v, uint8_t f) {
    if (f) hit[v] = 1;
  });
  for (int i = threadIdx.x; i < K; i += kThreads) {
    const int32_t v = v0 + i;
    const bool found = v < n && hit[i] && !bit_test(visited, v);
    if (found) depth[v] = level + 1;
    wave_bits_set(next, v, found);
    wave_bits_set(visited, v, found);
    block_append(found, v, queue, stats + kQLen);
  }
}

// Data-driven push (Algorithm 3's CAS pattern): the work-group's 256 queued
// vertices are laid end to end by a scan of their out-degrees and each lane
// takes one arc at a time; the CAS on depth admits every vertex once.
__global__ __launch_bounds__(kThreads) void k_bfs_push(const int32_t* __restrict__ queue_in, int32_t qn,
                                                       const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ colidx,
                                                       int32_t* __restrict__ depth, int32_t level,
                                                       uint32_t* __restrict__ next, uint32_t* __restrict__ visited,
                                                       int32_t* __restrict__ queue, int32_t* __restrict__ stats) {
  __shared__ int32_t start[kThreads];
  __shared__ int32_t first[kThreads];
  __shared__ int32_t wave_tot[kThreads / kWave];
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  int32_t b = 0, len = 0;
  if (i < qn) {
    const int32_t u = queue_in[i];
    b = rowptr[u];
    len = rowptr[u + 1] - b;
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
  __syncthreads();
  // every thread runs the same number of rounds (block_append synchronises the work-group)
  const int32_t rounds = (total + kThreads - 1) / kThreads;
  for (int32_t r = 0; r < rounds; ++r) {
    const int32_t a = r * kThreads + threadIdx.x;
    bool disc = false;
    int32_t v = 0;
    if (a < total) {
      int lo = 0, hi = kThreads - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= a) lo = mid;
        else hi = mid - 1;
      }
      v = colidx[first[lo] + (a - start[lo])];
      if (depth[v] == kInf && atomicCAS(&depth[v], kInf, level + 1) == kInf) {
        disc = true;
        bit_set(next, v);
        bit_set(visited, v);
      }
    }
    block_append(disc, v, queue, stats + kQLen);
  }
}

// ---------------------------------------------------------------------------
// SSSP (synchronous Bellman-Ford rounds over the vertices changed last round)

// Minimum of dist[u] + w over in-arcs [b, e) from active sources u (kInf if
// none); rows longer than kHeavy are reduced by the whole wave. *ovf is set
// when a candidate path length reaches INT32_MAX.
__device__ __forceinline__ int64_t scan_min(const int32_t* __restrict__ col, const int32_t* __restrict__ w,
                                            const uint32_t* __restrict__ front, const int32_t* __restrict__ dist,
                                            bool active, int32_t b, int32_t e, bool* ovf) {
  const int lane = gcd::lane_id();
  const bool heavy = active && (e - b) > kHeavy;
  int64_t best = kInf;
  bool over = false;
  if (active && !heavy) {
    int32_t i = b;
    for (; i + 4 <= e; i += 4) {  // four arcs' loads in flight at a time
      int32_t u[4], wk[4];
      bool on[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        u[k] = col[i + k];
        wk[k] = w[i + k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) on[k] = bit_test(front, u[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t cand = on[k] ? static_cast<int64_t>(dist[u[k]]) + wk[k] : static_cast<int64_t>(kInf);
        over |= on[k] && cand >= kInf;
        best = min(best, cand);
      }
    }
    for (; i < e; ++i) {
      const int32_t u = col[i];
      if (bit_test(front, u)) {
        const int64_t cand = static_cast<int64_t>(dist[u]) + w[i];
        over |= cand >= kInf;
        best = min(best, cand);
      }
    }
  }
  uint64_t pending = __ballot(heavy);
  while (pending) {
    const int owner = __ffsll(static_cast<long long>(pending)) - 1;
    pending &= pending - 1;
    const int32_t hb = __shfl(b, owner, kWave), he = __shfl(e, owner, kWave);
    int64_t m = kInf;
    for (int32_t i = hb + lane; i < he; i += kWave) {
      const int32_t u = col[i];
      if (bit_test(front, u)) {
        const int64_t cand = static_cast<int64_t>(dist[u]) + w[i];
        over |= cand >= kInf;
        m = min(m, cand);
      }
    }
    for (int o = 32; o > 0; o >>= 1) m = min(m, static_cast<int64_t>(__shfl_xor(m, o, kWave)));
    if (lane == owner) best = m;
  }
  *ovf = over;
  return min<int64_t>(best, kInf);
}

__global__ __launch_bounds__(kThreads) void k_sssp_pull(const int32_t* __restrict__ t_rowptr,
                                                        const int32_t* __restrict__ t_col,
                                                        const int32_t* __restrict__ t_w, int32_t n,
                                                        const uint32_t* __restrict__ front, int32_t* __restrict__ dist,
                                                        uint32_t* __restrict__ next, int32_t* __restrict__ queue,
                                                        int32_t* __restrict__ stats) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  int32_t b = 0, e = 0;
  if (v < n) {
    b = t_rowptr[v];
    e = t_rowptr[v + 1];
  }
  bool ovf;
  const int64_t best = scan_min(t_col, t_w, front, dist, v < n, b, e, &ovf);
  if (ovf) stats[kOverflow] = 1;
  bool improved = false;
  if (v < n && best < dist[v]) {
    dist[v] = static_cast<int32_t>(best);
    improved = true;
  }
  wave_bits_set(next, v, improved);
  block_append(improved, v, queue, stats + kQLen);
}

// TOCAB pull, per block: pmin[l] = min over active sources of this block of
// dist[u] + w (INT32_MAX if none; saturated on overflow, which is flagged).
__global__ __launch_bounds__(kThreads) void k_sssp_tocab(const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col,
                                                         const int32_t* __restrict__ w, int64_t P,
                                                         const uint32_t* __restrict__ front,
                                                         const int32_t* __restrict__ dist, int32_t* __restrict__ pmin,
                                                         int32_t* __restrict__ stats) {
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kThreads; base < P;
       base += static_cast<int64_t>(gridDim.x) * kThreads) {  // uniform per work-group
    const int64_t l = base + threadIdx.x;
    int32_t b = 0, e = 0;
    if (l < P) {
      b = row_ptr[l];
      e = row_ptr[l + 1];
    }
    bool ovf;
    const int64_t best = scan_min(col, w, front, dist, l < P, b, e, &ovf);
    if (ovf) stats[kOverflow] = 1;
    if (l < P) pmin[l] = static_cast<int32_t>(best);
  }
}

// TOCAB pull for SSSP over the stream layout (blocks up to 2^15 wide, the
// layout the PageRank pull reads): the block's slice of the frontier's
// distances lives in LDS, so the random reads of a round never leave the
// CU. One work-group per chunk of the partition (rows [r0, r1) of block b);
// it first stores ad[i] = dist[bW + i] for sources in the frontier and
// INT32_MAX for the others, then each wave walks a contiguous range of
// 512-arc tiles: a lane holds 8 consecutive arcs (16-bit columns, their
// weights, the head bits of its head word), takes their candidates ad[col]
// + w, and a segmented minimum (lane-local runs, then a wave-wide
// segmented scan) gives the minimum of every row whose head lies in the
// wave's range; the row open at a tile's end carries into the next tile,
// and the one open at the range's end is finished by reading on. pmin[l]
// (block-major, as the wide-block kernel writes it) is the minimum over
// local row l's arcs, INT32_MAX when no source of the row is active.
constexpr int kLdsRowThreads = 1024;
// Buffer offset of a dropped store: past any partition's minima (whose
// stream layout keeps 4 (P + 8) below 2^31 bytes).
constexpr uint32_t kDropOff = 0x80000000u;
constexpr int kSeekPad = 4;  // position-table entries past the chunk's ns ranges: sb[ns] (past the chunk), sentinels
constexpr int kLdsRowWaves = kLdsRowThreads / kWave;
constexpr int kRowTile = 512;  // arcs per wave tile: 8 per lane

typedef uint32_t tu32x4 __attribute__((ext_vector_type(4)));
typedef int32_t ti32x4 __attribute__((ext_vector_type(4)));

// Value a DPP control moves into each lane; INT32_MAX (the identity of the
// minimum) where the move has no source lane or the lane's row is masked off.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int32_t dpp_in(int32_t a) {
  return __builtin_amdgcn_update_dpp(kInf, a, kCtrl, kRowMask, 0xF, false);
}

// Lanes of the wave selected by a mask held in scalar registers.
__device__ __forceinline__ bool lane_in_mask(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// One step of a wave-wide segmented inclusive minimum: a lane outside F
// (no head met yet within the reach of the steps so far) takes the minimum
// with the value the DPP control moves in. The move is made by every lane
// before the select: under a narrower EXEC mask it could not read the
// values of the lanes in F.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void seg_min_step(int32_t& A, uint64_t F) {
  const int32_t m = min(A, dpp_in<kCtrl, kRowMask>(A));
  A = lane_in_mask(F) ? A : m;
}

struct MinTile {
  int32_t x[8];     // candidates of the lane's 8 arcs
  uint32_t my9;     // head bits of the lane's arcs, bit 8: the arc after them
  int32_t row0;     // local row holding the lane's arc 0 when it is no head (row before the first head)
};

// Weights of a stream-layout partition in its arc order (kW): int32
// (kW32), one byte each when every weight lies in [0, 255] (kW8), or none:
// BFS, whose candidates are the sources' own values (0 when in the frontier).
constexpr int kW32 = 0, kW8 = 1, kWNone = 2;
// A tile's raw streams for one lane: its 8 columns, its head word and its
// 8 weights (as loaded), so that the loads of later tiles can be issued
// before an earlier tile is reduced.
struct RawTile {
  tu32x4 cols;
  tu32x4 hw;
  ti32x4 wa, wb;  // int32 weights (kW32)
  uint64_t w8;    // byte weights (kW8)
};

template <int kW>
__device__ __forceinline__ RawTile load_raw_tile(const uint16_t* __restrict__ col16,
                                                 const gc_head_word* __restrict__ heads,
                                                 const void* __restrict__ w_arcs, int64_t q, int lane) {
  RawTile r;
  const int64_t tb = q * kRowTile;
  r.cols = gcd::ld_stream(reinterpret_cast<const tu32x4*>(col16 + tb) + lane);
  r.w8 = 0;
  r.wa = ti32x4{0, 0, 0, 0};
  r.wb = ti32x4{0, 0, 0, 0};
  if (kW == kW8) {
    r.w8 = gcd::ld_stream(reinterpret_cast<const uint64_t*>(static_cast<const uint8_t*>(w_arcs) + tb) + lane);
  } else if (kW == kW32) {
    const int32_t* w_pad = static_cast<const int32_t*>(w_arcs);
    r.wa = gcd::ld_stream(reinterpret_cast<const ti32x4*>(w_pad + tb) + 2 * lane);
    r.wb = gcd::ld_stream(reinterpret_cast<const ti32x4*>(w_pad + tb) + 2 * lane + 1);
  }
  r.hw = *reinterpret_cast<const tu32x4*>(heads + (tb >> 6) + (lane >> 3));
  return r;
}

// The lane's candidates ad[col] + w and its row structure from a raw tile.
template <int kW>
__device__ __forceinline__ MinTile finish_min_tile(const RawTile& r, const int32_t* ad, int lane, bool* ovf) {
  MinTile t;
  const uint64_t bits = static_cast<uint64_t>(r.hw[0]) | (static_cast<uint64_t>(r.hw[1]) << 32);
  const int sub = lane & 7;
  const uint32_t after = sub < 7 ? static_cast<uint32_t>(bits >> (8 * sub + 8)) & 1u : r.hw[3] & 1u;
  t.my9 = (static_cast<uint32_t>(bits >> (8 * sub)) & 0xFFu) | (after << 8);
  const uint64_t below = sub ? (bits & ((1ull << (8 * sub)) - 1ull)) : 0ull;
  t.row0 = static_cast<int32_t>(r.hw[2]) + __popcll(below) - 1;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t c = (r.cols[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
    const int32_t a = ad[c];
    if (kW == kWNone) {  // BFS: the source's own value
      t.x[e] = a;
      continue;
    }
    uint32_t w = 0;
    if (kW == kW8) w = static_cast<uint32_t>(r.w8 >> (8 * e)) & 0xFFu;
    else w = static_cast<uint32_t>(e < 4 ? r.wa[e] : r.wb[e - 4]);
    // a <= INT32_MAX and 0 <= w <= INT32_MAX, so the sum fits in 32 unsigned bits
    const uint32_t cand = static_cast<uint32_t>(a) + w;
    const bool sat = cand >= static_cast<uint32_t>(kInf);
    *ovf |= a != kInf && sat;
    t.x[e] = (a == kInf || sat) ? kInf : static_cast<int32_t>(cand);
  }
  return t;
}

template <int kW>
__device__ __forceinline__ MinTile load_min_tile(const uint16_t* __restrict__ col16,
                                                 const gc_head_word* __restrict__ heads,
                                                 const void* __restrict__ w_arcs, const int32_t* ad, int64_t q,
                                                 int lane, bool* ovf) {
  return finish_min_tile<kW>(load_raw_tile<kW>(col16, heads, w_arcs, q, lane), ad, lane, ovf);
}

template <int kW>
__global__ __launch_bounds__(kLdsRowThreads) void k_sssp_tocab_lds(
    const int32_t* __restrict__ row_ptr, const uint16_t* __restrict__ col16, const gc_head_word* __restrict__ heads,
    const void* __restrict__ w_arcs, const int32_t* __restrict__ chunk_beg, const int32_t* __restrict__ chunk_end,
    const int32_t* __restrict__ chunk_blk, const int32_t* __restrict__ chunk_j0, const int32_t* __restrict__ chunk_ns,
    const int2* __restrict__ seg, int32_t R, int32_t log2W, int32_t n, const uint32_t* __restrict__ front,
    const int32_t* __restrict__ dist, int32_t* __restrict__ pmin, uint32_t pmin_bytes, int32_t* __restrict__ stats) {
  extern __shared__ int32_t ad[];
  const __amdgpu_buffer_rsrc_t out = __builtin_amdgcn_make_buffer_rsrc(pmin, 0, static_cast<int>(pmin_bytes), 0x00020000);
  const int32_t ch = blockIdx.x;
  const int32_t r0 = chunk_beg[ch], r1 = chunk_end[ch], b = chunk_blk[ch], j0 = chunk_j0[ch], ns = chunk_ns[ch];
  if (r0 >= r1) return;  // padding of the dispatch order (uniform)
  // Each wave streams a contiguous range [qa, qz] of the chunk's tiles. Its
  // bounds, its first owned row and its first two tiles depend on the
  // chunk alone, so their loads are issued before the block's LDS fill and
  // overlap it.
  const int lane = gcd::lane_id();
  const int wid = static_cast<int>(threadIdx.x) / kWave;
  const int32_t q0 = row_ptr[r0] / kRowTile, q1 = (row_ptr[r1] - 1) / kRowTile;
  const int32_t nt = q1 - q0 + 1;
  const int32_t qa = q0 + static_cast<int32_t>(static_cast<int64_t>(nt) * wid / kLdsRowWaves);
  const int32_t qz = q0 + static_cast<int32_t>(static_cast<int64_t>(nt) * (wid + 1) / kLdsRowWaves) - 1;
  // rows this wave writes: heads at or after its first arc, inside the chunk
  int32_t own0 = r0;
  // the raw streams of the next two tiles are in flight while a tile is
  // reduced (loads clamped to the wave's last tile, so every path issues them)
  RawTile n1{}, n2{};
  if (qa <= qz) {  // uniform over the wave
    own0 = max(heads[static_cast<int64_t>(qa) * (kRowTile / 64)].row, r0);
    n1 = load_raw_tile<kW>(col16, heads, w_arcs, qa, lane);
    n2 = load_raw_tile<kW>(col16, heads, w_arcs, min(qa + 1, qz), lane);
  }
  const int32_t W = 1 << log2W, v0 = b << log2W, cnt = min(W, n - v0);  // cnt >= 1
  // The block's frontier values in LDS, in batches of kFill vertices per
  // thread whose loads are all issued before the first is used: the status
  // words first, then the distances, a load whose vertex lies outside the
  // frontier's words (or past n) reading the block's first vertex instead,
  // so that a sparse frontier costs no slice of distances.
  constexpr int kFill = 16;
  for (int32_t k0 = 0; k0 < W; k0 += kFill * kLdsRowThreads) {
    uint32_t wd[kFill];
    int32_t dv[kFill];
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const int32_t i = min(k0 + u * kLdsRowThreads + static_cast<int32_t>(threadIdx.x), cnt - 1);
      wd[u] = front[(v0 + i) >> 5];
    }
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const int32_t i = k0 + u * kLdsRowThreads + static_cast<int32_t>(threadIdx.x);
      dv[u] = 0;
      if (kW != kWNone) dv[u] = dist[v0 + ((wd[u] != 0u && i < cnt) ? i : 0)];
    }
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const int32_t i = k0 + u * kLdsRowThreads + static_cast<int32_t>(threadIdx.x);
      const bool on = i < cnt && ((wd[u] >> ((v0 + i) & 31)) & 1u);
      if (i < W) ad[i] = on ? dv[u] : kInf;
    }
  }
  // the chunk's part of the position table: sb[i] = first row of merge range
  // j0 + i, sd[i] = its shift to the range-major index; sb[ns] lies past the
  // chunk, then sentinels
  int32_t* sb = ad + W;
  int32_t* sd = sb + ns + kSeekPad;
  {
    const int2* sg = seg + static_cast<int64_t>(b) * (R + 1) + j0;
    for (int32_t i = threadIdx.x; i < ns + kSeekPad; i += kLdsRowThreads) {
      const int2 e = i <= ns ? sg[i] : make_int2(INT32_MAX, 0);
      sb[i] = e.x;
      sd[i] = e.y;
    }
  }
  __syncthreads();
  if (qa > qz) return;  // no barrier follows
  bool ovf = false;
  int32_t carry = kInf;  // minimum so far of the row open at the previous tile's end
  int32_t open_row = -1;
  int32_t jw = 0;  // merge range of the wave's rows so far (ranges ascend with rows)
  // window of the position table's row boundaries: lane l holds sb[jwin + l]
  // (past the table: its last sentinel)
  int32_t jwin = 0;
  int32_t sbw = sb[min(lane, ns + kSeekPad - 1)];
  for (int32_t q = qa; q <= qz; ++q) {
    const RawTile cur = n1;
    n1 = n2;
    n2 = load_raw_tile<kW>(col16, heads, w_arcs, min(q + 2, qz), lane);
    const MinTile t = finish_min_tile<kW>(cur, ad, lane, &ovf);
    // lane-local runs: reset at every head; lane 0 starts from the carry
    int32_t run = (lane == 0) ? carry : kInf;
    int32_t rv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      run = ((t.my9 >> e) & 1u) ? t.x[e] : min(run, t.x[e]);
      rv[e] = run;
    }
    // Wave-wide segmented inclusive minimum of the lanes' open runs, with DPP
    // lane moves: a lane that has met a head within the reach of the steps
    // so far (a lane mask in scalar registers, widened after each step the
    // way the moves carry data) keeps its value, the others take the minimum
    // with the value moved in (INT32_MAX where a move has no source).
    const uint64_t H = __ballot((t.my9 & 0xFFu) != 0u);
    int32_t A = run;
    uint64_t F = H;
    seg_min_step<0x111, 0xF>(A, F);  // row_shr:1
    F |= (F << 1) & 0xFFFEFFFEFFFEFFFEull;
    seg_min_step<0x112, 0xF>(A, F);  // row_shr:2
    F |= (F << 2) & 0xFFFCFFFCFFFCFFFCull;
    seg_min_step<0x114, 0xF>(A, F);  // row_shr:4
    F |= (F << 4) & 0xFFF0FFF0FFF0FFF0ull;
    seg_min_step<0x118, 0xF>(A, F);  // row_shr:8
    F |= (F << 8) & 0xFF00FF00FF00FF00ull;
    seg_min_step<0x142, 0xA>(A, F);  // row_bcast:15 into rows 1 and 3
    F |= ((F & (1ull << 15)) ? 0x00000000FFFF0000ull : 0ull) | ((F & (1ull << 47)) ? 0xFFFF000000000000ull : 0ull);
    seg_min_step<0x143, 0xC>(A, F);  // row_bcast:31 into rows 2 and 3
    const int32_t lin = dpp_in<0x138, 0xF>(A);  // wave_shr:1, the row flowing into this lane (lane 0: none)
    // Merge range of the rows this lane may store (those of its arcs 0 .. 7,
    // rows rlo .. rhi). The range boundaries inside the tile's rows are
    // counted from the register window (a ballot gives how many lie at or
    // below the tile's last row) and walked through scalar registers, each
    // lane counting those at or below its first and last row; the window
    // moves on when the tile's rows run past its last entry. A lane's rows
    // cross at most one boundary when the block's ranges hold 8 rows or
    // more (tens to hundreds here): the row's shift is then one of the two
    // read below, and only a lane crossing several looks each row's range up.
    const int32_t rlo = t.row0 + static_cast<int32_t>(t.my9 & 1u);
    const int32_t rhi = t.row0 + __popc(t.my9 & 0xFFu);
    const int32_t maxrow = __builtin_amdgcn_readlane(rhi, kWave - 1);
    int32_t cf = 0, cl = 0, jz = jw;
    for (;;) {  // uniform
      if (jz + 1 - jwin >= kWave) {
        jwin = jz;
        sbw = sb[min(jwin + lane, ns + kSeekPad - 1)];
      }
      const int32_t cnt = __popcll(__ballot(sbw <= maxrow));  // a prefix: the table ascends
      const int32_t jend = jwin + cnt - 1;
      for (int32_t jj = jz + 1; jj <= jend; ++jj) {
        const int32_t bnd = __builtin_amdgcn_readlane(sbw, jj - jwin);
        cf += rlo >= bnd;
        cl += rhi >= bnd;
      }
      jz = max(jz, jend);
      if (cnt < kWave) break;
    }
    // jz <= ns (sb[ns + 1 ..] are sentinels above every row), so jf + 1 lies
    // inside the table
    const int32_t jf = jw + cf;
    const int32_t nx = cl - cf;  // boundaries inside the lane's rows
    const int32_t d0 = sd[jf], b1 = sb[jf + 1], d1 = sd[jf + 1];
    jw = jz;
    // Every lane issues its 8 stores, one per arc: an arc that ends a row
    // the wave writes stores the row's minimum at its range-major index, any
    // other store gets an offset past the buffer and is dropped (no branch
    // around a store: the loads of the next tiles stay in flight). Lanes
    // crossing several boundaries store on the path below instead.
    const bool slow = nx > 1;
    int32_t row = t.row0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      row += static_cast<int32_t>((t.my9 >> e) & 1u);
      const bool ends = (t.my9 >> (e + 1)) & 1u;  // arc e ends its row
      const bool started_here = (t.my9 & ((2u << e) - 1u)) != 0u;
      const int32_t v = started_here ? rv[e] : min(rv[e], lin);
      const int32_t d = row >= b1 ? d1 : d0;
      const bool ok = ends && !slow && row >= own0 && row < r1;
      const uint32_t off = ok ? 4u * static_cast<uint32_t>(row + d) : kDropOff + 4u * e;
      __builtin_amdgcn_raw_buffer_store_b32(static_cast<uint32_t>(v), out, off, 0, 0);
    }
    if (__any(slow)) {
      row = t.row0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        row += static_cast<int32_t>((t.my9 >> e) & 1u);
        if (slow && ((t.my9 >> (e + 1)) & 1u) && row >= own0 && row < r1) {
          const bool started_here = (t.my9 & ((2u << e) - 1u)) != 0u;
          int32_t j = jf;
          while (sb[j + 1] <= row) ++j;
          pmin[row + sd[j]] = started_here ? rv[e] : min(rv[e], lin);
        }
      }
    }
    carry = __builtin_amdgcn_readlane(A, kWave - 1);
    open_row = __builtin_amdgcn_readlane(row, kWave - 1);
  }
  // the row open at the range's end, if the wave owns it: read on to its end
  const int64_t end_arc = static_cast<int64_t>(qz + 1) * kRowTile;
  const bool continues = !((heads[end_arc >> 6].bits) & 1ull);
  if (continues && open_row >= own0 && open_row < r1) {
    for (int64_t q = qz + 1;; ++q) {
      const MinTile t = load_min_tile<kW>(col16, heads, w_arcs, ad, q, lane, &ovf);
      // arcs before the tile's first head belong to the open row
      const int fh = (t.my9 & 0xFFu) ? __ffs(t.my9 & 0xFFu) - 1 : 8;  // first head in the lane
      const uint64_t hl = __ballot(fh < 8);
      const int first_lane = hl ? __ffsll(static_cast<long long>(hl)) - 1 : kWave;
      int32_t mine = kInf;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (lane < first_lane || (lane == first_lane && e < fh)) mine = min(mine, t.x[e]);
      carry = min(carry, gcd::wave_min(mine));
      if (first_lane < kWave) break;  // bits past the last arc are set, so this ends
    }
    if (lane == 0) {
      int32_t j = jw;
      while (sb[j + 1] <= open_row) ++j;
      pmin[open_row + sd[j]] = carry;
    }
  }
  if (__any(ovf) && lane == 0) stats[kOverflow] = 1;
}

// Size in bytes of the partial minima of a stream-layout partition (P + 8
// entries, below 2^31 bytes by the layout's own limit).
inline uint32_t pmin_bytes(const gc_tocab_s* t) { return static_cast<uint32_t>(sizeof(int32_t) * (t->P + 8)); }

// Figure 5 merge of the stream-layout SSSP partial minima, read as streams:
// range j's partials of every block are one contiguous slice [rstart[j],
// rstart[j+1]) of pmin / id16s (the position table's range-major order). A
// persistent work-group (two per CU) walks ranges j = blockIdx.x,
// blockIdx.x + gridDim.x, ...: 16-byte / 8-byte loads of 4 entries, LDS
// minima, then the range's vertices are updated (distance, next status
// bit, queue) and the minima reset for the next range, whose first loads
// are issued before that update.
template <int K, int NT, bool kBfs>
__global__ __launch_bounds__(NT) void k_sssp_merge_stream(const int32_t* __restrict__ rstart,
                                                          const uint16_t* __restrict__ id16s,
                                                          const int32_t* __restrict__ pmin, int32_t R, int32_t n,
                                                          int32_t* __restrict__ dist, uint32_t* __restrict__ next,
                                                          int32_t* __restrict__ queue, int32_t* __restrict__ stats,
                                                          int32_t level, uint32_t* __restrict__ visited) {
  __shared__ int32_t best[K];
  for (int i = threadIdx.x; i < K; i += NT) best[i] = kInf;
  __syncthreads();
  const ti32x4* p4 = reinterpret_cast<const ti32x4*>(pmin);
  const uint64_t* i4 = reinterpret_cast<const uint64_t*>(id16s);
  constexpr int kU = 4;  // groups of 4 entries per thread and step (two register sets in turn)
  constexpr int32_t kStep = NT * kU;
  ti32x4 pa[kU], pb[kU];
  uint64_t ia[kU], ib[kU];
  int32_t a = 0, z = 0, g0 = 0, g1 = 0;
  auto bounds = [&](int32_t j) {
    a = rstart[j];
    z = rstart[j + 1];
    g0 = a >> 2;
    g1 = (z + 3) >> 2;
  };
  // loads clamped to the range's last group: no branch, so the compiler's
  // count of outstanding loads holds on every path
  auto load = [&](int32_t g, ti32x4 (&p)[kU], uint64_t (&id)[kU]) {
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int32_t gg = min(g + k * NT, g1 - 1);
      p[k] = gcd::ld_stream(p4 + gg);
      id[k] = gcd::ld_stream(i4 + gg);
    }
  };
  auto take = [&](int32_t g, const ti32x4 (&p)[kU], const uint64_t (&id)[kU]) {
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int32_t e0 = 4 * (g + k * NT);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (e0 + e >= a && e0 + e < z && p[k][e] != kInf) atomicMin(&best[(id[k] >> (16 * e)) & 0xFFFFu], p[k][e]);
    }
  };
  const int32_t tid = threadIdx.x;
  int32_t j = blockIdx.x;
  if (j < R) {
    bounds(j);
    if (g0 < g1) load(g0 + tid, pa, ia);  // uniform
  }
  for (; j < R; j += gridDim.x) {
    for (int32_t g = g0 + tid; g < g1; g += 2 * kStep) {
      load(g + kStep, pb, ib);
      take(g, pa, ia);
      load(g + 2 * kStep, pa, ia);
      take(g + kStep, pb, ib);
    }
    __syncthreads();
    const int32_t v0 = j * K;
    static_assert(K % NT == 0 && NT % kWave == 0, "whole waves over the range");
    constexpr int kPer = K / NT;
    // The range's vertices v0 + tid + u NT. Their minima come from LDS and,
    // for those with a candidate, their distance (BFS: their visited word)
    // is loaded into registers before the next range's first minima, so
    // that the update waits for neither those loads nor one load per step;
    // a vertex with no candidate (or past n) reads the range's first vertex
    // instead, one line per wave.
    int32_t bi[kPer], cur[kPer];
    const uint32_t last = static_cast<uint32_t>(n - 1 - v0);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int32_t i = tid + u * NT;
      bi[u] = best[i];
      best[i] = kInf;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const uint32_t o = static_cast<uint32_t>(tid + u * NT);
      const bool need = o <= last && (kBfs ? bi[u] == 0 : bi[u] != kInf);
      const uint32_t oo = need ? o : 0u;
      cur[u] = kBfs ? static_cast<int32_t>(visited[(static_cast<uint32_t>(v0) + oo) >> 5]) : dist[v0 + oo];
    }
    const int32_t jn = j + gridDim.x;
    if (jn < R) {  // uniform: the next range's first loads, in flight during the update
      bounds(jn);
      if (g0 < g1) load(g0 + tid, pa, ia);
    }
    // distance (or depth) and status bits, with one atomic per 32-bit status
    // word (a wave's 32 lanes hold one word's vertices, the range starts on
    // a word), then one queue append for the work-group
    uint32_t took = 0;  // bit u: vertex v0 + tid + u NT entered the next frontier
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int32_t v = v0 + tid + u * NT;
      bool improved;
      if (kBfs) {  // depth: a vertex not yet reached with an in-neighbour in the frontier
        improved = v < n && bi[u] == 0 && !((static_cast<uint32_t>(cur[u]) >> (v & 31)) & 1u);
        if (improved) dist[v] = level + 1;
      } else {
        improved = v < n && bi[u] != kInf && bi[u] < cur[u];
        if (improved) dist[v] = bi[u];
      }
      const uint64_t m = __ballot(improved);
      const int lane = tid & (kWave - 1);
      const uint32_t word = static_cast<uint32_t>(m >> (lane & 32));
      if ((lane & 31) == 0 && word != 0u) {
        atomicOr(&next[v >> 5], word);
        if (kBfs) atomicOr(&visited[v >> 5], word);
      }
      took |= static_cast<uint32_t>(improved) << u;
    }
    block_append_bits<NT>(took, v0 + tid, NT, queue, stats + kQLen);
    __syncthreads();
  }
}

template <int K, bool kFlat>
__global__ __launch_bounds__(kThreads) void k_sssp_merge(const int32_t* __restrict__ range_ptr, int32_t B,
                                                         const uint16_t* __restrict__ id16,
                                                         const int32_t* __restrict__ pmin, int32_t n,
                                                         int32_t* __restrict__ dist, uint32_t* __restrict__ next,
                                                         int32_t* __restrict__ queue, int32_t* __restrict__ stats) {
  __shared__ int32_t best[K];
  const int32_t v0 = blockIdx.x * K;
  for (int i = threadIdx.x; i < K; i += kThreads) best[i] = kInf;
  gcm::merge_slices<kFlat, kThreads>(range_ptr, B, id16, pmin, blockIdx.x, [&](uint32_t v, int32_t p) {
    if (p != kInf) atomicMin(&best[v], p);
  });
  for (int i = threadIdx.x; i < K; i += kThreads) {
    const int32_t v = v0 + i;
    bool improved = false;
    if (v < n && best[i] < dist[v]) {
      dist[v] = best[i];
      improved = true;
    }
    wave_bits_set(next, v, improved);
    block_append(improved, v, queue, stats + kQLen);
  }
}

// Data-driven push relaxation: atomicMin on dist; a vertex whose distance
// dropped enters the next frontier once (round stamp in mark).
__global__ __launch_bounds__(kThreads) void k_sssp_push(const int32_t* __restrict__ queue_in, int32_t qn,
                                                        const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colidx,
                                                        const int32_t* __restrict__ w, int32_t* __restrict__ dist,
                                                        int32_t round, int32_t* __restrict__ mark,
                                                        uint32_t* __restrict__ next, int32_t* __restrict__ queue,
                                                        int32_t* __restrict__ stats) {
  __shared__ int32_t start[kThreads];
  __shared__ int32_t first[kThreads];
  __shared__ int32_t du_s[kThreads];
  __shared__ int32_t wave_tot[kThreads / kWave];
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  int32_t b = 0, len = 0, du = 0;
  if (i < qn) {
    const int32_t u = queue_in[i];
    b = rowptr[u];
    len = rowptr[u + 1] - b;
    du = dist[u];
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int incl = gcd::wave_incl_scan(len);
  if (lane == kWave - 1) wave_tot[wid] = incl;
  __syncthreads();
  int off = 0, total = 0;
#pragma unroll
  for (int w2 = 0; w2 < kThreads / kWave; ++w2) {
    off += (w2 < wid) ? wave_tot[w2] : 0;
    total += wave_tot[w2];
  }
  start[threadIdx.x] = off + incl - len;
  first[threadIdx.x] = b;
  du_s[threadIdx.x] = du;
  __syncthreads();
  const int32_t rounds = (total + kThreads - 1) / kThreads;
  for (int32_t r = 0; r < rounds; ++r) {
    const int32_t a = r * kThreads + threadIdx.x;
    bool fresh = false;
    int32_t v = 0;
    if (a < total) {
      int lo = 0, hi = kThreads - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= a) lo = mid;
        else hi = mid - 1;
      }
      const int32_t e = first[lo] + (a - start[lo]);
      v = colidx[e];
      const int64_t nd = static_cast<int64_t>(du_s[lo]) + w[e];
      if (nd >= kInf) {
        stats[kOverflow] = 1;
      } else if (static_cast<int32_t>(nd) < dist[v]) {
        const int32_t old = atomicMin(&dist[v], static_cast<int32_t>(nd));
        if (static_cast<int32_t>(nd) < old) {
          bit_set(next, v);
          fresh = atomicExch(&mark[v], round) != round;
        }
      }
    }
    block_append(fresh, v, queue, stats + kQLen);
  }
}

// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Betweenness centrality (Section 4's BC benchmark): the BFS levels above
// also count shortest paths, sigma[v] = sum of sigma[u] over in-neighbours u
// one level up (Algorithm 3's update); then the dependencies are
// accumulated level by level backwards (Brandes).

__global__ void k_set_sigma(int32_t src, double* __restrict__ sigma) { sigma[src] = 1.0; }

__global__ void k_fill_f64(double* __restrict__ a, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = 0.0;
}

// Sum of sigma[u] over in-arcs [b, e) from active sources u (FP64); rows
// longer than kHeavy are summed by the whole wave.
__device__ __forceinline__ double scan_sigma(const int32_t* __restrict__ col, const uint32_t* __restrict__ front,
                                             const double* __restrict__ sigma, bool active, int32_t b, int32_t e) {
  const int lane = gcd::lane_id();
  const bool heavy = active && (e - b) > kHeavy;
  double s = 0.0;
  if (active && !heavy) {
    int32_t i = b;
    for (; i + 4 <= e; i += 4) {  // four arcs' loads in flight at a time
      int32_t u[4];
      bool on[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) u[k] = col[i + k];
#pragma unroll
      for (int k = 0; k < 4; ++k) on[k] = bit_test(front, u[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k) s += on[k] ? sigma[u[k]] : 0.0;
    }
    for (; i < e; ++i) {
      const int32_t u = col[i];
      if (bit_test(front, u)) s += sigma[u];
    }
  }
  uint64_t pending = __ballot(heavy);
  while (pending) {
    const int owner = __ffsll(static_cast<long long>(pending)) - 1;
    pending &= pending - 1;
    const int32_t hb = __shfl(b, owner, kWave), he = __shfl(e, owner, kWave);
    double m = 0.0;
    for (int32_t i = hb + lane; i < he; i += kWave) {
      const int32_t u = col[i];
      if (bit_test(front, u)) m += sigma[u];
    }
    m = gcd::wave_sum(m);
    if (lane == owner) s = m;
  }
  return s;
}

// Topology-driven pull: an unvisited vertex with an active in-neighbour
// joins the next level with the sum of their path counts.
__global__ __launch_bounds__(kThreads) void k_bc_pull(const int32_t* __restrict__ t_rowptr,
                                                      const int32_t* __restrict__ t_col, int32_t n,
                                                      const uint32_t* __restrict__ front, int32_t* __restrict__ depth,
                                                      int32_t level, double* __restrict__ sigma,
                                                      uint32_t* __restrict__ next, uint32_t* __restrict__ visited,
                                                      int32_t* __restrict__ queue, int32_t* __restrict__ stats) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  bool active = false;
  int32_t b = 0, e = 0;
  if (v < n && !bit_test(visited, v)) {
    active = true;
    b = t_rowptr[v];
    e = t_rowptr[v + 1];
  }
  const double sum = scan_sigma(t_col, front, sigma, active, b, e);
  const bool found = active && sum > 0.0;  // every active vertex has sigma >= 1
  if (found) {
    depth[v] = level + 1;
    sigma[v] = sum;
  }
  wave_bits_set(next, v, found);
  wave_bits_set(visited, v, found);
  block_append(found, v, queue, stats + kQLen);
}

// TOCAB pull, per block: part[l] = sum of sigma over the active sources of
// this block among the in-arcs of local row l (0 when its vertex is visited).
__global__ __launch_bounds__(kThreads) void k_bc_tocab(const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ id_map, int64_t P,
                                                       const uint32_t* __restrict__ visited,
                                                       const uint32_t* __restrict__ front,
                                                       const double* __restrict__ sigma, double* __restrict__ part) {
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kThreads; base < P;
       base += static_cast<int64_t>(gridDim.x) * kThreads) {  // uniform per work-group
    const int64_t l = base + threadIdx.x;
    bool active = false;
    int32_t b = 0, e = 0;
    if (l < P && !bit_test(visited, id_map[l])) {
      active = true;
      b = row_ptr[l];
      e = row_ptr[l + 1];
    }
    const double sum = scan_sigma(col, front, sigma, active, b, e);
    if (l < P) part[l] = sum;
  }
}

// Merge of the per-block path counts over vertex range j (FP64 LDS sums),
// fused with the depth / sigma update and the next frontier.
template <int K, bool kFlat>
__global__ __launch_bounds__(kThreads) void k_bc_merge(const int32_t* __restrict__ range_ptr, int32_t B,
                                                       const uint16_t* __restrict__ id16,
                                                       const double* __restrict__ part, int32_t n,
                                                       int32_t* __restrict__ depth, int32_t level,
                                                       double* __restrict__ sigma, uint32_t* __restrict__ next,
                                                       uint32_t* __restrict__ visited, int32_t* __restrict__ queue,
                                                       int32_t* __restrict__ stats) {
  __shared__ double acc[K];
  gcm::merge_accumulate<K, kFlat, kThreads>(range_ptr, B, id16, part, blockIdx.x, acc);
  const int32_t v0 = blockIdx.x * K;
  for (int i = threadIdx.x; i < K; i += kThreads) {
    const int32_t v = v0 + i;
    const bool found = v < n && acc[i] > 0.0 && !bit_test(visited, v);
    if (found) {
      depth[v] = level + 1;
      sigma[v] = acc[i];
    }
    wave_bits_set(next, v, found);
    wave_bits_set(visited, v, found);
    block_append(found, v, queue, stats + kQLen);
  }
}

// Data-driven push (Algorithm 3): like the BFS push, plus sigma[v] +=
// sigma[u] (FP64 atomic) for every arc u -> v that lands one level down.
__global__ __launch_bounds__(kThreads) void k_bc_push(const int32_t* __restrict__ queue_in, int32_t qn,
                                                      const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colidx,
                                                      int32_t* __restrict__ depth, int32_t level,
                                                      double* __restrict__ sigma, uint32_t* __restrict__ next,
                                                      uint32_t* __restrict__ visited, int32_t* __restrict__ queue,
                                                      int32_t* __restrict__ stats) {
  __shared__ int32_t start[kThreads];
  __shared__ int32_t first[kThreads];
  __shared__ double su[kThreads];
  __shared__ int32_t wave_tot[kThreads / kWave];
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  int32_t b = 0, len = 0;
  double sg = 0.0;
  if (i < qn) {
    const int32_t u = queue_in[i];
    b = rowptr[u];
    len = rowptr[u + 1] - b;
    sg = sigma[u];
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
  su[threadIdx.x] = sg;
  __syncthreads();
  // every thread runs the same number of rounds (block_append synchronises the work-group)
  const int32_t rounds = (total + kThreads - 1) / kThreads;
  for (int32_t r = 0; r < rounds; ++r) {
    const int32_t a = r * kThreads + threadIdx.x;
    bool disc = false;
    int32_t v = 0;
    if (a < total) {
      int lo = 0, hi = kThreads - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= a) lo = mid;
        else hi = mid - 1;
      }
      v = colidx[first[lo] + (a - start[lo])];
      int32_t old = depth[v];
      if (old == kInf) {
        old = atomicCAS(&depth[v], kInf, level + 1);
        if (old == kInf) {
          disc = true;
          bit_set(next, v);
          bit_set(visited, v);
        }
      }
      if (old == kInf || old == level + 1) atomicAdd(&sigma[v], su[lo]);
    }
    block_append(disc, v, queue, stats + kQLen);
  }
}

// ---------------------------------------------------------------------------
// Data-driven push balanced over arcs, for frontiers with many arcs: pre is
// the exclusive scan of the queued vertices' out-degrees, and each lane takes
// kPushArcs consecutive arcs of their concatenated out-arc lists, so a hub's
// arcs spread over many work-groups instead of one. The relaxation is a
// functor: src(u) loads what u passes along its arcs, relax(v, e, x)
// handles arc e into v and returns true when v enters the next frontier.
constexpr int kPushArcs = 8;

struct BfsRelax {  // Algorithm 3's CAS on depth
  int32_t* depth;
  int32_t level;
  uint32_t* next;
  uint32_t* visited;
  __device__ int32_t src(int32_t) const { return 0; }
  __device__ bool relax(int32_t v, int64_t, int32_t) const {
    if (depth[v] == kInf && atomicCAS(&depth[v], kInf, level + 1) == kInf) {
      bit_set(next, v);
      bit_set(visited, v);
      return true;
    }
    return false;
  }
};

struct SsspRelax {  // atomicMin on dist; a vertex is queued once per round (stamp in mark)
  const int32_t* w;
  int32_t* dist;
  int32_t round;
  int32_t* mark;
  uint32_t* next;
  int32_t* stats;
  __device__ int32_t src(int32_t u) const { return dist[u]; }
  __device__ bool relax(int32_t v, int64_t e, int32_t du) const {
    const int64_t nd = static_cast<int64_t>(du) + w[e];
    if (nd >= kInf) {
      stats[kOverflow] = 1;
    } else if (static_cast<int32_t>(nd) < dist[v]) {
      const int32_t old = atomicMin(&dist[v], static_cast<int32_t>(nd));
      if (static_cast<int32_t>(nd) < old) {
        bit_set(next, v);
        return atomicExch(&mark[v], round) != round;
      }
    }
    return false;
  }
};

struct BcRelax {  // the BFS CAS plus sigma[v] += sigma[u] for arcs that land one level down
  int32_t* depth;
  int32_t level;
  double* sigma;
  uint32_t* next;
  uint32_t* visited;
  __device__ double src(int32_t u) const { return sigma[u]; }
  __device__ bool relax(int32_t v, int64_t, double su) const {
    bool disc = false;
    int32_t old = depth[v];
    if (old == kInf) {
      old = atomicCAS(&depth[v], kInf, level + 1);
      if (old == kInf) {
        disc = true;
        bit_set(next, v);
        bit_set(visited, v);
      }
    }
    if (old == kInf || old == level + 1) atomicAdd(&sigma[v], su);
    return disc;
  }
};

template <class Relax>
__global__ __launch_bounds__(kThreads) void k_push_arcs(const int32_t* __restrict__ queue_in,
                                                        const int32_t* __restrict__ pre, int32_t qn,
                                                        const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colidx, Relax r,
                                                        int32_t* __restrict__ queue, int32_t* __restrict__ stats) {
  const int64_t end = pre[qn];
  const int64_t a0 = (static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x) * kPushArcs;
  int32_t i = 0;
  if (a0 < end) {  // the queued vertex whose arcs contain a0: the last i with pre[i] <= a0
    int32_t h = qn - 1;
    while (i < h) {
      const int32_t mid = i + ((h - i + 1) >> 1);
      if (pre[mid] <= a0) i = mid;
      else h = mid - 1;
    }
  }
  int64_t ub = 0, ue = 0, rb = 0;
  auto x = r.src(0);
  if (a0 < end) {
    const int32_t u = queue_in[i];
    ub = pre[i];
    ue = pre[i + 1];
    rb = rowptr[u];
    x = r.src(u);
  }
  // the thread's kPushArcs arcs; the vertices they discover are appended
  // together at the end (a work-group append per arc step kept the waves in
  // lock-step through two barriers per step)
  int32_t found[kPushArcs];
  uint32_t took = 0;
#pragma unroll
  for (int k = 0; k < kPushArcs; ++k) {
    const int64_t a = a0 + k;
    found[k] = 0;
    if (a < end) {
      while (a >= ue) {  // next queued vertex with an arc at a
        ++i;
        const int32_t u = queue_in[i];
        ub = ue;
        ue = pre[i + 1];
        rb = rowptr[u];
        x = r.src(u);
      }
      const int64_t e = rb + (a - ub);
      const int32_t v = colidx[e];
      found[k] = v;
      took |= static_cast<uint32_t>(r.relax(v, e, x)) << k;
    }
  }
  block_append_list<kThreads, kPushArcs>(took, found, queue, stats + kQLen);
}

__global__ void k_order_degree(const int32_t* __restrict__ order, int32_t cnt, const int32_t* __restrict__ rowptr,
                               int32_t* __restrict__ deg) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) {
    const int32_t v = order[i];
    deg[i] = rowptr[v + 1] - rowptr[v];
  }
}

// Backward sweep. coef[v] = (1 + delta[v]) / sigma[v]; two arrays alternate
// from level to level. When depth d is processed, the array it reads holds
// the coefficients of depth d + 1 and zero for depth d and every depth above
// (an arc from depth d reaches depth d + 1 at most), so the sum over all
// out-arcs of coef needs no depth test; the array it writes is zero at the
// vertices of depth d.
constexpr int kBackArcs = 8;  // consecutive arcs per lane

// Sums for the vertices order[lo, hi) of one depth, balanced over arcs: the
// level's out-arcs, concatenated in level order (pre = exclusive scan of the
// degrees along order), are cut into kBackArcs-arc pieces, one per lane. A
// lane adds the sum of coef_in over each vertex's arcs in its piece into
// coef_out[v] (FP64 atomic), or stores it when the piece holds all of v's
// arcs.
__global__ __launch_bounds__(kThreads) void k_bc_back_arcs(const int32_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ colidx,
                                                           const int32_t* __restrict__ order,
                                                           const int32_t* __restrict__ pre, int32_t lo, int32_t hi,
                                                           const double* __restrict__ coef_in,
                                                           double* __restrict__ coef_out) {
  const int64_t end = pre[hi];
  const int64_t a0 = pre[lo] + (static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x) * kBackArcs;
  if (a0 >= end) return;
  const int64_t a1 = a0 + kBackArcs < end ? a0 + kBackArcs : end;
  // the vertex whose arcs contain a0: the last i in [lo, hi) with pre[i] <= a0
  int32_t l = lo, h = hi - 1;
  while (l < h) {
    const int32_t mid = l + ((h - l + 1) >> 1);
    if (pre[mid] <= a0) l = mid;
    else h = mid - 1;
  }
  // owner and position of each of the lane's arcs, then all column loads,
  // then all coefficient gathers, so that kBackArcs gathers are in flight
  int64_t pos[kBackArcs];
  int32_t vid[kBackArcs];
  bool whole[kBackArcs];
  {
    int32_t i = l;
    int32_t v = order[i];
    int64_t vb = pre[i], ve = pre[i + 1];
    int64_t rb = rowptr[v];
#pragma unroll
    for (int k = 0; k < kBackArcs; ++k) {
      const int64_t a = a0 + k;
      if (a < a1) {
        while (a >= ve) {  // next vertex with an arc at a (vertices without out-arcs are skipped)
          ++i;
          vb = ve;
          ve = pre[i + 1];
          v = order[i];
          rb = rowptr[v];
        }
        pos[k] = rb + (a - vb);
        vid[k] = v;
        whole[k] = vb >= a0 && ve <= a1;
      } else {
        pos[k] = pos[0];
        vid[k] = -1;
        whole[k] = false;
      }
    }
  }
  int32_t w[kBackArcs];
#pragma unroll
  for (int k = 0; k < kBackArcs; ++k) w[k] = colidx[pos[k]];
  double c[kBackArcs];
#pragma unroll
  for (int k = 0; k < kBackArcs; ++k) c[k] = coef_in[w[k]];
  // sums per vertex run: a plain store when the lane holds all of v's arcs
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < kBackArcs; ++k) {
    if (vid[k] < 0) break;
    sum += c[k];
    if (k == kBackArcs - 1 || vid[k + 1] != vid[k]) {
      if (whole[k]) coef_out[vid[k]] = sum;
      else if (sum != 0.0) atomicAdd(&coef_out[vid[k]], sum);
      sum = 0.0;
    }
  }
}

// The same step in the push direction, chosen when the next level's in-arcs
// are fewer than this level's out-arcs: over the in-arcs v -> w of the
// vertices w = order[lo, hi) of depth d + 1 (pre = exclusive scan of their
// in-degrees along order), balanced like k_bc_back_arcs, coef_in[w] is
// added into coef_out[v] for every v of depth d (FP64 atomic).
__global__ __launch_bounds__(kThreads) void k_bc_back_push(const int32_t* __restrict__ t_rowptr,
                                                           const int32_t* __restrict__ t_colidx,
                                                           const int32_t* __restrict__ order,
                                                           const int32_t* __restrict__ pre, int32_t lo, int32_t hi,
                                                           const int32_t* __restrict__ depth, int32_t d,
                                                           const double* __restrict__ coef_in,
                                                           double* __restrict__ coef_out) {
  const int64_t end = pre[hi];
  const int64_t a0 = pre[lo] + (static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x) * kBackArcs;
  if (a0 >= end) return;
  const int64_t a1 = a0 + kBackArcs < end ? a0 + kBackArcs : end;
  int32_t l = lo, h = hi - 1;  // the vertex whose in-arcs contain a0
  while (l < h) {
    const int32_t mid = l + ((h - l + 1) >> 1);
    if (pre[mid] <= a0) l = mid;
    else h = mid - 1;
  }
  // position and coefficient of each of the lane's arcs, then all column
  // loads, then all depth gathers
  int64_t pos[kBackArcs];
  double cw[kBackArcs];
  {
    int32_t i = l;
    int32_t w = order[i];
    int64_t wb = pre[i], we = pre[i + 1];
    int64_t rb = t_rowptr[w];
    double c = coef_in[w];
#pragma unroll
    for (int k = 0; k < kBackArcs; ++k) {
      const int64_t a = a0 + k;
      if (a < a1) {
        while (a >= we) {  // next vertex with an in-arc at a
          ++i;
          wb = we;
          we = pre[i + 1];
          w = order[i];
          rb = t_rowptr[w];
          c = coef_in[w];
        }
        pos[k] = rb + (a - wb);
        cw[k] = c;
      } else {
        pos[k] = pos[0];
        cw[k] = 0.0;
      }
    }
  }
  int32_t v[kBackArcs];
#pragma unroll
  for (int k = 0; k < kBackArcs; ++k) v[k] = t_colidx[pos[k]];
  bool on[kBackArcs];
#pragma unroll
  for (int k = 0; k < kBackArcs; ++k) on[k] = a0 + k < a1 && depth[v[k]] == d;
#pragma unroll
  for (int k = 0; k < kBackArcs; ++k)
    if (on[k]) atomicAdd(&coef_out[v[k]], cw[k]);
}

// delta[v] = sigma[v] * (sum held in coef[v]) is added into bc[v], and
// coef[v] becomes (1 + delta[v]) / sigma[v].
__global__ void k_bc_finish(const int32_t* __restrict__ order, int32_t cnt, const double* __restrict__ sigma,
                            double* __restrict__ coef, double* __restrict__ bc) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) {
    const int32_t v = order[i];
    const double sg = sigma[v];
    const double d = sg * coef[v];
    bc[v] += d;
    coef[v] = (1.0 + d) / sg;
  }
}

template <int K>
struct BcMerge {
  template <class... A>
  static void run(int32_t R, hipStream_t s, const int32_t* range_ptr, int32_t B, A... a) {
    if (B <= gcm::kFlatB) k_bc_merge<K, true><<<R, kThreads, 0, s>>>(range_ptr, B, a...);
    else k_bc_merge<K, false><<<R, kThreads, 0, s>>>(range_ptr, B, a...);
  }
};

// Work-groups for one item per thread. Item counts here are vertex, queue
// or arc counts below 2^31, so the grid never needs a cap.
inline int grid_for(int64_t items, int threads) {
  return static_cast<int>(std::max<int64_t>(1, (items + threads - 1) / threads));
}

// Work-groups of the grid-stride TOCAB row kernels: at most kRowGrid, so
// partitions with more than kRowGrid * kThreads local rows take several
// passes (RMAT-24 partitions do).
constexpr int64_t kRowGrid = 1 << 16;
inline int row_grid(int64_t rows) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((rows + kThreads - 1) / kThreads, kRowGrid)));
}

enum class Mode { kPull, kTocab, kPush };

// Direction choice (Section 3.3): with the direction-optimising rule of
// Beamer et al. (the paper's [Direction] reference; alpha = 14, beta = 24)
// a level pulls when the frontier's out-arcs exceed the unexplored arcs /
// alpha and returns to push when the frontier shrinks below n / beta. A
// pull level is blocked (TOCAB) when its working set exceeds the cache: the
// frontier must be large (4 bytes per frontier out-arc above one XCD's L2,
// the paper's test) and the array its random reads land in must not fit in
// that L2 either. With one status bit per vertex a BFS pull reads only the
// bitmap (n / 8 bytes: 2 MB at 2^24 vertices, so plain pull's reads already
// hit L2 and blocking only adds its local rows); an SSSP pull also gathers
// the 4-byte distances of active sources.
struct Heuristic {
  static constexpr double kAlpha = 14.0, kBeta = 24.0;
  static constexpr double kCacheBytes = 4.0 * 1024 * 1024;  // one XCD's L2
  // BFS over a stream-layout partition: TOCAB pull on graphs with at most
  // kBfsTocabDegree arcs per vertex, while at least 1/64 of the arcs still
  // end at unvisited vertices. Measured per level on the grid (4 arcs per
  // vertex), uniform (8) and R-MAT 22 / 24 (16) graphs: a TOCAB pull level
  // costs 3-6 ps per arc, a plain-pull level about 50 ps per vertex while
  // many vertices are unvisited (one thread per vertex, early exit, status
  // bits in L2), so TOCAB halves the grid's dense levels, gains a quarter
  // on the uniform graph's and ties on R-MAT's; once fewer than 1/64 of the
  // arcs end at unvisited vertices the plain pull is up to three times
  // faster.
  static constexpr double kBfsTocabShare = 1.0 / 64.0;
  static constexpr double kBfsTocabDegree = 10.0;
  bool pulling = false;
  // m_u: unexplored out-arcs (the direction test); m_u_in: in-arcs of the
  // unvisited vertices; stream: the TOCAB partition has the stream layout
  Mode pick(int64_t n, int64_t n_f, int64_t m_f, int64_t m_u, bool have_tocab, bool bfs, int64_t m = 0,
            int64_t m_u_in = 0, bool stream = false) {
    if (!pulling && static_cast<double>(m_f) > static_cast<double>(m_u) / kAlpha) pulling = true;
    else if (pulling && static_cast<double>(n_f) < static_cast<double>(n) / kBeta) pulling = false;
    if (!pulling) return Mode::kPush;
    if (bfs && have_tocab && stream)
      return static_cast<double>(m) <= kBfsTocabDegree * static_cast<double>(n) &&
                     static_cast<double>(m_u_in) >= kBfsTocabShare * static_cast<double>(m)
                 ? Mode::kTocab
                 : Mode::kPull;
    const double gathered = static_cast<double>(n) / 8.0 + (bfs ? 0.0 : 4.0 * static_cast<double>(n));
    const bool large = 4.0 * static_cast<double>(m_f) > kCacheBytes && gathered > kCacheBytes;
    return (have_tocab && large) ? Mode::kTocab : Mode::kPull;
  }
};

using gcx::kLearnedGate;

template <template <int> class Kern, class... Args>
hipError_t launch_by_k(int32_t k, int32_t R, hipStream_t s, Args... args) {
  switch (k) {
    case 256: Kern<256>::run(R, s, args...); break;
    case 512: Kern<512>::run(R, s, args...); break;
    case 1024: Kern<1024>::run(R, s, args...); break;
    case 2048: Kern<2048>::run(R, s, args...); break;
    case 4096: Kern<4096>::run(R, s, args...); break;
    case 8192: Kern<8192>::run(R, s, args...); break;
    case 16384: Kern<16384>::run(R, s, args...); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int K>
struct BfsMerge {
  template <class... A>
  static void run(int32_t R, hipStream_t s, const int32_t* range_ptr, int32_t B, A... a) {
    if (B <= gcm::kFlatB) k_bfs_merge<K, true><<<R, kThreads, 0, s>>>(range_ptr, B, a...);
    else k_bfs_merge<K, false><<<R, kThreads, 0, s>>>(range_ptr, B, a...);
  }
};

template <int K>
struct SsspMerge {
  template <class... A>
  static void run(int32_t R, hipStream_t s, const int32_t* range_ptr, int32_t B, A... a) {
    if (B <= gcm::kFlatB) k_sssp_merge<K, true><<<R, kThreads, 0, s>>>(range_ptr, B, a...);
    else k_sssp_merge<K, false><<<R, kThreads, 0, s>>>(range_ptr, B, a...);
  }
};

// Compute units of the GPU (read once).
int32_t device_cus() {
  static const int32_t cus = [] {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || c <= 0)
      c = 256;
    return c;
  }();
  return cus;
}

template <int K>
struct SsspMergeStream {
  // LDS minima of K int32: two work-groups per CU; no more threads than K
  static constexpr int kNT = K >= 8192 ? 1024 : (K >= 512 ? 512 : K);
  template <class... A>
  static void run(int32_t R, hipStream_t s, A... a) {
    const int32_t grid = std::max(1, std::min(R, 2 * device_cus()));
    k_sssp_merge_stream<K, kNT, false><<<grid, kNT, 0, s>>>(a...);
  }
};

template <int K>
struct BfsMergeStream {
  static constexpr int kNT = SsspMergeStream<K>::kNT;
  template <class... A>
  static void run(int32_t R, hipStream_t s, A... a) {
    const int32_t grid = std::max(1, std::min(R, 2 * device_cus()));
    k_sssp_merge_stream<K, kNT, true><<<grid, kNT, 0, s>>>(a...);
  }
};

// *flag = 1 if a weight lies outside [0, 255].
__global__ void k_weight_range(const int32_t* __restrict__ w, int64_t m, int32_t* __restrict__ flag) {
  bool wide = false;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    wide |= static_cast<uint32_t>(w[i]) > 255u;
  if (__any(wide) && gcd::lane_id() == 0) *flag = 1;
}

// Weights as bytes in arc order, zero past m.
__global__ void k_weight_bytes(const int32_t* __restrict__ w, int64_t m, int64_t m_pad, uint8_t* __restrict__ w8) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m_pad;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    w8[i] = i < m ? static_cast<uint8_t>(w[i]) : 0;
}

// One device int32 for the weight check (per process, allocated once).
int32_t* g_range_flag() {
  static int32_t* flag = [] {
    void* p = nullptr;
    return hipMalloc(&p, sizeof(int32_t)) == hipSuccess ? static_cast<int32_t*>(p) : nullptr;
  }();
  return flag;
}

// Integer weights of a stream-layout partition in its arc order, padded with
// zeros to the layout's length (built by the first SSSP round over it), and
// the LDS limit of the kernel that reads them.
// The LDS limit of the stream-layout traversal pull (a block's values and
// its chunk's position table).
hipError_t stream_pull_setup() {
  static const hipError_t attr = [] {
    const int lds = gcx::lds_budget(gcx::kLdsMaxWidth);
    hipError_t e = hipSuccess;
    for (const void* k : {reinterpret_cast<const void*>(&k_sssp_tocab_lds<kW32>),
                          reinterpret_cast<const void*>(&k_sssp_tocab_lds<kW8>),
                          reinterpret_cast<const void*>(&k_sssp_tocab_lds<kWNone>)})
      if (e == hipSuccess) e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    return e;
  }();
  return attr;
}

hipError_t stream_weights(gc_tocab t, hipStream_t s) {
  GC_HIP_TRY(stream_pull_setup());
  if (t->w_pad || t->w8) return hipSuccess;
  if (!t->w) return hipErrorInvalidValue;
  // one byte per weight when every weight fits (checked once, on the device)
  int32_t* flag = g_range_flag();
  if (!flag) return hipErrorOutOfMemory;
  GC_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
  if (t->m > 0) k_weight_range<<<grid_for(t->m, kThreads), kThreads, 0, s>>>(t->w, t->m, flag);
  GC_HIP_TRY(hipGetLastError());
  int32_t wide = 0;
  GC_HIP_TRY(hipMemcpyAsync(&wide, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GC_HIP_TRY(hipStreamSynchronize(s));
  if (!wide) {
    t->w8 = static_cast<uint8_t*>(gcx::dev_alloc(static_cast<size_t>(t->m_pad), s));
    if (!t->w8) return hipErrorOutOfMemory;
    t->bytes += t->m_pad;
    k_weight_bytes<<<grid_for(t->m_pad, kThreads), kThreads, 0, s>>>(t->w, t->m, t->m_pad, t->w8);
    return hipGetLastError();
  }
  t->w_pad = static_cast<int32_t*>(gcx::dev_alloc(sizeof(int32_t) * static_cast<size_t>(t->m_pad), s));
  if (!t->w_pad) return hipErrorOutOfMemory;
  t->bytes += static_cast<int64_t>(sizeof(int32_t)) * t->m_pad;
  if (t->m > 0) GC_HIP_TRY(hipMemcpyAsync(t->w_pad, t->w, sizeof(int32_t) * t->m, hipMemcpyDeviceToDevice, s));
  return hipMemsetAsync(t->w_pad + t->m, 0, sizeof(int32_t) * (t->m_pad - t->m), s);
}

// Per-level bookkeeping: reads the next frontier's size and out-arc count,
// clears the old frontier's status bytes, and swaps the buffers.
struct Frontier {
  gc_graph g;
  hipStream_t s;
  int cur = 0;
  int32_t n_f = 1;
  int64_t m_f = 0;
  int64_t m_f_in = 0;  // in-arcs of the frontier when count_in (the source's are not counted)
  bool count_in = false;
  uint32_t* front() { return cur == 0 ? g->front : g->next; }
  uint32_t* next() { return cur == 0 ? g->next : g->front; }
  int32_t* queue() { return g->queue[cur]; }
  int32_t* queue_next() { return g->queue[cur ^ 1]; }

  hipError_t begin_level() {
    k_level_begin<<<1, kWave, 0, s>>>(g->stats);
    return hipGetLastError();
  }

  // Device time of the level just ended (its relaxation kernels), in ms,
  // from the clock stamps in the host mirror.
  double level_ms() const {
    const uint64_t t0 = *reinterpret_cast<const uint64_t*>(g->stats_host + gcx::kStatT0);
    const uint64_t t1 = *reinterpret_cast<const uint64_t*>(g->stats_host + gcx::kStatT1);
    return t1 > t0 ? static_cast<double>(t1 - t0) / g->clock_khz : 0.0;
  }

  // Ends a level: counts the next frontier's out-arcs, queues the learned
  // scheduler's decision for the next level when `decide` is given (read
  // back with the counters, so it costs no synchronisation of its own),
  // and reads the counters.
  hipError_t end_level(bool* overflow, gc_sched decide = nullptr, int32_t next_level = 0,
                       LevelDecide dec = LevelDecide()) {
    size_t lds = 0;
    if (decide) {
      lds = level_decide_lds(gcx::sched_actions(decide));
      dec.params = gcx::sched_params(decide);
      dec.frange = gcx::sched_range(decide);
      dec.K = gcx::sched_actions(decide);
      dec.n = g->n;
      dec.m = g->m;
      dec.level = next_level;
      dec.prior_arcs = m_f;
      dec.clock_khz = g->clock_khz;
    }
    k_queue_degree<<<1024, kThreads, 0, s>>>(queue_next(), g->stats + kQLen, g->rowptr, count_in ? g->t_rowptr : nullptr,
                                            g->stats);
    if (decide) k_level_decide<<<1, kThreads, lds, s>>>(g->stats, dec);
    GC_HIP_TRY(hipGetLastError());
    GC_HIP_TRY(hipMemcpyAsync(g->stats_host, g->stats, sizeof(int32_t) * gcx::kStatSlots, hipMemcpyDeviceToHost, s));
    if (n_f > 0) {
      // the old frontier's bits: through its queue, or, for a frontier of at
      // least one vertex per 16 words (one per 64-byte line), every word
      const int64_t words = (static_cast<int64_t>(g->n) + 31) / 32;
      if (16 * static_cast<int64_t>(n_f) >= words)
        k_fill_i32<<<grid_for(words, kThreads), kThreads, 0, s>>>(reinterpret_cast<int32_t*>(front()), words, 0);
      else
        k_clear_front<<<grid_for(n_f, kThreads), kThreads, 0, s>>>(front(), queue(), n_f);
    }
    GC_HIP_TRY(hipGetLastError());
    GC_HIP_TRY(hipStreamSynchronize(s));
    n_f = g->stats_host[kQLen];
    m_f = static_cast<int64_t>(static_cast<uint32_t>(g->stats_host[kDegLo])) |
          (static_cast<int64_t>(g->stats_host[kDegLo + 1]) << 32);
    m_f_in = static_cast<int64_t>(static_cast<uint32_t>(g->stats_host[gcx::kStatInDegLo])) |
             (static_cast<int64_t>(g->stats_host[gcx::kStatInDegLo + 1]) << 32);
    if (overflow && g->stats_host[kOverflow]) *overflow = true;
    cur ^= 1;
    return hipSuccess;
  }
};

hipError_t init_state(gc_graph g, int32_t* value, int32_t source, bool bfs, hipStream_t s) {
  const int32_t n = g->n;
  k_fill_i32<<<grid_for(n, kThreads), kThreads, 0, s>>>(value, n, kInf);
  const int64_t words = (static_cast<int64_t>(n) + 31) / 32;
  k_fill_i32<<<grid_for(words, kThreads), kThreads, 0, s>>>(reinterpret_cast<int32_t*>(g->front), words, 0);
  k_fill_i32<<<grid_for(words, kThreads), kThreads, 0, s>>>(reinterpret_cast<int32_t*>(g->next), words, 0);
  k_fill_i32<<<grid_for(words, kThreads), kThreads, 0, s>>>(reinterpret_cast<int32_t*>(g->visited), words, 0);
  if (!bfs) k_fill_i32<<<grid_for(n, kThreads), kThreads, 0, s>>>(g->mark, n, -1);
  k_set_source<<<1, 1, 0, s>>>(source, value, g->front, g->queue[0], bfs ? g->visited : nullptr);
  return hipGetLastError();
}

// Arc-balanced push of one level with relaxation r (see arc_balanced).
template <class Relax>
hipError_t push_arcs(gc_graph g, Frontier& f, Relax r, hipStream_t s) {
  k_order_degree<<<grid_for(f.n_f, kThreads), kThreads, 0, s>>>(f.queue(), f.n_f, g->rowptr, g->arc_deg);
  GC_HIP_TRY(hipGetLastError());
  GC_HIP_TRY(gcx::scan_exclusive(g->arc_deg, g->arc_pre, f.n_f, s));
  const int64_t pieces = (f.m_f + kPushArcs - 1) / kPushArcs;
  k_push_arcs<<<grid_for(pieces, kThreads), kThreads, 0, s>>>(f.queue(), g->arc_pre, f.n_f, g->rowptr, g->colidx, r,
                                                               f.queue_next(), g->stats);
  return hipGetLastError();
}

// The vertex-parallel push kernels balance the arcs of each work-group's
// kThreads vertices across its threads, so only the spread between
// work-groups is left: on a graph whose out-degrees are all small a
// frontier takes one launch instead of the five of the arc-balanced form
// (degree order, scan, push), up to frontiers large enough for launches
// not to matter.
constexpr int32_t kBlockPushDegree = 64;
constexpr int64_t kBlockPushArcs = int64_t{1} << 20;

bool arc_balanced(const gc_graph_s* g, const Frontier& f) {
  return f.m_f > kThreads * kPushArcs && (g->max_out_deg > kBlockPushDegree || f.m_f > kBlockPushArcs);
}

// Enqueues one level (BFS depth `level` -> level+1, or SSSP round `level`)
// in the given mode; t is the partition used by a TOCAB level.
hipError_t run_level(gc_graph g, Frontier& f, bool bfs, int32_t* value, int32_t level, Mode mode, gc_tocab t,
                     hipStream_t s) {
  const int32_t n = g->n;
  if (bfs) {
    if (mode == Mode::kPush && arc_balanced(g, f)) {
      ProfScope prof("bfs_push", s);
      GC_HIP_TRY(push_arcs(g, f, BfsRelax{value, level, f.next(), g->visited}, s));
    } else if (mode == Mode::kPush) {
      ProfScope prof("bfs_push", s);
      k_bfs_push<<<grid_for(f.n_f, kThreads), kThreads, 0, s>>>(f.queue(), f.n_f, g->rowptr, g->colidx, value,
                                                                 level, f.next(), g->visited, f.queue_next(),
                                                                 g->stats);
    } else if (mode == Mode::kPull) {
      ProfScope prof("bfs_pull", s);
      k_bfs_pull<<<grid_for(n, kThreads), kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, n, f.front(), value, level,
                                                             f.next(), g->visited, f.queue_next(), g->stats);
    } else if (t->col16) {
      // stream layout: the block's frontier bits (as 0 / INT32_MAX) in LDS,
      // per-(row, block) minima stored range-major (0: an in-neighbour of
      // the row is in the frontier), merged as one stream per range
      GC_HIP_TRY(stream_pull_setup());
      {
        ProfScope prof("bfs_tocab", s);
        const size_t lds = sizeof(int32_t) * (static_cast<size_t>(t->W) + 2 * (t->seg_max + kSeekPad));
        if (t->n_chunks > 0)
          k_sssp_tocab_lds<kWNone><<<t->n_chunks, kLdsRowThreads, lds, s>>>(
              t->row_ptr, t->col16, t->heads, nullptr, t->chunk_beg, t->chunk_end, t->chunk_blk, t->chunk_j0,
              t->chunk_ns, t->seg, t->R, t->log2W, n, f.front(), nullptr, t->pmin, pmin_bytes(t), g->stats);
      }
      ProfScope prof("bfs_merge", s);
      GC_HIP_TRY((launch_by_k<BfsMergeStream>(t->k, t->R, s, static_cast<const int32_t*>(t->rstart),
                                              static_cast<const uint16_t*>(t->id16s),
                                              static_cast<const int32_t*>(t->pmin), t->R, n, value, f.next(),
                                              f.queue_next(), g->stats, level, g->visited)));
    } else {
      uint8_t* flag = reinterpret_cast<uint8_t*>(t->pmin);
      {
        ProfScope prof("bfs_tocab", s);
        k_bfs_tocab<<<row_grid(t->P), kThreads, 0, s>>>(t->row_ptr, t->col, t->id_map, t->P, g->visited,
                                                                   f.front(), flag);
      }
      ProfScope prof("bfs_merge", s);
      GC_HIP_TRY((launch_by_k<BfsMerge>(t->k, t->R, s, static_cast<const int32_t*>(t->range_ptr), t->B,
                                        static_cast<const uint16_t*>(t->id16),
                                        static_cast<const uint8_t*>(flag), n, value, level, f.next(), g->visited,
                                        f.queue_next(), g->stats)));
    }
  } else {
    if (mode == Mode::kPush && arc_balanced(g, f)) {
      ProfScope prof("sssp_push", s);
      GC_HIP_TRY(push_arcs(g, f, SsspRelax{g->w, value, level, g->mark, f.next(), g->stats}, s));
    } else if (mode == Mode::kPush) {
      ProfScope prof("sssp_push", s);
      k_sssp_push<<<grid_for(f.n_f, kThreads), kThreads, 0, s>>>(f.queue(), f.n_f, g->rowptr, g->colidx, g->w,
                                                                  value, level, g->mark, f.next(), f.queue_next(),
                                                                  g->stats);
    } else if (mode == Mode::kPull) {
      ProfScope prof("sssp_pull", s);
      k_sssp_pull<<<grid_for(n, kThreads), kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, g->t_w, n, f.front(), value,
                                                              f.next(), f.queue_next(), g->stats);
    } else {
      if (t->col16) {  // stream layout: the block's distances in LDS, partial minima range-major
        GC_HIP_TRY(stream_weights(t, s));
        {
          ProfScope prof("sssp_tocab", s);
          const size_t lds = sizeof(int32_t) * (static_cast<size_t>(t->W) + 2 * (t->seg_max + kSeekPad));
          if (t->n_chunks > 0 && t->w8)
            k_sssp_tocab_lds<kW8><<<t->n_chunks, kLdsRowThreads, lds, s>>>(
                t->row_ptr, t->col16, t->heads, t->w8, t->chunk_beg, t->chunk_end, t->chunk_blk, t->chunk_j0,
                t->chunk_ns, t->seg, t->R, t->log2W, n, f.front(), value, t->pmin, pmin_bytes(t), g->stats);
          else if (t->n_chunks > 0)
            k_sssp_tocab_lds<kW32><<<t->n_chunks, kLdsRowThreads, lds, s>>>(
                t->row_ptr, t->col16, t->heads, t->w_pad, t->chunk_beg, t->chunk_end, t->chunk_blk, t->chunk_j0,
                t->chunk_ns, t->seg, t->R, t->log2W, n, f.front(), value, t->pmin, pmin_bytes(t), g->stats);
        }
        ProfScope prof("sssp_merge", s);
        GC_HIP_TRY((launch_by_k<SsspMergeStream>(t->k, t->R, s, static_cast<const int32_t*>(t->rstart),
                                                 static_cast<const uint16_t*>(t->id16s),
                                                 static_cast<const int32_t*>(t->pmin), t->R, n, value, f.next(),
                                                 f.queue_next(), g->stats, level, g->visited)));
        return hipGetLastError();
      } else {
        ProfScope prof("sssp_tocab", s);
        k_sssp_tocab<<<row_grid(t->P), kThreads, 0, s>>>(t->row_ptr, t->col, t->w, t->P, f.front(), value,
                                                         t->pmin, g->stats);
      }
      ProfScope prof("sssp_merge", s);
      GC_HIP_TRY((launch_by_k<SsspMerge>(t->k, t->R, s, static_cast<const int32_t*>(t->range_ptr), t->B,
                                         static_cast<const uint16_t*>(t->id16),
                                         static_cast<const int32_t*>(t->pmin), n, value, f.next(), f.queue_next(),
                                         g->stats)));
    }
  }
  return hipGetLastError();
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int64_t source_degree(gc_graph g, int32_t source, hipStream_t s, hipError_t* e) {
  int32_t rp[3] = {0, 0, 0};
  *e = hipMemcpyAsync(rp, g->rowptr + source, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (*e == hipSuccess && g->max_out_deg < 0) {
    // once per graph: its largest out-degree (arc_balanced), through the
    // first word of the push's degree scratch
    k_fill_i32<<<1, kThreads, 0, s>>>(g->arc_deg, 1, 0);
    k_max_out_degree<<<std::min<int64_t>(grid_for(g->n, kThreads), 1024), kThreads, 0, s>>>(g->rowptr, g->n,
                                                                                           g->arc_deg);
    *e = hipGetLastError();
    if (*e == hipSuccess) *e = hipMemcpyAsync(rp + 2, g->arc_deg, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (*e == hipSuccess) *e = hipStreamSynchronize(s);
    if (*e == hipSuccess) g->max_out_deg = rp[2];
    return rp[1] - rp[0];
  }
  if (*e == hipSuccess) *e = hipStreamSynchronize(s);
  return rp[1] - rp[0];
}

// Two HIP events released on scope exit.
struct EventPair {
  hipEvent_t e[2] = {nullptr, nullptr};
  hipError_t create() {
    GC_HIP_TRY(hipEventCreate(&e[0]));
    return hipEventCreate(&e[1]);
  }
  ~EventPair() {
    for (hipEvent_t x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

// Action k of the learned scheduler: 0 push, 1 plain pull, 2 + i TOCAB pull
// over the i-th attached partition.
void action_mode(int32_t a, gc_tocab* parts, Mode* mode, gc_tocab* t) {
  *t = nullptr;
  if (a == 0) *mode = Mode::kPush;
  else if (a == 1) *mode = Mode::kPull;
  else {
    *mode = Mode::kTocab;
    *t = parts[a - 2];
  }
}

int32_t mode_action(Mode m) { return m == Mode::kPush ? 0 : (m == Mode::kPull ? 1 : 2); }

// One forward BC level (depth `level` -> level+1): depth, sigma and the next
// frontier, in the given mode.
hipError_t run_bc_level(gc_graph g, Frontier& f, int32_t level, Mode mode, gc_tocab t, hipStream_t s) {
  const int32_t n = g->n;
  if (mode == Mode::kPush && arc_balanced(g, f)) {
    ProfScope prof("bc_push", s);
    GC_HIP_TRY(push_arcs(g, f, BcRelax{g->bc_depth, level, g->bc_sigma, f.next(), g->visited}, s));
  } else if (mode == Mode::kPush) {
    ProfScope prof("bc_push", s);
    k_bc_push<<<grid_for(f.n_f, kThreads), kThreads, 0, s>>>(f.queue(), f.n_f, g->rowptr, g->colidx, g->bc_depth,
                                                              level, g->bc_sigma, f.next(), g->visited,
                                                              f.queue_next(), g->stats);
  } else if (mode == Mode::kPull) {
    ProfScope prof("bc_pull", s);
    k_bc_pull<<<grid_for(n, kThreads), kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, n, f.front(), g->bc_depth, level,
                                                          g->bc_sigma, f.next(), g->visited, f.queue_next(),
                                                          g->stats);
  } else {
    {
      ProfScope prof("bc_tocab", s);
      k_bc_tocab<<<row_grid(t->P), kThreads, 0, s>>>(t->row_ptr, t->col, t->id_map, t->P, g->visited,
                                                                f.front(), g->bc_sigma, t->bc_part);
    }
    ProfScope prof("bc_merge", s);
    GC_HIP_TRY((launch_by_k<BcMerge>(t->k, t->R, s, static_cast<const int32_t*>(t->range_ptr), t->B,
                                     static_cast<const uint16_t*>(t->id16), static_cast<const double*>(t->bc_part),
                                     n, g->bc_depth, level, g->bc_sigma, f.next(), g->visited, f.queue_next(),
                                     g->stats)));
  }
  return hipGetLastError();
}

}  // namespace

namespace gcx {

void sched_features(int64_t n, int64_t m, int64_t n_f, int64_t m_f, int32_t level, double prior_ms,
                    int64_t prior_arcs, float* f) {
  level_features(n, m, n_f, m_f, level, prior_ms, prior_arcs, f);
}

hipError_t traverse(gc_graph g, gc_tocab t, int32_t source, int32_t* value, int32_t* count, uint32_t policy,
                    hipStream_t s, bool bfs, bool* overflow) {
  const int32_t n = g->n;
  GC_HIP_TRY(init_state(g, value, source, bfs, s));
  Frontier f{g, s};
  hipError_t e;
  f.m_f = source_degree(g, source, s, &e);
  GC_HIP_TRY(e);
  int64_t m_u = g->m - f.m_f;
  int64_t m_u_in = g->m;  // in-arcs of the unvisited vertices (the source's own few left in)
  Heuristic h;
  int32_t level = 0;
  g->trace_action.clear();
  g->trace_ms.clear();
  if (overflow) *overflow = false;
  // Learned policy: the network's decision for every level after the first
  // is computed on the device from the level counters at the end of the
  // previous level and read back with them; the first level's from host
  // features. Its working-set fallback uses the attached partition nearest
  // the paper's 2^18 when the call gives none.
  const gc_sched net = sched_for(g, bfs ? 0 : 1);
  const bool learned = policy == GC_POLICY_LEARNED && net;
  const int32_t K = learned ? sched_actions(net) : 0;
  gc_tocab fall_t = t;
  int32_t fall_action = -1;  // action index of TOCAB over fall_t
  if (learned) {
    const int32_t np = static_cast<int32_t>(g->sched_parts.size());
    int32_t best = INT32_MAX;
    for (int32_t j = 0; j < np && 2 + j < K; ++j) {
      const int32_t d = std::abs(g->sched_parts[j]->log2W - 18);
      if (d < best) {
        best = d;
        fall_action = 2 + j;
      }
    }
    if (!t && fall_action >= 0) fall_t = g->sched_parts[fall_action - 2];
    if (t) fall_action = -1;  // the caller's partition is not among the network's actions
  }
  // the working-set rule's BFS arm over a stream-layout partition reads the
  // unvisited vertices' in-arcs
  f.count_in = bfs && (policy == GC_POLICY_HEURISTIC || policy == GC_POLICY_LEARNED) && fall_t != nullptr &&
               fall_t->col16 != nullptr && static_cast<double>(g->m) <= Heuristic::kBfsTocabDegree * n;
  std::vector<float> outs(static_cast<size_t>(std::max(K, 1)));
  while (f.n_f > 0) {
    if (!bfs && level > n) return hipErrorInvalidValue;  // cannot happen with positive weights
    // SSSP revisits vertices, so the unexplored-arc count of BFS does not
    // apply; the whole arc set stands in for it.
    const int64_t unexplored = bfs ? m_u : g->m;
    // the working-set rule's choice: the policy itself, the fallback of the
    // learned one, and the reference its decision is gated against
    Mode hmode;
    if (policy == GC_POLICY_PUSH) hmode = Mode::kPush;
    else if (policy == GC_POLICY_PULL) hmode = t ? Mode::kTocab : Mode::kPull;
    else
      hmode = h.pick(n, f.n_f, f.m_f, unexplored, fall_t != nullptr, bfs, g->m, m_u_in,
                     fall_t != nullptr && fall_t->col16 != nullptr);
    Mode mode = hmode;
    gc_tocab lt = fall_t;
    int32_t action = -1;
    if (learned) {
      int32_t a = -1;
      if (level == 0) {
        if (hmode != Mode::kPush) {
          float feats[GC_SCHED_INPUTS];
          sched_features(n, g->m, f.n_f, f.m_f, level, 0.0, 0, feats);
          GC_HIP_TRY(sched_decide(net, feats, s, &a, outs.data()));
        }
      } else {
        a = g->stats_host[gcx::kStatChoice];
        std::memcpy(outs.data(), g->stats_host + gcx::kStatOut, sizeof(float) * K);
      }
      if (a >= 0 && a < K && hmode != Mode::kPush) {
        // The rule keeps the direction (its push / pull switch is the
        // direction-optimising test, close to the best on every graph
        // measured); on a pull level the network picks the form: plain pull
        // or TOCAB pull over one of the attached widths, the rule's own form
        // kept unless the network predicts its pick faster by more than the
        // gate.
        a = 1;
        for (int32_t k = 2; k < K; ++k)
          if (outs[k] < outs[a]) a = k;
        const int32_t ha = hmode == Mode::kPull ? 1 : fall_action;
        if (ha >= 1 && ha < K && outs[ha] <= outs[a] + kLearnedGate) a = ha;
        action_mode(a, g->sched_parts.data(), &mode, &lt);
        action = a;
      }
    }
    if (action < 0) {
      mode = hmode;
      lt = mode == Mode::kTocab ? fall_t : t;
      action = mode_action(mode);
    }
    const double t0 = now_ms();
    GC_HIP_TRY(f.begin_level());
    GC_HIP_TRY(run_level(g, f, bfs, value, level, mode, lt, s));
    LevelDecide dec;
    if (learned) {
      dec.pulling = h.pulling;
      dec.sub_next = bfs;
      dec.unexplored = bfs ? m_u : g->m;
      dec.alpha = Heuristic::kAlpha;
      dec.beta = Heuristic::kBeta;
    }
    GC_HIP_TRY(f.end_level(overflow, learned ? net : nullptr, level + 1, dec));
    const double wall_ms = now_ms() - t0;
    g->trace_action.push_back(action);
    g->trace_ms.push_back(static_cast<float>(wall_ms));
    if (overflow && *overflow) break;
    if (bfs) {
      m_u -= f.m_f;
      m_u_in -= f.m_f_in;
    }
    ++level;
  }
  if (count) *count = level;
  return hipSuccess;
}

hipError_t bfs_run(gc_graph g, gc_tocab t, int32_t source, int32_t* depth, int32_t* levels, uint32_t policy,
                   hipStream_t s) {
  return traverse(g, t, source, depth, levels, policy, s, true, nullptr);
}

hipError_t sssp_run(gc_graph g, gc_tocab t, int32_t source, int32_t* dist, int32_t* rounds, uint32_t policy,
                    hipStream_t s, bool* overflow) {
  return traverse(g, t, source, dist, rounds, policy, s, false, overflow);
}

// Betweenness centrality from the given sources (Brandes): per source, the
// forward levels count shortest paths (push, pull or TOCAB pull per level,
// chosen as for BFS), then the backward steps accumulate the dependencies
// deepest level first into bc. The per-graph sigma / delta / depth arrays
// and the partition's FP64 partials are allocated by the first call.
hipError_t bc_run(gc_graph g, gc_tocab t, const int32_t* sources, int32_t n_src, double* bc, uint32_t policy,
                  hipStream_t s) {
  const int32_t n = g->n;
  if (!g->bc_sigma) {
    g->bc_sigma = static_cast<double*>(dev_alloc(sizeof(double) * n, s));
    g->bc_coef = static_cast<double*>(dev_alloc(sizeof(double) * 2 * static_cast<size_t>(n), s));
    g->bc_depth = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * n, s));
    g->bc_order = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * n, s));
    if (!g->bc_sigma || !g->bc_coef || !g->bc_depth || !g->bc_order) {
      for (void* p : {static_cast<void*>(g->bc_sigma), static_cast<void*>(g->bc_coef),
                      static_cast<void*>(g->bc_depth), static_cast<void*>(g->bc_order)})
        if (p) dev_free(p, s);
      g->bc_sigma = g->bc_coef = nullptr;
      g->bc_depth = g->bc_order = nullptr;
      return hipErrorOutOfMemory;
    }
  }
  if (t && !t->bc_part) {
    t->bc_part = static_cast<double*>(dev_alloc(sizeof(double) * std::max<int64_t>(t->P, 1), s));
    if (!t->bc_part) return hipErrorOutOfMemory;
  }
  g->trace_action.clear();
  g->trace_ms.clear();
  for (int32_t si = 0; si < n_src; ++si) {
    const int32_t src = sources[si];
    GC_HIP_TRY(init_state(g, g->bc_depth, src, true, s));
    k_fill_f64<<<grid_for(n, kThreads), kThreads, 0, s>>>(g->bc_sigma, n);
    k_fill_f64<<<grid_for(2 * static_cast<int64_t>(n), kThreads), kThreads, 0, s>>>(g->bc_coef,
                                                                                   2 * static_cast<int64_t>(n));
    k_set_sigma<<<1, 1, 0, s>>>(src, g->bc_sigma);
    GC_HIP_TRY(hipGetLastError());
    // order holds the vertices level by level (the source first); level d
    // occupies [lv_off[d], lv_off[d + 1])
    std::vector<int32_t> lv_off{0, 1};
    std::vector<int64_t> lv_arcs;  // out-arcs of each level's vertices
    GC_HIP_TRY(hipMemcpyAsync(g->bc_order, g->queue[0], sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    Frontier f{g, s};
    hipError_t e;
    f.m_f = source_degree(g, src, s, &e);
    GC_HIP_TRY(e);
    int64_t m_u = g->m - f.m_f;
    lv_arcs.push_back(f.m_f);
    Heuristic h;
    int32_t level = 0;
    while (f.n_f > 0) {
      Mode mode;
      if (policy == GC_POLICY_PUSH) mode = Mode::kPush;
      else if (policy == GC_POLICY_PULL) mode = t ? Mode::kTocab : Mode::kPull;
      else mode = h.pick(n, f.n_f, f.m_f, m_u, t != nullptr, true);
      const double t0 = now_ms();
      GC_HIP_TRY(f.begin_level());
      GC_HIP_TRY(run_bc_level(g, f, level, mode, t, s));
      GC_HIP_TRY(f.end_level(nullptr));
      g->trace_action.push_back(mode_action(mode));
      g->trace_ms.push_back(static_cast<float>(now_ms() - t0));
      if (f.n_f > 0) {
        GC_HIP_TRY(hipMemcpyAsync(g->bc_order + lv_off.back(), f.queue(), sizeof(int32_t) * f.n_f,
                                  hipMemcpyDeviceToDevice, s));
        lv_off.push_back(lv_off.back() + f.n_f);
        lv_arcs.push_back(f.m_f);
      }
      m_u -= f.m_f;
      ++level;
    }
    // depths run 0 .. level-1 (level = lv_off.size() - 1). Each step d runs
    // in the direction with fewer arcs: pull over the out-arcs of depth d
    // (arc_pre = exclusive scan of out-degrees along order) or push over
    // the in-arcs of depth d + 1 (pre_in, the same for in-degrees). The
    // deepest level's step only sets coef = 1 / sigma; the source (depth 0)
    // takes no share.
    ProfScope prof("bc_back", s);
    const int32_t reached = lv_off.back();
    Buf pre_in(sizeof(int32_t) * (static_cast<size_t>(reached) + 1), s);
    if (!pre_in.p) return hipErrorOutOfMemory;
    k_order_degree<<<grid_for(reached, kThreads), kThreads, 0, s>>>(g->bc_order, reached, g->rowptr, g->arc_deg);
    GC_HIP_TRY(hipGetLastError());
    GC_HIP_TRY(scan_exclusive(g->arc_deg, g->arc_pre, reached, s));
    k_order_degree<<<grid_for(reached, kThreads), kThreads, 0, s>>>(g->bc_order, reached, g->t_rowptr, g->arc_deg);
    GC_HIP_TRY(hipGetLastError());
    GC_HIP_TRY(scan_exclusive(g->arc_deg, pre_in.as<int32_t>(), reached, s));
    std::vector<int32_t> in_at(lv_off.size());  // in-arcs before each level's first vertex
    for (size_t k = 0; k < lv_off.size(); ++k)
      GC_HIP_TRY(hipMemcpyAsync(&in_at[k], pre_in.as<int32_t>() + lv_off[k], sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
    GC_HIP_TRY(hipStreamSynchronize(s));
    for (int32_t d = level - 1; d >= 1; --d) {
      const int32_t lo = lv_off[d], hi = lv_off[d + 1];
      double* coef_out = g->bc_coef + static_cast<size_t>(d & 1) * n;
      const double* coef_in = g->bc_coef + static_cast<size_t>((d + 1) & 1) * n;
      const int64_t out_arcs = lv_arcs[d];
      const int64_t in_next = d + 1 < level ? static_cast<int64_t>(in_at[d + 2]) - in_at[d + 1] : 0;
      if (d + 1 < level && in_next < out_arcs) {
        const int64_t pieces = (in_next + kBackArcs - 1) / kBackArcs;
        if (pieces > 0)
          k_bc_back_push<<<grid_for(pieces, kThreads), kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, g->bc_order,
                                                                         pre_in.as<int32_t>(), hi, lv_off[d + 2],
                                                                         g->bc_depth, d, coef_in, coef_out);
      } else if (d + 1 < level) {
        const int64_t pieces = (out_arcs + kBackArcs - 1) / kBackArcs;
        if (pieces > 0)
          k_bc_back_arcs<<<grid_for(pieces, kThreads), kThreads, 0, s>>>(g->rowptr, g->colidx, g->bc_order,
                                                                         g->arc_pre, lo, hi, coef_in, coef_out);
      }
      k_bc_finish<<<grid_for(hi - lo, kThreads), kThreads, 0, s>>>(g->bc_order + lo, hi - lo, g->bc_sigma, coef_out,
                                                                    bc);
    }
    GC_HIP_TRY(hipGetLastError());
  }
  return hipStreamSynchronize(s);
}

// Training data for the scheduler: at every level of a traversal from each
// source, the level is run once per action from the same state (snapshot
// and restore of the frontier state), each run timed with HIP events; the
// traversal then continues with the fastest action. One row per level:
// 6 features and K = 2 + n_parts times in ms.
hipError_t collect(gc_graph g, gc_tocab* parts, int32_t n_parts, bool bfs, const int32_t* sources, int32_t n_src,
                   float* features, float* times, int32_t max_rows, int32_t* rows, hipStream_t s) {
  const int32_t n = g->n;
  const int32_t K = 2 + n_parts;
  const size_t words = (static_cast<size_t>(n) + 31) / 32;
  Buf value(sizeof(int32_t) * n, s), sv(sizeof(int32_t) * n, s), sfront(sizeof(uint32_t) * words, s),
      snext(sizeof(uint32_t) * words, s),
      svis(sizeof(uint32_t) * words, s), smark(sizeof(int32_t) * n, s), squeue(sizeof(int32_t) * n, s);
  if (!value.p || !sv.p || !sfront.p || !snext.p || !svis.p || !smark.p || !squeue.p) return hipErrorOutOfMemory;
  hipEvent_t e0, e1;
  GC_HIP_TRY(hipEventCreate(&e0));
  GC_HIP_TRY(hipEventCreate(&e1));
  int32_t r = 0;
  hipError_t err = hipSuccess;
  for (int32_t si = 0; si < n_src && err == hipSuccess; ++si) {
    err = init_state(g, value.as<int32_t>(), sources[si], bfs, s);
    if (err != hipSuccess) break;
    Frontier f{g, s};
    f.m_f = source_degree(g, sources[si], s, &err);
    int32_t level = 0;
    double prior_ms = 0.0;  // device time of the previous level (its fastest action), from the clock stamps
    int64_t prior_arcs = 0;
    bool overflow = false;
    std::vector<double> stamp_ms(static_cast<size_t>(K));
    while (err == hipSuccess && f.n_f > 0 && r < max_rows && !overflow) {
      sched_features(n, g->m, f.n_f, f.m_f, level, prior_ms, prior_arcs,
                     features + static_cast<size_t>(r) * GC_SCHED_INPUTS);
      // snapshot the state this level starts from
      const hipMemcpyKind dd = hipMemcpyDeviceToDevice;
      err = hipMemcpyAsync(sv.p, value.p, sizeof(int32_t) * n, dd, s);
      if (err == hipSuccess) err = hipMemcpyAsync(sfront.p, f.front(), sizeof(uint32_t) * words, dd, s);
      if (err == hipSuccess) err = hipMemcpyAsync(snext.p, f.next(), sizeof(uint32_t) * words, dd, s);
      if (err == hipSuccess) err = hipMemcpyAsync(svis.p, g->visited, sizeof(uint32_t) * words, dd, s);
      if (err == hipSuccess && !bfs) err = hipMemcpyAsync(smark.p, g->mark, sizeof(int32_t) * n, dd, s);
      if (err == hipSuccess) err = hipMemcpyAsync(squeue.p, f.queue(), sizeof(int32_t) * f.n_f, dd, s);
      const Frontier start = f;
      auto restore = [&]() -> hipError_t {
        f = start;
        GC_HIP_TRY(hipMemcpyAsync(value.p, sv.p, sizeof(int32_t) * n, dd, s));
        GC_HIP_TRY(hipMemcpyAsync(f.front(), sfront.p, sizeof(uint32_t) * words, dd, s));
        GC_HIP_TRY(hipMemcpyAsync(f.next(), snext.p, sizeof(uint32_t) * words, dd, s));
        GC_HIP_TRY(hipMemcpyAsync(g->visited, svis.p, sizeof(uint32_t) * words, dd, s));
        if (!bfs) GC_HIP_TRY(hipMemcpyAsync(g->mark, smark.p, sizeof(int32_t) * n, dd, s));
        return hipMemcpyAsync(f.queue(), squeue.p, sizeof(int32_t) * f.n_f, dd, s);
      };
      float* row_t = times + static_cast<size_t>(r) * K;
      int32_t best = 0;
      for (int32_t a = 0; a < K && err == hipSuccess; ++a) {
        Mode mode;
        gc_tocab lt;
        action_mode(a, parts, &mode, &lt);
        if (a > 0) err = restore();
        if (err == hipSuccess) err = f.begin_level();
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        if (err == hipSuccess) err = run_level(g, f, bfs, value.as<int32_t>(), level, mode, lt, s);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = f.end_level(&overflow);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        row_t[a] = ms;
        stamp_ms[a] = f.level_ms();
        if (ms < row_t[best]) best = a;
      }
      if (err != hipSuccess) break;
      // continue the traversal with the fastest action
      if (best != K - 1) {
        Mode mode;
        gc_tocab lt;
        action_mode(best, parts, &mode, &lt);
        err = restore();
        if (err == hipSuccess) err = f.begin_level();
        if (err == hipSuccess) err = run_level(g, f, bfs, value.as<int32_t>(), level, mode, lt, s);
        if (err == hipSuccess) err = f.end_level(&overflow);
      }
      prior_ms = stamp_ms[best];
      prior_arcs = start.m_f;
      ++r;
      ++level;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *rows = r;
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  return err;
}

}  // namespace gcx
