// Device code shared by the PageRank kernels and the batched persistent
// kernel: the fused per-vertex update, pull tiles and the merge of the
// partial sums of one vertex range.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gc_device.h"
#include "gc_merge.h"

namespace {


using gcd::kWave;

constexpr int kThreads = 256;

constexpr int kTileArcs = 2048;                  // arcs per pull tile (tile table granularity)
constexpr int kStageCap = 4096;                  // arcs a tile may stage in LDS
constexpr int kPerThread = kStageCap / kThreads;  // staged arcs per thread
constexpr int kFlatB = gcm::kFlatB;              // merges over at most this many blocks flatten their slices

static_assert(kTileArcs <= kStageCap, "a tile's short rows must fit the stage");

struct Update {
  double base;      // (1 - d) / n
  double d;         // damping
  double inv_n;     // 1 / n, applied to D in uniform mode (0 in leak mode)
  const double* dtotal_in;
  double* dpart;    // one dangling partial per work-group of the update kernel
  const int32_t* rowptr;  // out-arc CSR: outdeg(v) = rowptr[v+1] - rowptr[v]
  float* contrib;         // written for the next iteration
  float* rank_out;        // written on the last iteration only (else null)
  const float* rank_prev = nullptr;  // convergence mode: the previous iterate
  double* lpart = nullptr;           // convergence mode: L1 change per work-group
  int32_t n;
};

// r'[v] from the neighbour sum; writes c'[v] (and r'[v] on the last pass),
// returns r'[v] when v has no out-arcs (its share of the next D), else 0.
// In convergence mode also adds |r'[v] - r[v]| (FP64 over the FP32
// iterates) to dl.
// The new contribution is also returned in cv (u.contrib may be null when
// the caller keeps it elsewhere). update_vertex_loaded takes v's out-degree
// and previous rank (read only in convergence mode) from the caller.
__device__ __forceinline__ double update_vertex_loaded(const Update& u, int32_t v, double sum, double D, double& dl,
                                                       float& cv, int32_t deg, float prev) {
  const double r = u.base + u.d * (sum + D * u.inv_n);
  const float r32 = static_cast<float>(r);
  cv = deg ? static_cast<float>(static_cast<double>(r32) / deg) : 0.0f;
  if (u.contrib) u.contrib[v] = cv;
  if (u.rank_out) u.rank_out[v] = r32;
  if (u.rank_prev) dl += fabs(static_cast<double>(r32) - static_cast<double>(prev));
  return deg ? 0.0 : static_cast<double>(r32);
}

__device__ __forceinline__ double update_vertex(const Update& u, int32_t v, double sum, double D, double& dl,
                                                float& cv) {
  return update_vertex_loaded(u, v, sum, D, dl, cv, u.rowptr[v + 1] - u.rowptr[v], u.rank_prev ? u.rank_prev[v] : 0.0f);
}

__device__ __forceinline__ double update_vertex(const Update& u, int32_t v, double sum, double D, double& dl) {
  float cv;
  return update_vertex(u, v, sum, D, dl, cv);
}

__device__ __forceinline__ double update_vertex(const Update& u, int32_t v, double sum, double D) {
  double dl = 0.0;
  return update_vertex(u, v, sum, D, dl);
}

// Orders LDS accesses between the lanes of one wave.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Work-group sum of one double per thread (fixed reduction tree), returned
// to every thread.
template <int NT = kThreads>
__device__ __forceinline__ double wg_sum(double x) {
  __shared__ double part[NT / kWave];
  x = gcd::wave_sum(x);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) t += part[w];
  __syncthreads();
  return t;
}

template <int NT = kThreads>
__device__ __forceinline__ void publish_dangling(const Update& u, double mine) {
  const double t = wg_sum<NT>(mine);
  if (threadIdx.x == 0) u.dpart[blockIdx.x] = t;
}

// publish_dangling plus, in convergence mode, the work-group's L1 change.
template <int NT = kThreads>
__device__ __forceinline__ void publish_update(const Update& u, double mine, double dl) {
  publish_dangling<NT>(u, mine);
  if (u.lpart) {  // uniform
    const double t = wg_sum<NT>(dl);
    if (threadIdx.x == 0) u.lpart[blockIdx.x] = t;
  }
}

// The value an arc contributes to its row's sum, given its index i in the
// arc array and the gathered source value x: x itself (PageRank, where the
// source value is already c[u] = r[u] / outdeg(u)), or x times the arc's
// value (SpMV: FP32 values stored as their bits, or integer weights).
struct PlainArc {
  __device__ __forceinline__ float operator()(int32_t, float x) const { return x; }
};
struct ValuedArc {
  const int32_t* val;  // null: every value is 1
  bool f32;            // val holds FP32 bit patterns (else integers)
  __device__ __forceinline__ float operator()(int32_t i, float x) const {
    if (!val) return x;
    const int32_t b = gcd::ld_stream(val + i);
    return x * (f32 ? __int_as_float(b) : static_cast<float>(b));
  }
};

// Gathers arc(i, c[col[i]]) for i = a0 + [0, len) (len <= kStageCap) into
// LDS: every lane first issues its column loads (coalesced across the
// work-group, streamed past the cache), then the gathers, so all loads of a
// tile are in flight together. Indices past the end are clamped to the last
// arc instead of branched around, which keeps the loads free of control flow
// (a branch per load would make each one wait for the previous).
template <class Arc = PlainArc>
__device__ __forceinline__ void stage_gather(const int32_t* __restrict__ col, const float* __restrict__ c,
                                             int32_t a0, int32_t len, float* vals, Arc arc = Arc()) {
  if (len <= 0) return;
  int32_t idx[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int32_t i = min(static_cast<int32_t>(threadIdx.x) + k * kThreads, len - 1);
    idx[k] = gcd::ld_stream(col + a0 + i);
  }
  float x[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) x[k] = c[idx[k]];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int32_t i = threadIdx.x + k * kThreads;
    if (i < len) vals[i] = arc(a0 + i, x[k]);
  }
}

// Sum of arc(i, c[col[i]]) over arcs [b, e) (b < e) by the whole
// work-group (hub rows).
template <class Arc = PlainArc>
__device__ double wg_row_sum(const int32_t* __restrict__ col, const float* __restrict__ c, int32_t b, int32_t e,
                             Arc arc = Arc()) {
  double s = 0.0;
  for (int32_t base = b; base < e; base += kStageCap) {
    int32_t idx[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k)
      idx[k] = gcd::ld_stream(col + min(base + static_cast<int32_t>(threadIdx.x) + k * kThreads, e - 1));
    float x[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) x[k] = c[idx[k]];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int32_t i = base + static_cast<int32_t>(threadIdx.x) + k * kThreads;
      if (i < e) s += static_cast<double>(arc(i, x[k]));
    }
  }
  return wg_sum(s);
}

// One pull tile (coarse-grained load balancing of the pull direction,
// Section 3.2): the tile owns the rows whose first arc lies in its
// kTileArcs-wide slice of the arc array. Their arcs are gathered into LDS
// together; then each thread sums whole short rows serially in FP64, and a
// last row too long for the stage is summed by the whole work-group. No
// atomics. emit(row, sum) is called once per owned row.
template <class Emit, class Arc = PlainArc>
__device__ __forceinline__ void pull_tile(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                          const float* __restrict__ c, int32_t r0, int32_t r1, float* vals,
                                          Emit&& emit, Arc arc = Arc()) {
  const int32_t a0 = row_ptr[r0];
  const int32_t last_b = row_ptr[r1 - 1];
  const int32_t a_end = row_ptr[r1];
  const bool long_last = (a_end - a0) > kStageCap;
  stage_gather(col, c, a0, (long_last ? last_b : a_end) - a0, vals, arc);
  __syncthreads();
  const int32_t r_short_end = long_last ? r1 - 1 : r1;
  for (int32_t r = r0 + threadIdx.x; r < r_short_end; r += kThreads) {
    const int32_t b = row_ptr[r] - a0, e = row_ptr[r + 1] - a0;
    double s = 0.0;
    for (int32_t i = b; i < e; ++i) s += static_cast<double>(vals[i]);
    emit(r, s);
  }
  if (long_last) {
    const double s = wg_row_sum(col, c, last_b, a_end, arc);
    if (threadIdx.x == 0) emit(r1 - 1, s);
  }
}

// Figure 5 merge, accumulation part, for vertex range j (FP64 LDS sums).
template <int K, bool kFlat, class T>
__device__ __forceinline__ void merge_accumulate(const int32_t* __restrict__ range_ptr, int32_t B,
                                                 const uint16_t* __restrict__ id16, const T* __restrict__ partial,
                                                 int32_t j, double* acc) {
  gcm::merge_accumulate<K, kFlat, kThreads>(range_ptr, B, id16, partial, j, acc);
}

}  // namespace
