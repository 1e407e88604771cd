// Figure 5 merge, the walk over every block's partial results of one vertex
// range by a work-group of NT threads, shared by the PageRank, SpMV, batched
// and BC merges (FP64 LDS sums) and the BFS / SSSP merges (OR / min).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gc_device.h"

namespace gcm {

using gcd::kWave;

constexpr int kFlatB = 1024;  // merges over at most this many blocks flatten their slices

// Walk of range j's entries: for every block s the local rows mapping into
// [j*K, (j+1)*K) form one contiguous slice of the per-row arrays (local ids
// ascend with global ids). visit(pos, value) is called once per entry with
// its position inside the range (id16) and its value. With B <= kFlatB the
// slices are walked as one flattened list so every lane keeps several
// independent loads in flight. The walk synchronises the work-group before
// its first visit and after its last, so LDS the visits update may be
// initialised right before the call.
template <bool kFlat, int NT, class T, class Visit>
__device__ __forceinline__ void merge_slices(const int32_t* __restrict__ range_ptr, int32_t B,
                                             const uint16_t* __restrict__ id16, const T* __restrict__ partial,
                                             int32_t j, Visit&& visit) {
  __shared__ int32_t seg_lo[kFlat ? kFlatB : 1];
  __shared__ int32_t seg_pre[kFlat ? kFlatB + 1 : 1];
  const int32_t* lo = range_ptr + static_cast<int64_t>(j) * B;
  const int32_t* hi = lo + B;
  if (kFlat) {
    // slice starts and an exclusive scan of slice lengths (one pass, B <= kFlatB)
    __shared__ int32_t wave_tot[NT / kWave];
    constexpr int kItems = kFlatB / NT;
    int32_t len[kItems];
    int32_t mine = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int32_t s = threadIdx.x * kItems + k;
      len[k] = 0;
      if (s < B) {
        const int32_t a = lo[s];
        seg_lo[s] = a;
        len[k] = hi[s] - a;
      }
      mine += len[k];
    }
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int32_t incl = gcd::wave_incl_scan(mine);
    if (lane == kWave - 1) wave_tot[wid] = incl;
    __syncthreads();
    int32_t off = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) off += (w < wid) ? wave_tot[w] : 0;
    int32_t run = off + incl - mine;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int32_t s = threadIdx.x * kItems + k;
      if (s < B) seg_pre[s] = run;
      run += len[k];
    }
    if (threadIdx.x == NT - 1) seg_pre[B] = run;
    __syncthreads();
    const int32_t total = seg_pre[B];
    constexpr int kUnroll = 8;
    int32_t s = 0;
    for (int32_t f0 = threadIdx.x; f0 < total; f0 += NT * kUnroll) {
      // flat positions past the end reuse the first (valid) local row and are masked
      int32_t l[kUnroll];
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const int32_t f = f0 + k * NT;
        if (f < total) {
          while (seg_pre[s + 1] <= f) ++s;
          l[k] = seg_lo[s] + (f - seg_pre[s]);
        } else {
          l[k] = l[0];
        }
      }
      uint16_t v[kUnroll];
      T p[kUnroll];
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        v[k] = gcd::ld_stream(id16 + l[k]);
        p[k] = gcd::ld_stream(partial + l[k]);
      }
#pragma unroll
      for (int k = 0; k < kUnroll; ++k)
        if (f0 + k * NT < total) visit(static_cast<uint32_t>(v[k]), p[k]);
    }
  } else {
    __syncthreads();
    for (int32_t s = 0; s < B; ++s) {
      const int32_t a = lo[s], z = hi[s];
      for (int32_t l = a + threadIdx.x; l < z; l += NT)
        visit(static_cast<uint32_t>(gcd::ld_stream(id16 + l)), gcd::ld_stream(partial + l));
    }
  }
  __syncthreads();
}

// FP64 sums of range j's partial results (float or double) into acc[K] in
// LDS; zero partials are skipped.
template <int K, bool kFlat, int NT, class T>
__device__ __forceinline__ void merge_accumulate(const int32_t* __restrict__ range_ptr, int32_t B,
                                                 const uint16_t* __restrict__ id16, const T* __restrict__ partial,
                                                 int32_t j, double* acc) {
  for (int i = threadIdx.x; i < K; i += NT) acc[i] = 0.0;
  merge_slices<kFlat, NT>(range_ptr, B, id16, partial, j, [&](uint32_t v, T p) {
    if (p != T(0)) atomicAdd(&acc[v], static_cast<double>(p));
  });
}

}  // namespace gcm
