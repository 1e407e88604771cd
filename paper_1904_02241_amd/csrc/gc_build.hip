// Graph construction on the GPU: exclusive scan, CSR transpose with sorted
// rows, and the TOCAB static partition (Section 3.1, preprocessing phase).
// Runs once per graph / per block width; timed apart from the iterations.

#include <algorithm>
#include <climits>
#include <vector>

#include "gc_device.h"
#include "gc_internal.h"

namespace {

using gcd::kWave;

// ---------------------------------------------------------------------------
// Exclusive scan (reduce tiles -> scan tile totals -> rescan tiles).

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// Work-group exclusive scan of one int per thread; *total gets the sum.
__device__ int wg_excl_scan(int v, int* total) {
  __shared__ int wave_tot[kScanThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int incl = gcd::wave_incl_scan(v);
  if (lane == kWave - 1) wave_tot[wid] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    const int x = wave_tot[w];
    off += (w < wid) ? x : 0;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* __restrict__ in, int64_t n,
                                                              int32_t* __restrict__ tile_sum) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i * kScanThreads + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  int tot;
  wg_excl_scan(s, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// One work-group scans all tile sums in place (exclusive).
__global__ __launch_bounds__(kScanThreads) void k_scan_top(int32_t* __restrict__ tile_sum, int64_t nt) {
  int carry = 0;
  for (int64_t base = 0; base < nt; base += kScanTile) {
    int vals[kScanItems];
    int local = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      const int64_t idx = base + static_cast<int64_t>(threadIdx.x) * kScanItems + i;
      vals[i] = idx < nt ? tile_sum[idx] : 0;
      local += vals[i];
    }
    int tot;
    int run = carry + wg_excl_scan(local, &tot);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      const int64_t idx = base + static_cast<int64_t>(threadIdx.x) * kScanItems + i;
      if (idx < nt) tile_sum[idx] = run;
      run += vals[i];
    }
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* __restrict__ in,
                                                             int32_t* __restrict__ out, int64_t n,
                                                             const int32_t* __restrict__ tile_off) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile +
                       static_cast<int64_t>(threadIdx.x) * kScanItems;
  int vals[kScanItems];
  int local = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    vals[i] = idx < n ? in[idx] : 0;
    local += vals[i];
  }
  int tot;
  int run = tile_off[blockIdx.x] + wg_excl_scan(local, &tot);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    if (idx < n) out[idx] = run;
    if (idx == n - 1) out[n] = run + vals[i];
    run += vals[i];
  }
}

// ---------------------------------------------------------------------------
// Transpose: in-degree count, scatter of (source, weight) keys, per-row sort.

__global__ void k_indegree(const int32_t* __restrict__ colidx, int64_t m, int32_t* __restrict__ cnt) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < m; e += stride)
    atomicAdd(&cnt[colidx[e]], 1);
}

constexpr int kScatterTile = 4096;

// Row owning arc e: the last r with rowptr[r] <= e, searched in [lo, hi].
__device__ __forceinline__ int32_t owner_row(const int32_t* rowptr, int32_t lo, int32_t hi, int64_t e) {
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo + 1) >> 1);
    if (rowptr[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ rowptr, int32_t n,
                                                 const int32_t* __restrict__ colidx,
                                                 const int32_t* __restrict__ w, int64_t m,
                                                 int32_t* __restrict__ cursor, uint64_t* __restrict__ keys) {
  __shared__ int32_t r_lo, r_hi;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * kScatterTile;
  const int64_t e1 = min(e0 + kScatterTile, m);
  if (threadIdx.x == 0) {
    r_lo = owner_row(rowptr, 0, n, e0);
    r_hi = owner_row(rowptr, 0, n, e1 - 1);
  }
  __syncthreads();
  const int32_t lo = r_lo, hi = r_hi;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int32_t u = owner_row(rowptr, lo, hi, e);
    const int32_t v = colidx[e];
    const int32_t pos = atomicAdd(&cursor[v], 1);
    const uint32_t wv = w ? static_cast<uint32_t>(w[e]) : 0u;
    keys[pos] = (static_cast<uint64_t>(static_cast<uint32_t>(u)) << 32) | wv;
  }
}

constexpr int kSmallRow = 32;
constexpr int kMidRow = 4096;  // rows up to this length sort inside LDS

__device__ __forceinline__ void unpack_to(uint64_t key, int32_t* col, int32_t* w, int64_t pos) {
  col[pos] = static_cast<int32_t>(key >> 32);
  if (w) w[pos] = static_cast<int32_t>(key & 0xFFFFFFFFull);
}

// Rows of at most kSmallRow keys: insertion sort in place, then unpack.
// Longer rows are queued for the work-group sorters.
__global__ __launch_bounds__(256) void k_sort_small(const int32_t* __restrict__ t_rowptr, int32_t n,
                                                    uint64_t* __restrict__ keys, int32_t* __restrict__ t_col,
                                                    int32_t* __restrict__ t_w, int32_t* __restrict__ lists,
                                                    int32_t* __restrict__ list_len) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t b = t_rowptr[v], e = t_rowptr[v + 1];
  const int32_t len = e - b;
  if (len > kMidRow) {
    lists[n + atomicAdd(&list_len[1], 1)] = v;  // second half of lists: large rows
    return;
  }
  if (len > kSmallRow) {
    lists[atomicAdd(&list_len[0], 1)] = v;
    return;
  }
  uint64_t* a = keys + b;
  for (int32_t i = 1; i < len; ++i) {
    const uint64_t x = a[i];
    int32_t j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
  for (int32_t i = 0; i < len; ++i) unpack_to(a[i], t_col, t_w, b + i);
}

// Bitonic sort of `cnt` keys staged in LDS (padded to a power of two with
// the largest key), ascending. All threads of the work-group take part.
__device__ void lds_bitonic(uint64_t* s, int32_t cnt) {
  int32_t p2 = 1;
  while (p2 < cnt) p2 <<= 1;
  for (int32_t i = cnt + threadIdx.x; i < p2; i += blockDim.x) s[i] = ~0ull;
  __syncthreads();
  for (int32_t size = 2; size <= p2; size <<= 1) {
    for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (int32_t i = threadIdx.x; i < (p2 >> 1); i += blockDim.x) {
        const int32_t lo = 2 * i - (i & (stride - 1));
        const int32_t hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t a = s[lo], b = s[hi];
        if ((a > b) == up) {
          s[lo] = b;
          s[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void k_sort_mid(const int32_t* __restrict__ t_rowptr,
                                                  const int32_t* __restrict__ rows, uint64_t* __restrict__ keys,
                                                  int32_t* __restrict__ t_col, int32_t* __restrict__ t_w) {
  __shared__ uint64_t s[kMidRow];
  const int32_t v = rows[blockIdx.x];
  const int32_t b = t_rowptr[v], len = t_rowptr[v + 1] - b;
  for (int32_t i = threadIdx.x; i < len; i += blockDim.x) s[i] = keys[b + i];
  __syncthreads();
  lds_bitonic(s, len);
  for (int32_t i = threadIdx.x; i < len; i += blockDim.x) unpack_to(s[i], t_col, t_w, b + i);
}

// Rows longer than kMidRow: sort kMidRow-sized chunks in LDS, then merge
// runs pairwise (merge-path split per thread), ping-ponging between the
// key buffer and `alt`; the last pass unpacks.
__global__ __launch_bounds__(256) void k_sort_large(const int32_t* __restrict__ t_rowptr,
                                                    const int32_t* __restrict__ rows, uint64_t* __restrict__ keys,
                                                    uint64_t* __restrict__ alt, int32_t* __restrict__ t_col,
                                                    int32_t* __restrict__ t_w) {
  __shared__ uint64_t s[kMidRow];
  const int32_t v = rows[blockIdx.x];
  const int64_t b = t_rowptr[v];
  const int64_t len = t_rowptr[v + 1] - b;
  for (int64_t c0 = 0; c0 < len; c0 += kMidRow) {
    const int32_t cnt = static_cast<int32_t>(min<int64_t>(kMidRow, len - c0));
    for (int32_t i = threadIdx.x; i < cnt; i += blockDim.x) s[i] = keys[b + c0 + i];
    __syncthreads();
    lds_bitonic(s, cnt);
    for (int32_t i = threadIdx.x; i < cnt; i += blockDim.x) keys[b + c0 + i] = s[i];
    __syncthreads();
  }
  uint64_t* src = keys + b;
  uint64_t* dst = alt + b;
  const int64_t per = (len + blockDim.x - 1) / blockDim.x;
  for (int64_t width = kMidRow; width < len; width <<= 1) {
    int64_t p = static_cast<int64_t>(threadIdx.x) * per;
    const int64_t pend = min(len, p + per);
    while (p < pend) {
      const int64_t pair = (p / (2 * width)) * (2 * width);
      const int64_t a0 = pair, a1 = min(pair + width, len);
      const int64_t b0 = a1, b1 = min(pair + 2 * width, len);
      const int64_t la = a1 - a0, lb = b1 - b0;
      const int64_t d = p - pair;
      int64_t lo = max<int64_t>(0, d - lb), hi = min(d, la);
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (src[a0 + mid] < src[b0 + d - 1 - mid]) lo = mid + 1;
        else hi = mid;
      }
      int64_t i = lo, j = d - lo;
      const int64_t stop = min(pend, pair + la + lb);
      for (; p < stop; ++p) {
        const bool take_a = (j >= lb) || (i < la && src[a0 + i] < src[b0 + j]);
        dst[p] = take_a ? src[a0 + i++] : src[b0 + j++];
      }
    }
    __syncthreads();
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  for (int64_t i = threadIdx.x; i < len; i += blockDim.x) unpack_to(src[i], t_col, t_w, b + i);
}

// ---------------------------------------------------------------------------
// TOCAB partition.
//
// One wave per merge range j (rows [j*k, (j+1)*k)). The wave takes the range's
// rows 64 at a time, one row per lane, and visits the (row, block) segments
// in ascending block order across the wave: in each round the smallest
// current block s among the lanes is found, the lanes sitting on s are
// ranked by lane (= by row, so local ids stay ascending), and they jump past
// their segment with a binary search. Counting mode tallies rows per block;
// assigning mode hands out local ids from the per-block bases of the range.

__device__ __forceinline__ int32_t first_at_least(const int32_t* a, int32_t lo, int32_t hi, int64_t key) {
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (static_cast<int64_t>(a[mid]) < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <bool kAssign>
__global__ __launch_bounds__(64) void k_part_walk(const int32_t* __restrict__ a_rowptr,
                                                  const int32_t* __restrict__ a_col, int32_t n_rows,
                                                  int32_t log2W, int32_t B, int32_t log2k,
                                                  int32_t* __restrict__ cnt_jmajor,
                                                  const int32_t* __restrict__ range_ptr,
                                                  int32_t* __restrict__ id_map, int32_t* __restrict__ len,
                                                  int32_t* __restrict__ seg_start) {
  extern __shared__ int32_t base[];  // [B], touched by lane 0 only inside the walk
  const int32_t j = blockIdx.x;
  const int lane = threadIdx.x;
  for (int32_t s = lane; s < B; s += kWave)
    base[s] = kAssign ? range_ptr[static_cast<int64_t>(j) * B + s] : 0;
  __syncthreads();
  const int32_t r_begin = j << log2k;
  const int32_t r_end = static_cast<int32_t>(min<int64_t>(n_rows, static_cast<int64_t>(r_begin) + (1 << log2k)));
  for (int32_t rb = r_begin; rb < r_end; rb += kWave) {
    const int32_t r = rb + lane;
    int32_t pos = 0, end = 0;
    if (r < r_end) {
      pos = a_rowptr[r];
      end = a_rowptr[r + 1];
    }
    int32_t cur = pos < end ? (a_col[pos] >> log2W) : INT_MAX;
    for (;;) {
      const int32_t smin = gcd::wave_min(cur);
      if (smin == INT_MAX) break;
      const bool mine = cur == smin;
      const uint64_t mask = __ballot(mine);
      int32_t b0 = 0;
      if (lane == 0) {
        b0 = base[smin];
        base[smin] = b0 + __popcll(mask);
      }
      b0 = __shfl(b0, 0, kWave);
      if (mine) {
        const int32_t seg_end = first_at_least(a_col, pos, end, (static_cast<int64_t>(smin) + 1) << log2W);
        if (kAssign) {
          const int32_t l = b0 + __popcll(mask & gcd::lanemask_lt());
          id_map[l] = r;
          len[l] = seg_end - pos;
          seg_start[l] = pos;
        }
        pos = seg_end;
        cur = pos < end ? (a_col[pos] >> log2W) : INT_MAX;
      }
    }
  }
  if (!kAssign) {
    __syncthreads();
    for (int32_t s = lane; s < B; s += kWave) cnt_jmajor[static_cast<int64_t>(j) * B + s] = base[s];
  }
}

__global__ void k_transpose_counts(const int32_t* __restrict__ cnt_jmajor, int32_t* __restrict__ cnt_smajor,
                                   int32_t B, int32_t R) {
  const int64_t total = static_cast<int64_t>(B) * R;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t s = i / R, j = i - s * R;
    cnt_smajor[i] = cnt_jmajor[j * B + s];
  }
}

// range_ptr[j*B + s] = first local row of block s at range j (j = R: block end)
__global__ void k_range_ptr(const int32_t* __restrict__ base_smajor, int32_t B, int32_t R,
                            int32_t* __restrict__ range_ptr, int32_t* __restrict__ blk_rowoff) {
  const int64_t total = static_cast<int64_t>(R + 1) * B;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t j = i / B, s = i - j * B;
    range_ptr[i] = (j < R) ? base_smajor[s * R + j] : base_smajor[(s + 1) * R];
    if (j == 0) blk_rowoff[s] = base_smajor[s * R];
    if (i == 0) blk_rowoff[B] = base_smajor[static_cast<int64_t>(B) * R];
  }
}

// Copies every local row's segment of columns (and weights); rows longer
// than a wave are copied by the whole wave.
__global__ __launch_bounds__(256) void k_part_copy(const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ seg_start, int64_t P,
                                                   const int32_t* __restrict__ a_col,
                                                   const int32_t* __restrict__ a_w, int32_t* __restrict__ col,
                                                   int32_t* __restrict__ w) {
  const int64_t l = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  int32_t dst = 0, src = 0, cnt = 0;
  if (l < P) {
    dst = row_ptr[l];
    cnt = row_ptr[l + 1] - dst;
    src = seg_start[l];
  }
  const bool wide = cnt > kWave;
  if (!wide) {
    for (int32_t i = 0; i < cnt; ++i) {
      col[dst + i] = a_col[src + i];
      if (w) w[dst + i] = a_w[src + i];
    }
  }
  uint64_t pending = __ballot(wide);
  while (pending) {
    const int owner = __ffsll(static_cast<long long>(pending)) - 1;
    pending &= pending - 1;
    const int32_t d2 = __shfl(dst, owner, kWave), s2 = __shfl(src, owner, kWave), c2 = __shfl(cnt, owner, kWave);
    for (int32_t i = lane; i < c2; i += kWave) {
      col[d2 + i] = a_col[s2 + i];
      if (w) w[d2 + i] = a_w[s2 + i];
    }
  }
}

// Structural check that keeps later kernels in bounds: rowptr[0] = 0,
// rowptr[n] = m, rowptr non-decreasing, every column in [0, n).
__global__ void k_check_csr(const int32_t* __restrict__ rowptr, int32_t n, const int32_t* __restrict__ colidx,
                            int64_t m, int32_t* __restrict__ bad) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t top = m > n ? m : n;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < top; i += stride) {
    if (i < n) {
      const int32_t a = rowptr[i], b = rowptr[i + 1];
      if (b < a || a < 0 || b > m) atomicOr(bad, 1);
      if (i == 0 && a != 0) atomicOr(bad, 1);
      if (i == n - 1 && b != m) atomicOr(bad, 1);
    }
    if (i < m) {
      const int32_t v = colidx[i];
      if (v < 0 || v >= n) atomicOr(bad, 2);
    }
  }
}

__global__ void k_tile_rows(const int32_t* __restrict__ row_ptr, int32_t rows, int32_t tile_arcs, int32_t n_tiles,
                            int32_t* __restrict__ tile_row) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_tiles) return;
  if (t == n_tiles) {
    tile_row[t] = rows;
    return;
  }
  tile_row[t] = first_at_least(row_ptr, 0, rows, static_cast<int64_t>(t) * tile_arcs);
}

// Low 16 bits of (value & mask): a column inside its block, or a row inside
// its merge range.
__global__ void k_col16(const int32_t* __restrict__ col, int64_t m, int32_t mask, uint16_t* __restrict__ col16) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += stride)
    col16[i] = static_cast<uint16_t>(col[i] & mask);
}

// Head bit of every local row: bit row_ptr[r] of the arc bitmap.
__global__ void k_heads_set(const int32_t* __restrict__ row_ptr, int64_t P, gc_head_word* __restrict__ heads) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < P; r += stride) {
    const int64_t i = row_ptr[r];
    atomicOr(reinterpret_cast<unsigned long long*>(&heads[i >> 6].bits), 1ull << (i & 63));
  }
}

// Bits at and past arc m are set, so a row walk always stops at the end;
// every word records the first local row whose head lies at or after it.
__global__ void k_heads_finish(const int32_t* __restrict__ row_ptr, int64_t P, int64_t m, int64_t words,
                               gc_head_word* __restrict__ heads) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < words; w += stride) {
    const int64_t lo = w << 6;
    if (lo + 64 > m) heads[w].bits |= lo >= m ? ~0ull : (~0ull << (m - lo));
    heads[w].row = first_at_least(row_ptr, 0, static_cast<int32_t>(P), lo);
  }
}

// Bit 0 of the following word (after k_heads_finish; the last word's is set).
__global__ void k_heads_next(int64_t words, gc_head_word* __restrict__ heads) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < words; w += stride)
    heads[w].next = w + 1 < words ? static_cast<int32_t>(heads[w + 1].bits & 1ull) : 1;
}

// Rows of block b in merge range j, from the j-major range table.
__global__ void k_seg_counts(const int32_t* __restrict__ range_ptr, int32_t B, int32_t R, int32_t* __restrict__ cnt) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;  // i = j*B + b
  if (i >= static_cast<int64_t>(B) * R) return;
  cnt[i] = range_ptr[i + B] - range_ptr[i];
}

// seg[b][j] = (first local row of block b in range j, shift that moves the
// block-major row index to its range-major index); rstart[j] = first
// range-major index of range j.
__global__ void k_seg_table(const int32_t* __restrict__ range_ptr, const int32_t* __restrict__ rm_start, int32_t B,
                            int32_t R, int64_t P, int2* __restrict__ seg, int32_t* __restrict__ rstart) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;  // i = b*(R+1) + j
  if (i >= static_cast<int64_t>(B) * (R + 1)) return;
  const int32_t b = static_cast<int32_t>(i / (R + 1)), j = static_cast<int32_t>(i % (R + 1));
  const int64_t jb = static_cast<int64_t>(j) * B + b;
  const int32_t first = range_ptr[jb];
  seg[i] = make_int2(first, j < R ? rm_start[jb] - first : 0);
  if (b == 0) rstart[j] = j < R ? rm_start[jb] : static_cast<int32_t>(P);
}

// First arc of every (block, range) boundary row.
__global__ void k_seg_arcs(const int2* __restrict__ seg, int64_t count, const int32_t* __restrict__ row_ptr,
                           int32_t* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = row_ptr[seg[i].x];
}

// id16 of every local row, scattered to the row's range-major index.
__global__ void k_id16_stream(const int32_t* __restrict__ id_map, int64_t P, const int32_t* __restrict__ blk_rowoff,
                              int32_t B, int32_t R, int32_t log2k, const int2* __restrict__ seg,
                              uint16_t* __restrict__ id16s) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < P; r += stride) {
    const int32_t v = id_map[r];
    const int32_t j = v >> log2k;
    int32_t lo = 0, hi = B;  // block: last b with blk_rowoff[b] <= r
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (blk_rowoff[mid] <= r) lo = mid;
      else hi = mid;
    }
    id16s[r + seg[static_cast<int64_t>(lo) * (R + 1) + j].y] = static_cast<uint16_t>(v & ((1 << log2k) - 1));
  }
}

// cap: only for kernels that stride over their items; others get one thread per item.
inline int grid_for(int64_t items, int threads, int cap = INT_MAX) {
  const int64_t g = (items + threads - 1) / threads;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, cap)));
}

}  // namespace

namespace gcx {

hipError_t check_csr(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx, int32_t* bad_out,
                     hipStream_t s) {
  Buf bad(sizeof(int32_t), s);
  if (!bad.p) return hipErrorOutOfMemory;
  GC_HIP_TRY(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
  k_check_csr<<<grid_for(std::max<int64_t>(n, m), 256, 65536), 256, 0, s>>>(rowptr, n, colidx, m,
                                                                              bad.as<int32_t>());
  GC_HIP_TRY(hipGetLastError());
  GC_HIP_TRY(hipMemcpyAsync(bad_out, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  return hipStreamSynchronize(s);
}

hipError_t build_tiles(const int32_t* row_ptr, int64_t rows, int64_t arcs, int32_t tile_arcs, int32_t** out,
                       int32_t* n_tiles, hipStream_t s) {
  const int64_t nt = arcs / tile_arcs + 1;  // arc index `arcs` (trailing empty rows) falls in the last tile
  *n_tiles = static_cast<int32_t>(nt);
  *out = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * (nt + 1), s));
  if (!*out) return hipErrorOutOfMemory;
  k_tile_rows<<<grid_for(nt + 1, 256, INT_MAX), 256, 0, s>>>(row_ptr, static_cast<int32_t>(rows), tile_arcs,
                                                             static_cast<int32_t>(nt), *out);
  return hipGetLastError();
}

hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipMemsetAsync(out, 0, sizeof(int32_t), s);
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  Buf tile(sizeof(int32_t) * tiles, s);
  if (!tile.p) return hipErrorOutOfMemory;
  k_scan_reduce<<<tiles, kScanThreads, 0, s>>>(in, n, tile.as<int32_t>());
  k_scan_top<<<1, kScanThreads, 0, s>>>(tile.as<int32_t>(), tiles);
  k_scan_apply<<<tiles, kScanThreads, 0, s>>>(in, out, n, tile.as<int32_t>());
  GC_HIP_TRY(hipGetLastError());
  return hipStreamSynchronize(s);  // the tile buffer is released on return
}

hipError_t build_transpose(int32_t n, int64_t m, const int32_t* rowptr, const int32_t* colidx,
                           const int32_t* w, int32_t* t_rowptr, int32_t* t_colidx, int32_t* t_w,
                           hipStream_t s) {
  Buf cnt(sizeof(int32_t) * (static_cast<size_t>(n) + 1), s);
  Buf lists(sizeof(int32_t) * 2 * static_cast<size_t>(n), s);
  Buf list_len(sizeof(int32_t) * 2, s);
  Buf keys(sizeof(uint64_t) * std::max<int64_t>(m, 1), s);
  if (!cnt.p || !lists.p || !list_len.p || !keys.p) return hipErrorOutOfMemory;
  GC_HIP_TRY(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * n, s));
  GC_HIP_TRY(hipMemsetAsync(list_len.p, 0, sizeof(int32_t) * 2, s));
  if (m > 0) k_indegree<<<grid_for(m, 256, 65536), 256, 0, s>>>(colidx, m, cnt.as<int32_t>());
  GC_HIP_TRY(hipGetLastError());
  GC_HIP_TRY(scan_exclusive(cnt.as<int32_t>(), t_rowptr, n, s));
  GC_HIP_TRY(hipMemcpyAsync(cnt.p, t_rowptr, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
  if (m > 0)
    k_scatter<<<grid_for(m, kScatterTile), 256, 0, s>>>(rowptr, n, colidx, w, m, cnt.as<int32_t>(),
                                                         keys.as<uint64_t>());
  k_sort_small<<<grid_for(n, 256), 256, 0, s>>>(t_rowptr, n, keys.as<uint64_t>(), t_colidx, t_w,
                                                lists.as<int32_t>(), list_len.as<int32_t>());
  GC_HIP_TRY(hipGetLastError());
  int32_t counts[2];
  GC_HIP_TRY(hipMemcpyAsync(counts, list_len.p, sizeof(counts), hipMemcpyDeviceToHost, s));
  GC_HIP_TRY(hipStreamSynchronize(s));
  if (counts[0] > 0)
    k_sort_mid<<<counts[0], 256, 0, s>>>(t_rowptr, lists.as<int32_t>(), keys.as<uint64_t>(), t_colidx, t_w);
  if (counts[1] > 0) {
    Buf alt(sizeof(uint64_t) * m, s);
    if (!alt.p) return hipErrorOutOfMemory;
    k_sort_large<<<counts[1], 256, 0, s>>>(t_rowptr, lists.as<int32_t>() + n, keys.as<uint64_t>(),
                                           alt.as<uint64_t>(), t_colidx, t_w);
    GC_HIP_TRY(hipGetLastError());
    GC_HIP_TRY(hipStreamSynchronize(s));
  }
  GC_HIP_TRY(hipGetLastError());
  return hipStreamSynchronize(s);
}

// Stream layout of an LDS-resident pull partition: padded 16-bit columns,
// head bits, wave-tile rows, the range-major position table, range-major
// id16, and chunks (one work-group each) cut at merge-range boundaries so
// a chunk's slice of the position table fits in LDS beside the block's slice.
hipError_t build_lds_stream(gc_tocab t, hipStream_t s) {
  const int32_t B = t->B, R = t->R;
  const int64_t P = t->P, m = t->m;
  const int64_t entries = static_cast<int64_t>(B) * (R + 1);
  const int64_t tile = wave_tile_arcs();
  t->m_pad = (m / tile + 2) * tile;
  const int64_t words = t->m_pad / 64 + 1;
  t->col16 = static_cast<uint16_t*>(dev_alloc(sizeof(uint16_t) * t->m_pad, s));
  t->heads = static_cast<gc_head_word*>(dev_alloc(sizeof(gc_head_word) * words, s));
  t->seg = static_cast<int2*>(dev_alloc(sizeof(int2) * entries, s));
  t->rstart = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * (R + 1), s));
  t->id16s = static_cast<uint16_t*>(dev_alloc(sizeof(uint16_t) * (std::max<int64_t>(P, 1) + 8), s));
  if (!t->col16 || !t->heads || !t->seg || !t->rstart || !t->id16s) return hipErrorOutOfMemory;
  t->bytes += static_cast<int64_t>(sizeof(uint16_t)) * (t->m_pad + P) + 16 * words + 8 * entries + 4 * (R + 1);
  GC_HIP_TRY(hipMemsetAsync(t->col16, 0, sizeof(uint16_t) * t->m_pad, s));
  GC_HIP_TRY(hipMemsetAsync(t->heads, 0, sizeof(gc_head_word) * words, s));
  if (m > 0) k_col16<<<grid_for(m, 256, 65536), 256, 0, s>>>(t->col, m, t->W - 1, t->col16);
  if (P > 0) k_heads_set<<<grid_for(P, 256, 65536), 256, 0, s>>>(t->row_ptr, P, t->heads);
  k_heads_finish<<<grid_for(words, 256, 65536), 256, 0, s>>>(t->row_ptr, P, m, words, t->heads);
  k_heads_next<<<grid_for(words, 256, 65536), 256, 0, s>>>(words, t->heads);
  GC_HIP_TRY(hipGetLastError());

  // range-major start of every (range j, block b) slice: exclusive scan of
  // the slice sizes in j-major order
  const int64_t BR = static_cast<int64_t>(B) * R;
  Buf cnt(sizeof(int32_t) * std::max<int64_t>(BR, 1), s), rm(sizeof(int32_t) * (BR + 1), s);
  Buf arcs(sizeof(int32_t) * entries, s);
  if (!cnt.p || !rm.p || !arcs.p) return hipErrorOutOfMemory;
  k_seg_counts<<<grid_for(BR, 256, INT_MAX), 256, 0, s>>>(t->range_ptr, B, R, cnt.as<int32_t>());
  GC_HIP_TRY(hipGetLastError());
  GC_HIP_TRY(scan_exclusive(cnt.as<int32_t>(), rm.as<int32_t>(), BR, s));
  k_seg_table<<<grid_for(entries, 256, INT_MAX), 256, 0, s>>>(t->range_ptr, rm.as<int32_t>(), B, R, P, t->seg,
                                                              t->rstart);
  if (P > 0)
    k_id16_stream<<<grid_for(P, 256, 65536), 256, 0, s>>>(t->id_map, P, t->blk_rowoff, B, R, t->log2k, t->seg,
                                                          t->id16s);
  k_seg_arcs<<<grid_for(entries, 256, INT_MAX), 256, 0, s>>>(t->seg, entries, t->row_ptr, arcs.as<int32_t>());
  GC_HIP_TRY(hipGetLastError());

  // chunks on the host from the boundary rows and their first arcs
  std::vector<int2> hseg(entries);
  std::vector<int32_t> harc(entries);
  GC_HIP_TRY(hipMemcpyAsync(hseg.data(), t->seg, sizeof(int2) * entries, hipMemcpyDeviceToHost, s));
  GC_HIP_TRY(hipMemcpyAsync(harc.data(), arcs.p, sizeof(int32_t) * entries, hipMemcpyDeviceToHost, s));
  GC_HIP_TRY(hipStreamSynchronize(s));
  // A block's ranges are cut into chunks of about equal arc counts (near
  // `target`, at most `cap` ranges each); chunks are launched largest first,
  // so the work-groups that start last are the short ones.
  const int64_t target = std::max<int64_t>(kLdsChunkArcs, m / 1024);
  const int32_t cap = lds_seg_cap(t->W);
  struct Chunk {
    int32_t beg, end, blk, j0, ns;
    int64_t arcs;
  };
  std::vector<Chunk> ch;
  int32_t seg_max = 1;
  for (int32_t b = 0; b < B; ++b) {
    const int64_t o = static_cast<int64_t>(b) * (R + 1);
    const int64_t mb = harc[o + R] - harc[o];
    const int64_t pieces = std::max<int64_t>(1, (mb + target - 1) / target);
    const int64_t per = (mb + pieces - 1) / pieces;  // arcs per chunk of this block
    int32_t j = 0;
    while (j < R) {
      const int32_t ja = j;
      int64_t a = 0;
      while (j < R && j - ja < cap && (j == ja || a < per)) {
        a += harc[o + j + 1] - harc[o + j];
        ++j;
      }
      const int32_t r0 = hseg[o + ja].x, r1 = hseg[o + j].x;
      if (r1 > r0) {
        ch.push_back({r0, r1, b, ja, j - ja, a});
        seg_max = std::max(seg_max, j - ja);
      }
    }
  }
  // Dispatch order, XCD aware: the GPU hands consecutive work-groups to its
  // kXcds XCDs in turn (work-group i to XCD i mod kXcds), and each XCD has
  // its own L2. All chunks of a block go to one XCD, next to each other in
  // its sequence, so the block's slice of c comes from memory once and
  // from that L2 for the block's other chunks. Blocks are dealt largest
  // first, each to the XCD with the fewest arcs so far; within a block the
  // largest chunk runs first; shorter lists are padded with empty chunks.
  constexpr int kXcds = 8;
  std::vector<int64_t> blk_arcs(static_cast<size_t>(B), 0);
  for (const Chunk& c : ch) blk_arcs[c.blk] += c.arcs;
  std::vector<int32_t> order(static_cast<size_t>(B));
  for (int32_t b = 0; b < B; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return blk_arcs[x] > blk_arcs[y]; });
  std::stable_sort(ch.begin(), ch.end(), [](const Chunk& x, const Chunk& y) { return x.arcs > y.arcs; });
  std::vector<std::vector<int32_t>> blk_chunks(static_cast<size_t>(B));  // chunk ids per block, largest first
  for (int32_t i = 0; i < static_cast<int32_t>(ch.size()); ++i) blk_chunks[ch[i].blk].push_back(i);
  std::vector<std::vector<int32_t>> xcd(kXcds);
  std::vector<int64_t> load(kXcds, 0);
  for (int32_t b : order) {
    if (blk_chunks[b].empty()) continue;
    const int x = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += blk_arcs[b];
    for (int32_t i : blk_chunks[b]) xcd[x].push_back(i);
  }
  size_t longest = 0;
  for (const auto& l : xcd) longest = std::max(longest, l.size());
  std::vector<int32_t> beg, end, blk, j0v, nsv;
  for (size_t pos = 0; pos < longest; ++pos)
    for (int x = 0; x < kXcds; ++x) {
      if (pos < xcd[x].size()) {
        const Chunk& c = ch[xcd[x][pos]];
        beg.push_back(c.beg);
        end.push_back(c.end);
        blk.push_back(c.blk);
        j0v.push_back(c.j0);
        nsv.push_back(c.ns);
      } else {  // padding: no rows (the kernel returns at once)
        beg.push_back(0);
        end.push_back(0);
        blk.push_back(0);
        j0v.push_back(0);
        nsv.push_back(1);
      }
    }
  if (ch.empty()) beg.clear(), end.clear(), blk.clear(), j0v.clear(), nsv.clear();
  const int32_t nch = static_cast<int32_t>(beg.size());
  t->n_chunks = nch;
  t->seg_max = seg_max;
  const size_t cb = sizeof(int32_t) * std::max(nch, 1);
  t->chunk_beg = static_cast<int32_t*>(dev_alloc(cb, s));
  t->chunk_end = static_cast<int32_t*>(dev_alloc(cb, s));
  t->chunk_blk = static_cast<int32_t*>(dev_alloc(cb, s));
  t->chunk_j0 = static_cast<int32_t*>(dev_alloc(cb, s));
  t->chunk_ns = static_cast<int32_t*>(dev_alloc(cb, s));
  if (!t->chunk_beg || !t->chunk_end || !t->chunk_blk || !t->chunk_j0 || !t->chunk_ns) return hipErrorOutOfMemory;
  t->bytes += 5 * static_cast<int64_t>(cb);
  if (nch > 0) {
    GC_HIP_TRY(hipMemcpyAsync(t->chunk_beg, beg.data(), sizeof(int32_t) * nch, hipMemcpyHostToDevice, s));
    GC_HIP_TRY(hipMemcpyAsync(t->chunk_end, end.data(), sizeof(int32_t) * nch, hipMemcpyHostToDevice, s));
    GC_HIP_TRY(hipMemcpyAsync(t->chunk_blk, blk.data(), sizeof(int32_t) * nch, hipMemcpyHostToDevice, s));
    GC_HIP_TRY(hipMemcpyAsync(t->chunk_j0, j0v.data(), sizeof(int32_t) * nch, hipMemcpyHostToDevice, s));
    GC_HIP_TRY(hipMemcpyAsync(t->chunk_ns, nsv.data(), sizeof(int32_t) * nch, hipMemcpyHostToDevice, s));
  }
  return hipStreamSynchronize(s);  // host vectors and Bufs are released on return
}

// ---- expanded contributions of the TOCAB push ----
// A push block's local rows (source u, block b) are ordered by source, so
// the rows of block b whose source lies in source block s (the W sources
// [sW, (s+1)W)) are one run, bounded by the range table at the merge
// ranges s W/k and (s+1) W/k. The work-group that has just updated the
// vertices of source block s holds their new contributions and writes them
// to each of those B runs. Long runs (128 rows or more on average) are
// walked in place, with xid16[l] = the source of row l as an offset inside
// its source block. Short ones are listed block after block per source
// block (the source-major order): xperm[q] is the row at position q,
// xid16[q] its source offset, xstart[s] the first position of source
// block s.

// cnt[s*B + b] = local rows of block b whose source lies in source block s.
__global__ void k_push_run_counts(const int32_t* __restrict__ range_ptr, int32_t B, int32_t R, int32_t S,
                                  int32_t shift, int32_t* __restrict__ cnt) {
  const int64_t total = static_cast<int64_t>(S) * B;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t s = i / B, b = i - s * B;
    const int64_t j0 = s << shift, j1 = min<int64_t>(R, (s + 1) << shift);
    cnt[i] = range_ptr[j1 * B + b] - range_ptr[j0 * B + b];
  }
}

// Source-major position of every local row (base: exclusive scan of cnt).
__global__ void k_push_perm(const int32_t* __restrict__ range_ptr, const int32_t* __restrict__ base,
                            const int32_t* __restrict__ id_map, int32_t B, int32_t S, int32_t shift,
                            int32_t wmask, int32_t* __restrict__ xperm, uint16_t* __restrict__ xid16,
                            int32_t* __restrict__ xstart) {
  const int64_t total = static_cast<int64_t>(S) * B;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t s = i / B, b = i - s * B;
    const int32_t st = range_ptr[(s << shift) * B + b];
    const int32_t q0 = base[i], len = base[i + 1] - q0;
    for (int32_t k = 0; k < len; ++k) {
      xperm[q0 + k] = st + k;
      xid16[q0 + k] = static_cast<uint16_t>(id_map[st + k] & wmask);
    }
    if (b == 0) xstart[s] = q0;
    if (i == 0) xstart[S] = base[total];
  }
}

// Builds t's expanded-contribution form (GC_PUSH partitions whose block
// sums fit in LDS).
hipError_t build_push_expand(gc_tocab t, hipStream_t s) {
  const int32_t B = t->B, R = t->R;
  const int32_t S = static_cast<int32_t>((static_cast<int64_t>(t->n_rows) + t->W - 1) >> t->log2W);
  const int64_t SB = static_cast<int64_t>(S) * B;
  const size_t Pn = static_cast<size_t>(std::max<int64_t>(t->P, 1));
  t->n_sblk = S;
  // padded so that the 8-byte read of the last group of four rows stays inside
  t->xid16 = static_cast<uint16_t*>(dev_alloc(sizeof(uint16_t) * (Pn + 8), s));
  t->xc = static_cast<float*>(dev_alloc(sizeof(float) * 2 * push_xc_stride(t->P), s));
  if (!t->xid16 || !t->xc) return hipErrorOutOfMemory;
  t->bytes += static_cast<int64_t>(Pn) * 2 + 16 + 8 * push_xc_stride(t->P);
  GC_HIP_TRY(hipMemsetAsync(t->xid16, 0, sizeof(uint16_t) * (Pn + 8), s));
  if (t->P >= kPushLongRun * SB) {
    k_col16<<<grid_for(t->P, 256, 65536), 256, 0, s>>>(t->id_map, t->P, t->W - 1, t->xid16);
    GC_HIP_TRY(hipGetLastError());
  } else {
    const int32_t shift = t->log2W - t->log2k;
    Buf cnt(sizeof(int32_t) * SB, s), base(sizeof(int32_t) * (SB + 1), s);
    if (!cnt.p || !base.p) return hipErrorOutOfMemory;
    k_push_run_counts<<<grid_for(SB, 256, 65536), 256, 0, s>>>(t->range_ptr, B, R, S, shift, cnt.as<int32_t>());
    GC_HIP_TRY(hipGetLastError());
    GC_HIP_TRY(scan_exclusive(cnt.as<int32_t>(), base.as<int32_t>(), SB, s));
    t->xperm = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * Pn, s));
    t->xstart = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * (S + 1), s));
    if (!t->xperm || !t->xstart) return hipErrorOutOfMemory;
    t->bytes += static_cast<int64_t>(Pn) * 4 + 4 * (S + 1);
    k_push_perm<<<grid_for(SB, 256, 65536), 256, 0, s>>>(t->range_ptr, base.as<int32_t>(), t->id_map, B, S, shift,
                                                         t->W - 1, t->xperm, t->xid16, t->xstart);
    GC_HIP_TRY(hipGetLastError());
    GC_HIP_TRY(hipStreamSynchronize(s));  // before the Bufs are released
  }
  // the arc streams: destination offsets and head bits
  const int64_t m = t->m, tile = wave_tile_arcs();
  t->pm_pad = (m / tile + 2) * tile;
  const int64_t words = t->pm_pad / 64 + 1;
  t->pcol16 = static_cast<uint16_t*>(dev_alloc(sizeof(uint16_t) * t->pm_pad, s));
  t->pheads = static_cast<gc_head_word*>(dev_alloc(sizeof(gc_head_word) * words, s));
  if (!t->pcol16 || !t->pheads) return hipErrorOutOfMemory;
  t->bytes += static_cast<int64_t>(sizeof(uint16_t)) * t->pm_pad + 16 * words;
  GC_HIP_TRY(hipMemsetAsync(t->pcol16, 0, sizeof(uint16_t) * t->pm_pad, s));
  GC_HIP_TRY(hipMemsetAsync(t->pheads, 0, sizeof(gc_head_word) * words, s));
  if (m > 0) k_col16<<<grid_for(m, 256, 65536), 256, 0, s>>>(t->col, m, t->W - 1, t->pcol16);
  k_heads_set<<<grid_for(t->P, 256, 65536), 256, 0, s>>>(t->row_ptr, t->P, t->pheads);
  k_heads_finish<<<grid_for(words, 256, 65536), 256, 0, s>>>(t->row_ptr, t->P, m, words, t->pheads);
  k_heads_next<<<grid_for(words, 256, 65536), 256, 0, s>>>(words, t->pheads);
  GC_HIP_TRY(hipGetLastError());
  return hipStreamSynchronize(s);  // the Bufs are released on return
}

hipError_t build_partition(gc_tocab t, const int32_t* a_rowptr, const int32_t* a_col, const int32_t* a_w,
                           hipStream_t s) {
  const int32_t B = t->B, R = t->R;
  const int64_t BR = static_cast<int64_t>(B) * R;
  Buf cnt(sizeof(int32_t) * BR, s), cnt_s(sizeof(int32_t) * BR, s), base_s(sizeof(int32_t) * (BR + 1), s);
  if (!cnt.p || !cnt_s.p || !base_s.p) return hipErrorOutOfMemory;
  const size_t lds = sizeof(int32_t) * B;
  GC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_part_walk<false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  GC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_part_walk<true>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  k_part_walk<false><<<R, kWave, lds, s>>>(a_rowptr, a_col, t->n_rows, t->log2W, B, t->log2k,
                                           cnt.as<int32_t>(), nullptr, nullptr, nullptr, nullptr);
  k_transpose_counts<<<grid_for(BR, 256, 65536), 256, 0, s>>>(cnt.as<int32_t>(), cnt_s.as<int32_t>(), B, R);
  GC_HIP_TRY(hipGetLastError());
  GC_HIP_TRY(scan_exclusive(cnt_s.as<int32_t>(), base_s.as<int32_t>(), BR, s));

  t->range_ptr = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * (R + 1) * static_cast<size_t>(B), s));
  t->blk_rowoff = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * (B + 1), s));
  if (!t->range_ptr || !t->blk_rowoff) return hipErrorOutOfMemory;
  k_range_ptr<<<grid_for(static_cast<int64_t>(R + 1) * B, 256, 65536), 256, 0, s>>>(
      base_s.as<int32_t>(), B, R, t->range_ptr, t->blk_rowoff);
  GC_HIP_TRY(hipGetLastError());
  int32_t P32 = 0;
  GC_HIP_TRY(hipMemcpyAsync(&P32, base_s.as<int32_t>() + BR, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GC_HIP_TRY(hipStreamSynchronize(s));
  const int64_t P = P32;
  t->P = P;
  const size_t Pn = static_cast<size_t>(std::max<int64_t>(P, 1));
  const size_t mn = static_cast<size_t>(std::max<int64_t>(t->m, 1));
  t->id_map = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * Pn, s));
  t->row_ptr = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * (Pn + 1), s));
  // padded for 4-wide reads, and past the pull's buffer resource (its range
  // check leaves out a store's scalar offset, at most 512 floats)
  t->partial = static_cast<float*>(dev_alloc(sizeof(float) * (Pn + 8 + 512), s));
  t->pmin = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * (Pn + 8), s));  // padded for 16-byte reads
  t->col = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * mn, s));
  if (t->weighted) t->w = static_cast<int32_t*>(dev_alloc(sizeof(int32_t) * mn, s));
  if (!t->id_map || !t->row_ptr || !t->partial || !t->pmin || !t->col || (t->weighted && !t->w))
    return hipErrorOutOfMemory;
  t->bytes = sizeof(int32_t) * ((R + 1) * static_cast<int64_t>(B) + B + 1 + 4 * static_cast<int64_t>(Pn) + 1 +
                                mn * (t->weighted ? 2 : 1));

  Buf len(sizeof(int32_t) * Pn, s), seg(sizeof(int32_t) * Pn, s);
  if (!len.p || !seg.p) return hipErrorOutOfMemory;
  k_part_walk<true><<<R, kWave, lds, s>>>(a_rowptr, a_col, t->n_rows, t->log2W, B, t->log2k, nullptr,
                                          t->range_ptr, t->id_map, len.as<int32_t>(), seg.as<int32_t>());
  GC_HIP_TRY(hipGetLastError());
  GC_HIP_TRY(scan_exclusive(len.as<int32_t>(), t->row_ptr, P, s));
  if (P > 0)
    k_part_copy<<<grid_for(P, 256, INT_MAX), 256, 0, s>>>(t->row_ptr, seg.as<int32_t>(), P, a_col,
                                                          t->weighted ? a_w : nullptr, t->col, t->w);
  GC_HIP_TRY(hipGetLastError());
  GC_HIP_TRY(build_tiles(t->row_ptr, P, t->m, pull_tile_arcs(), &t->tile_row, &t->n_tiles, s));
  t->id16 = static_cast<uint16_t*>(dev_alloc(sizeof(uint16_t) * Pn, s));
  if (!t->id16) return hipErrorOutOfMemory;
  if (P > 0) k_col16<<<grid_for(P, 256, 65536), 256, 0, s>>>(t->id_map, P, t->k - 1, t->id16);
  t->bytes += static_cast<int64_t>(sizeof(uint16_t)) * P;
  // the stream layout needs the whole range table of a block on the host
  // once, and 32-bit arc indices past the padded end
  if (t->dir == GC_PULL && t->W <= kLdsMaxWidth && static_cast<int64_t>(B) * (R + 1) <= (int64_t(1) << 25) &&
      t->m + 1024 < INT32_MAX && 4 * (P + 8) < (int64_t(1) << 31))
    GC_HIP_TRY(build_lds_stream(t, s));
  if (t->dir == GC_PUSH && t->W <= kPushLdsMaxWidth && t->k <= t->W && P > 0 && t->m + 1024 < INT32_MAX &&
      B <= kPushExpandMaxBlocks)
    GC_HIP_TRY(build_push_expand(t, s));
  return hipStreamSynchronize(s);
}

}  // namespace gcx
