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
// 160 KB LDS of a compute unit rather than for the last-level cache.
//
// Stream layout: columns are 16-bit offsets inside the block and the row
// structure is one head bit per arc (set on the first arc of every local
// row, kept with a running row count per 64 arcs), so a tile of arcs is
// read as plain streams with no row offsets. One work-group takes a chunk
// (rows [r0, r1) of block b, whose rows fall in merge ranges j0 ..
// j0+ns-1): it loads the slice c[bW, bW + W) and the chunk's part of the
// range-major position table into LDS, then each wave walks kWaveTile-arc
// tiles of the chunk. In a tile every lane holds 8 consecutive arcs (one
// 16-byte load of columns), reads their contributions from the LDS slice
// and takes the row boundaries from its head word; a segmented inclusive
// scan across the wave (FP64) then gives the sum of every row whose head
// lies in the tile. A row that runs past the tile end is finished by the
// whole wave over the following tiles. Each row sum is stored at the row's
// range-major index, so the merge reads every range as one stream. Loads
// run two tiles ahead of the tile being reduced (all vector loads, which
// complete in order, so waiting for one tile leaves the next in flight).
constexpr int kLdsThreads = 1024;
constexpr int kLdsWaves = kLdsThreads / kWave;
constexpr int kArcsPerLane = 8;
constexpr int kWaveTile = kArcsPerLane * kWave;  // 512 arcs, 8 head words
constexpr int kStageRows = 320;                  // staged row sums per wave in the first pass
constexpr int kTileRowsMax = 512;                // rows one tile can complete
constexpr int kStageSpare = 16;                  // spare slots per wave for elements that end no staged row
static_assert(kStageRows % kWave == 0 && (kTileRowsMax - kStageRows) % kWave == 0 &&
              kTileRowsMax - kStageRows <= kStageRows, "staging passes of whole store instructions");

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct WaveTile {
  u32x4 cols;  // this lane's 8 columns (16 bits each)
  u32x4 hw;    // head word holding this lane's arcs: bits lo, bits hi, row count, next word's bit 0
};

__device__ __forceinline__ WaveTile load_wave_tile(const uint16_t* __restrict__ col16,
                                                   const gc_head_word* __restrict__ heads, int32_t q, int lane) {
  WaveTile t;
  const int64_t tb = static_cast<int64_t>(q) * kWaveTile;
  t.cols = gcd::ld_stream(reinterpret_cast<const u32x4*>(col16 + tb) + lane);
  t.hw = *reinterpret_cast<const u32x4*>(heads + (tb >> 6) + (lane >> 3));
  return t;
}

__device__ __forceinline__ uint64_t word_bits(const u32x4& w) {
  return static_cast<uint64_t>(w[0]) | (static_cast<uint64_t>(w[1]) << 32);
}

// Merge-range index of local row r, searching forward from j: sb[j] is the
// first row of the chunk's j-th merge range (ascending; sb[ns] lies past
// the chunk and sb[ns+1..ns+3] hold INT32_MAX), four entries per step.
__device__ __forceinline__ int32_t seek_range(const int32_t* sb, int32_t j, int32_t r) {
  for (;;) {
    const int32_t adv = (sb[j + 1] <= r) + (sb[j + 2] <= r) + (sb[j + 3] <= r) + (sb[j + 4] <= r);
    j += adv;
    if (adv < 4) return j;
  }
}
constexpr int kSegPad = 4;  // LDS entries past the position table read by seek_range and the cursor

// Buffer resource over the partial sums: a store whose offset lies past the
// resource's size is dropped by the hardware, which lets every lane issue
// the same number of stores per tile (no branch around a store, so the
// compiler can count outstanding memory operations and keep the prefetched
// tiles in flight while the stores drain).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t partial_rsrc(float* partial, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(partial, 0, static_cast<int>(bytes), 0x00020000);
}
constexpr uint32_t kDropOffset = 0x80000000u;  // past any resource size below 2^31

__device__ __forceinline__ void partial_store(__amdgpu_buffer_rsrc_t out, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), out, off, 0, 0);
}

// One step of a wave-wide segmented inclusive scan of (F, A) pairs, the
// value moved between lanes by a DPP control (lanes with no source receive
// the identity (0, 0)): (F1, A1) then (F2, A2) gives (F1 | F2, F2 ? A2 : A1 + A2).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void seg_scan_step(double& A, int& F) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(A), kCtrl, kRowMask, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(A), kCtrl, kRowMask, 0xF, false);
  const int f = __builtin_amdgcn_update_dpp(0, F, kCtrl, kRowMask, 0xF, false);
  if (!F) A += __hiloint2double(hi, lo);
  F |= f;
}

// DPP controls (gfx9): shift right by n lanes inside each row of 16, copy
// lane 15 / 31 into the following row(s), shift right by one lane across
// the whole wave.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;

// What a wave carries from one tile of its range to the next: the running
// sum of the row still open at the tile's end (when that row is one the wave
// must write) and a cursor into the chunk's position table with the next
// boundaries and shifts cached in registers.
struct PullCarry {
  double open = 0.0;
  int32_t open_row = -1;           // >= 0 when the wave owes that row's sum
  int32_t jc = 0;                  // sb[jc] <= every row the wave still writes
  int32_t b1, b2, b3, d0, d1, d2;  // sb[jc+1..jc+3], sd[jc..jc+2]
};

__device__ __forceinline__ void load_cursor(const int32_t* sb, const int32_t* sd, PullCarry& c) {
  c.b1 = sb[c.jc + 1];
  c.b2 = sb[c.jc + 2];
  c.b3 = sb[c.jc + 3];
  c.d0 = sd[c.jc];
  c.d1 = sd[c.jc + 1];
  c.d2 = sd[c.jc + 2];
}

// Sum over the tiles after tile q of the row open at q's end, up to its end
// (the first head bit that follows).
__device__ double finish_open_row(const uint16_t* __restrict__ col16, const gc_head_word* __restrict__ heads,
                                  const float* slice, int32_t q, int lane) {
  double acc = 0.0;
  for (int32_t qq = q + 1;; ++qq) {
    const WaveTile u = load_wave_tile(col16, heads, qq, lane);
    const uint64_t hb = word_bits(u.hw);
    // position of the tile's first head (kWaveTile if none): lowest lane group with a set bit
    const uint64_t has = __ballot(hb != 0ull && (lane & 7) == 0);
    const int32_t grp = has ? (__ffsll(static_cast<long long>(has)) - 1) >> 3 : 8;
    const uint64_t gb = grp < 8 ? static_cast<uint64_t>(__shfl(static_cast<long long>(hb), grp * 8, kWave)) : 0ull;
    const int32_t p = grp < 8 ? 64 * grp + __ffsll(static_cast<long long>(gb)) - 1 : kWaveTile;
    double part = 0.0;
#pragma unroll
    for (int e = 0; e < kArcsPerLane; ++e)
      if (kArcsPerLane * lane + e < p) part += static_cast<double>(slice[(u.cols[e >> 1] >> (16 * (e & 1))) & 0xFFFFu]);
    acc += gcd::wave_sum(part);
    if (p < kWaveTile) return acc;  // bits past the last arc are set, so this ends
  }
}

__device__ __forceinline__ void reduce_wave_tile(const WaveTile& t, int lane, const float* slice,
                                                 const int32_t* sb, const int32_t* sd, int32_t r0, int32_t r1,
                                                 PullCarry& cr, __amdgpu_buffer_rsrc_t out, float* stage) {
  const uint32_t wlo = t.hw[0], whi = t.hw[1];
  const int32_t wrow = static_cast<int32_t>(t.hw[2]);
  const int32_t ta = __builtin_amdgcn_readfirstlane(wrow);
  const int32_t tz = __builtin_amdgcn_readlane(wrow + __popc(wlo) + __popc(whi), kWave - 1);
  // rows the wave writes from this tile: those whose head is here and that
  // belong to the chunk, and the row left open by the previous tile
  const int32_t rz = min(tz, r1);
  const int32_t rmin = cr.open_row >= 0 ? cr.open_row : max(ta, r0);
  if (rmin < rz && rmin >= cr.b1) {  // advance the range cursor
    cr.jc = seek_range(sb, cr.jc, rmin);
    load_cursor(sb, sd, cr);
  }
  // this lane's 8 head bits, the bit after them, and the heads before them
  const int sub = lane & 7, sh = 8 * (sub & 3);
  const uint32_t half = sub < 4 ? wlo : whi;
  const uint32_t my8 = (half >> sh) & 0xFFu;
  const uint32_t after = sub == 7 ? (t.hw[3] & 1u) : sub == 3 ? (whi & 1u) : (half >> (sh + 8)) & 1u;
  const uint32_t ends = (my8 >> 1) | (after << 7);  // bit e: arc e is its row's last
  const int32_t first = wrow + (sub < 4 ? 0 : __popc(wlo)) + __popc(half & ((1u << sh) - 1u));
  // Sums inside the lane's 8 arcs in FP32 (at most 8 terms, one rounding per
  // add); everything that crosses lanes or tiles in FP64.
  float sf[kArcsPerLane];
  float run = 0.0f;
#pragma unroll
  for (int e = 0; e < kArcsPerLane; ++e) {
    const float x = slice[(t.cols[e >> 1] >> (16 * (e & 1))) & 0xFFFFu];
    run = ((my8 >> e) & 1u) ? x : run + x;
    sf[e] = run;
  }
  // segmented inclusive scan of the lanes' open sums (flag: lane holds a head)
  double A = static_cast<double>(run);
  int F = my8 != 0u;
  seg_scan_step<kDppRowShr1, 0xF>(A, F);
  seg_scan_step<kDppRowShr2, 0xF>(A, F);
  seg_scan_step<kDppRowShr4, 0xF>(A, F);
  seg_scan_step<kDppRowShr8, 0xF>(A, F);
  seg_scan_step<kDppRowBcast15, 0xA>(A, F);
  seg_scan_step<kDppRowBcast31, 0xC>(A, F);
  double carry = __hiloint2double(
      __builtin_amdgcn_update_dpp(0, __double2hiint(A), kDppWaveShr1, 0xF, 0xF, false),
      __builtin_amdgcn_update_dpp(0, __double2loint(A), kDppWaveShr1, 0xF, 0xF, false));
  const int Fx = __builtin_amdgcn_update_dpp(0, F, kDppWaveShr1, 0xF, 0xF, false);
  if (!Fx) carry += cr.open;  // no head before this lane in the tile: the open row continues
  // The lane's arcs before its first head belong to a row begun earlier; only
  // the last of them (just before that head, or the lane's last arc) can end
  // it, and it gets the carried sum (rounded to FP32 once, then one FP32 add).
  const int fh = my8 ? __builtin_ctz(my8) : kArcsPerLane;
  const float carry_f = static_cast<float>(carry);
  // The rows this tile completes form one run [rs, re): the open row (if
  // the wave owes it) and every row of the chunk with its head here, except
  // the last one when it continues into the next tile. Their sums are
  // staged in LDS by row and written back so that store k of the wave holds
  // rows rs + 64k .. rs + 64k + 63 (coalesced); the position table turns a
  // row into its range-major index. Every lane always issues the same 8
  // stores (unused ones get a dropped offset), so the compiler's count of
  // outstanding memory operations stays exact.
  const uint32_t next_head = __builtin_amdgcn_readlane(static_cast<int32_t>(t.hw[3]), kWave - 1) & 1u;
  const int32_t rs = rmin;
  const int32_t re = min(rz, next_head ? tz : tz - 1);
  // Staging slot of each element, computed once: for an element that ends
  // a row, the row's offset from rs (as unsigned: rows before rs wrap to
  // huge values); otherwise none. Rows at or past re may land in slots that
  // are never read back (the write-out stops at re), so only the row ends
  // need testing here.
  uint32_t slot[kArcsPerLane];
  float val[kArcsPerLane];
  {
    int32_t r = first - 1;
#pragma unroll
    for (int e = 0; e < kArcsPerLane; ++e) {
      r += static_cast<int32_t>((my8 >> e) & 1u);
      slot[e] = ((ends >> e) & 1u) ? static_cast<uint32_t>(r - rs) : 0xFFFFFFFFu;
      val[e] = e < fh ? sf[e] + carry_f : sf[e];
    }
  }
  // rows at or past the cached boundary b3 (three or more ranges in one tile)
  // are stored on the slow path below; the others index with the cursor
  const int32_t i1 = cr.b1 - rs, i2 = cr.b2 - rs, iz = min(re, cr.b3) - rs;
  // Two passes over the staging: rows [0, 320) of the run, then [320, 512)
  // (a tile completes at most 512 rows; the second pass's LDS work is
  // skipped when it has no rows, its 3 stores are then dropped).
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const uint32_t lo = pass == 0 ? 0u : static_cast<uint32_t>(kStageRows);
    const int n = pass == 0 ? kStageRows : kTileRowsMax - kStageRows;  // rows of this pass
    if (pass == 0 || re - rs > kStageRows) {  // uniform
      // every element writes (no branch): rows of this pass to their slot,
      // the rest to one of the wave's spare slots
#pragma unroll
      for (int e = 0; e < kArcsPerLane; ++e) {
        const uint32_t k = slot[e] - lo;
        stage[k < static_cast<uint32_t>(n) ? k : kStageRows + (lane & (kStageSpare - 1))] = val[e];
      }
      wave_lds_fence();
    }
    float v[kStageRows / kWave];
#pragma unroll
    for (int k = 0; k < n / kWave; ++k) v[k] = stage[k * kWave + lane];
#pragma unroll
    for (int k = 0; k < n / kWave; ++k) {
      const int32_t i = static_cast<int32_t>(lo) + k * kWave + lane;  // row rs + i
      const int32_t d = cr.d0 + (i >= i1) * (cr.d1 - cr.d0) + (i >= i2) * (cr.d2 - cr.d1);  // arithmetic keeps cr in registers
      const uint32_t off = i < iz ? 4u * static_cast<uint32_t>(rs + i + d) : kDropOffset;
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[k]), out, off, 0, 0);
    }
    wave_lds_fence();  // the staging is rewritten next
  }
  if (re > cr.b3) {  // uniform, rare: store the rows at or past b3
#pragma unroll
    for (int e = 0; e < kArcsPerLane; ++e) {
      const int32_t r = rs + static_cast<int32_t>(slot[e]);
      if (slot[e] < static_cast<uint32_t>(re - rs) && r >= cr.b3) {
        const int32_t j = seek_range(sb, cr.jc, r);
        partial_store(out, 4u * static_cast<uint32_t>(r + sd[j]), val[e]);
      }
    }
  }
  // the row open at the tile's end, if the wave writes it
  const double mytail = fh < kArcsPerLane ? static_cast<double>(run) : static_cast<double>(run) + carry;
  const double tail = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(mytail), kWave - 1),
                                       __builtin_amdgcn_readlane(__double2loint(mytail), kWave - 1));
  const int32_t ro = tz - 1;  // the row of the tile's last arc
  const bool owe = !next_head && (tz > ta ? (ro >= r0 && ro < r1) : cr.open_row >= 0);
  cr.open_row = owe ? ro : -1;
  cr.open = owe ? tail : 0.0;
}

__global__ __launch_bounds__(kLdsThreads) void k_pr_tocab_pull_lds(
    const int32_t* __restrict__ row_ptr, const uint16_t* __restrict__ col16,
    const gc_head_word* __restrict__ heads, const int32_t* __restrict__ chunk_beg,
    const int32_t* __restrict__ chunk_end, const int32_t* __restrict__ chunk_blk,
    const int32_t* __restrict__ chunk_j0, const int32_t* __restrict__ chunk_ns, const int2* __restrict__ seg,
    int32_t R, int32_t log2W, int32_t n, const float* __restrict__ c, float* __restrict__ partial,
    uint32_t partial_bytes) {
  extern __shared__ float lds[];
  const int32_t W = 1 << log2W;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const __amdgpu_buffer_rsrc_t out = partial_rsrc(partial, partial_bytes);
  const int32_t ch = blockIdx.x;
  const int32_t r0 = chunk_beg[ch], r1 = chunk_end[ch], b = chunk_blk[ch], j0 = chunk_j0[ch], ns = chunk_ns[ch];
  float* slice = lds;
  float* stage = lds + W + wid * (kStageRows + kStageSpare);  // this wave's output staging and spare slots
  int32_t* sb = reinterpret_cast<int32_t*>(lds + W + kLdsWaves * (kStageRows + kStageSpare));  // ns + 1 boundaries, then sentinels
  int32_t* sd = sb + ns + kSegPad;                    // ns shifts, then spares
  {
    const int32_t v0 = b << log2W;
    const int32_t cnt = min(W, n - v0);
    const float4* c4 = reinterpret_cast<const float4*>(c + v0);  // v0 is a multiple of W >= 2^10
    float4* s4 = reinterpret_cast<float4*>(slice);
    for (int32_t i = threadIdx.x; i < (cnt >> 2); i += kLdsThreads) s4[i] = c4[i];
    for (int32_t i = (cnt & ~3) + threadIdx.x; i < cnt; i += kLdsThreads) slice[i] = c[v0 + i];
    const int2* sg = seg + static_cast<int64_t>(b) * (R + 1) + j0;
    for (int32_t i = threadIdx.x; i < ns + kSegPad; i += kLdsThreads) {
      if (i <= ns) {
        const int2 e = sg[i];
        sb[i] = e.x;
        sd[i] = e.y;  // i == ns: a spare, never used for a row of the chunk
      } else {
        sb[i] = INT32_MAX;
        sd[i] = 0;
      }
    }
  }
  __syncthreads();
  // each wave streams a contiguous range [qa, qz] of the chunk's tiles
  const int32_t q0 = row_ptr[r0] / kWaveTile, q1 = (row_ptr[r1] - 1) / kWaveTile;
  const int32_t nt = q1 - q0 + 1;
  const int32_t qa = q0 + static_cast<int32_t>(static_cast<int64_t>(nt) * wid / kLdsWaves);
  const int32_t qz = q0 + static_cast<int32_t>(static_cast<int64_t>(nt) * (wid + 1) / kLdsWaves) - 1;
  if (qa > qz) return;
  PullCarry cr;
  load_cursor(sb, sd, cr);
  // three tiles in registers: one is reduced while the next two load
  int32_t q = qa;
  WaveTile t0 = load_wave_tile(col16, heads, q, lane);
  WaveTile t1 = load_wave_tile(col16, heads, min(q + 1, qz), lane);
  WaveTile t2;
#define GC_PULL_STEP(cur, k, refill)                                 \
  refill = load_wave_tile(col16, heads, min(q + (k + 2), qz), lane); \
  reduce_wave_tile(cur, lane, slice, sb, sd, r0, r1, cr, out, stage); \
  if (q + (k + 1) > qz) break;
  for (;;) {
    GC_PULL_STEP(t0, 0, t2)
    GC_PULL_STEP(t1, 1, t0)
    GC_PULL_STEP(t2, 2, t1)
    q += 3;
  }
#undef GC_PULL_STEP
  if (cr.open_row >= 0) {  // the range's last row continues past it
    const double v = cr.open + finish_open_row(col16, heads, slice, qz, lane);
    if (lane == 0) {
      const int32_t j = seek_range(sb, cr.jc, cr.open_row);
      partial[cr.open_row + sd[j]] = static_cast<float>(v);
    }
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

// Figure 5 merge over the stream layout, fused with the update: range j's
// partial sums of every block are one contiguous slice [rstart[j],
// rstart[j+1]) of partial / id16s, read with 16-byte / 8-byte loads (4
// entries per load) and added into an FP64 LDS accumulator per vertex.
// Work-group size: an FP64 accumulator of 16384 entries (128 KB) leaves room
// for one work-group per CU, which then runs 16 waves; smaller ranges run two
// or more 512-thread work-groups per CU.
template <int K>
constexpr int merge_threads() { return K >= 16384 ? 1024 : 512; }

template <int K, int kMergeThreads = merge_threads<K>()>
__global__ __launch_bounds__(kMergeThreads) void k_pr_merge_stream(const int32_t* __restrict__ rstart,
                                                                   const uint16_t* __restrict__ id16s,
                                                                   const float* __restrict__ partial, Update u) {
  __shared__ double acc[K];
  for (int i = threadIdx.x; i < K; i += kMergeThreads) acc[i] = 0.0;
  __syncthreads();
  const int32_t a = rstart[blockIdx.x], z = rstart[blockIdx.x + 1];
  const int32_t g0 = a >> 2, g1 = (z + 3) >> 2;  // 4-entry groups covering [a, z)
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4* p4 = reinterpret_cast<const f4*>(partial);
  const uint64_t* i4 = reinterpret_cast<const uint64_t*>(id16s);
  constexpr int kU = 4;
  for (int32_t g = g0 + static_cast<int32_t>(threadIdx.x); g < g1; g += kMergeThreads * kU) {
    f4 p[kU];
    uint64_t id[kU];
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int32_t gg = min(g + k * kMergeThreads, g1 - 1);  // clamped, masked below
      p[k] = gcd::ld_stream(p4 + gg);
      id[k] = gcd::ld_stream(i4 + gg);
    }
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int32_t e0 = 4 * (g + k * kMergeThreads);
      const float pv[4] = {p[k][0], p[k][1], p[k][2], p[k][3]};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (e0 + e >= a && e0 + e < z)
          atomicAdd(&acc[(id[k] >> (16 * e)) & 0xFFFFu], static_cast<double>(pv[e]));
    }
  }
  __syncthreads();
  const int32_t v0 = blockIdx.x * K;
  const double D = *u.dtotal_in;
  double mine = 0.0;
  for (int i = threadIdx.x; i < K; i += kMergeThreads) {
    const int32_t v = v0 + i;
    if (v < u.n) mine += update_vertex(u, v, acc[i], D);
  }
  publish_dangling<kMergeThreads>(u, mine);
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
  // the LDS-resident pull holds a slice of up to kLdsMaxWidth floats plus its position table
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pr_tocab_pull_lds),
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds_budget(kLdsMaxWidth));
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
        {
          ProfScope prof("pr_tocab_pull", s);
          const size_t lds = sizeof(float) * (static_cast<size_t>(t->W) + 2 * static_cast<size_t>(t->seg_max) + 2 * kSegPad) +
                             kLdsStageBytes;
          if (t->n_chunks > 0)
            k_pr_tocab_pull_lds<<<t->n_chunks, kLdsThreads, lds, s>>>(
                t->row_ptr, t->col16, t->heads, t->chunk_beg, t->chunk_end, t->chunk_blk, t->chunk_j0,
                t->chunk_ns, t->seg, t->R, t->log2W, n, g->contrib[0], t->partial,
                static_cast<uint32_t>(sizeof(float) * (t->P + 8)));
        }
        u.contrib = g->contrib[0];
        ProfScope prof("pr_merge", s);
        switch (t->k) {
          case 256: k_pr_merge_stream<256><<<t->R, merge_threads<256>(), 0, s>>>(t->rstart, t->id16s, t->partial, u); break;
          case 512: k_pr_merge_stream<512><<<t->R, merge_threads<512>(), 0, s>>>(t->rstart, t->id16s, t->partial, u); break;
          case 1024: k_pr_merge_stream<1024><<<t->R, merge_threads<1024>(), 0, s>>>(t->rstart, t->id16s, t->partial, u); break;
          case 2048: k_pr_merge_stream<2048><<<t->R, merge_threads<2048>(), 0, s>>>(t->rstart, t->id16s, t->partial, u); break;
          case 4096: k_pr_merge_stream<4096><<<t->R, merge_threads<4096>(), 0, s>>>(t->rstart, t->id16s, t->partial, u); break;
          case 8192: k_pr_merge_stream<8192><<<t->R, merge_threads<8192>(), 0, s>>>(t->rstart, t->id16s, t->partial, u); break;
          case 16384:
            k_pr_merge_stream<16384><<<t->R, merge_threads<16384>(), 0, s>>>(t->rstart, t->id16s, t->partial, u);
            break;
          default: return hipErrorInvalidValue;
        }
        parts = t->R;
      } else {
        {
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
