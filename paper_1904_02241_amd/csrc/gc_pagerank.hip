// PageRank iterations on gfx950: plain pull (Algorithm 1), plain push
// (Algorithm 2), TOCAB pull (Algorithm 4 + the Figure 5 merge) and TOCAB push
// (Algorithm 5), all with the same fused update and FP64 in-row
// accumulation (except inside one 512-arc tile of the LDS-resident TOCAB
// pull, which sums in FP32), so the comparison between them isolates the
// blocking.
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
#include <cstdlib>

#include <type_traits>
#include <vector>

#include "gc_device.h"
#include "gc_internal.h"

#include "gc_pr_device.h"

namespace {

int g_cus = 256;  // compute units of the GPU (read once by pagerank_setup)

// D for the next iteration: the partials summed in index order by one
// work-group (deterministic).
__device__ __forceinline__ double reduce_slots(const double* __restrict__ slots, int32_t count, double* part) {
  double acc = 0.0;
  for (int32_t i = threadIdx.x; i < count; i += 1024) acc += slots[i];
  acc = gcd::wave_sum(acc);
  __syncthreads();  // part may still be read by a previous call
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < 1024 / kWave; ++w) t += part[w];
  return t;
}

// Total of the per-work-group dangling partials (and, in convergence mode,
// of the L1-change partials), in a fixed order.
__global__ __launch_bounds__(1024) void k_reduce_dangling(const double* __restrict__ dpart, int32_t count,
                                                          double* __restrict__ dtotal,
                                                          const double* __restrict__ lpart,
                                                          double* __restrict__ ltotal) {
  __shared__ double part[1024 / kWave];
  const double t = reduce_slots(dpart, count, part);
  if (threadIdx.x == 0) *dtotal = t;
  if (lpart) {
    const double l = reduce_slots(lpart, count, part);
    if (threadIdx.x == 0) *ltotal = l;
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
// scan across the wave (FP32) then gives the sum of every row whose head
// lies in the tile. A row that runs past the tile end is carried to the
// wave's next tile as an FP64 sum, or finished by the whole wave over the
// following tiles (FP64) when it runs past the wave's range. Row partials
// are stored as FP32. Each row sum is stored at the row's
// range-major index, so the merge reads every range as one stream. Loads
// run two tiles ahead of the tile being reduced (all vector loads, which
// complete in order, so waiting for one tile leaves the next in flight).
constexpr int kLdsThreads = 1024;
constexpr int kLdsWaves = kLdsThreads / kWave;
constexpr int kArcsPerLane = 8;
constexpr int kWaveTile = kArcsPerLane * kWave;  // 512 arcs, 8 head words
constexpr int kStageRows = 384;                  // staged row sums per wave in the first pass
constexpr int kTileRowsMax = 512;                // rows one tile can complete
constexpr int kStageSpare = 16;                  // spare slots per wave for elements that end no staged row
static_assert(kStageRows % kWave == 0 && (kTileRowsMax - kStageRows) % kWave == 0 &&
              kTileRowsMax - kStageRows <= kStageRows, "staging passes of whole store instructions");

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct WaveTile {
  u32x4 cols;  // this lane's 8 columns (16 bits each)
  u32x4 hw;    // head word holding this lane's arcs: bits lo, bits hi, row count, next word's bit 0
  f32x4 va, vb;  // the 8 arcs' values (valued pull only)
};

// Arc values of the valued (SpMV) pull: FP32, in the partition's arc order,
// padded like col16; null for PageRank, whose contributions are summed as they are.
template <bool kVal>
__device__ __forceinline__ WaveTile load_wave_tile(const uint16_t* __restrict__ col16,
                                                   const gc_head_word* __restrict__ heads,
                                                   const float* __restrict__ vals, int32_t q, int lane) {
  WaveTile t;
  const int64_t tb = static_cast<int64_t>(q) * kWaveTile;
  t.cols = gcd::ld_stream(reinterpret_cast<const u32x4*>(col16 + tb) + lane);
  t.hw = *reinterpret_cast<const u32x4*>(heads + (tb >> 6) + (lane >> 3));
  if (kVal) {
    const f32x4* v4 = reinterpret_cast<const f32x4*>(vals + tb) + 2 * lane;
    t.va = gcd::ld_stream(v4);
    t.vb = gcd::ld_stream(v4 + 1);
  }
  return t;
}

template <bool kVal>
__device__ __forceinline__ float arc_value(const WaveTile& t, int e) {
  return kVal ? (e < 4 ? t.va[e] : t.vb[e - 4]) : 1.0f;
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

__device__ __forceinline__ void partial_store(__amdgpu_buffer_rsrc_t out, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), out, off, 0, 0);
}

constexpr int kStoresPerTile = 6;  // stores of the first staging pass, issued by every tile

// kStoresPerTile stores the hardware drops (offsets past any resource size
// below 2^31, distinct so that none is a dead store of another).
__device__ __forceinline__ void drop_stores(__amdgpu_buffer_rsrc_t out) {
#pragma unroll
  for (int i = 0; i < kStoresPerTile; ++i) __builtin_amdgcn_raw_buffer_store_b32(0u, out, 0x80000000u + 4u * i, 0, 0);
}

// Lanes of the wave selected by a mask held in scalar registers.
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }


// Value a DPP control moves into each lane (lanes with no source get 0).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_moved(float a) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), kCtrl, kRowMask, 0xF, false));
}

// One step of a wave-wide segmented inclusive scan: a lane that has met no
// head yet within the reach of the steps so far (not in F) adds the value
// the DPP control moves in. F itself is kept as a lane mask in scalar
// registers and widened by the caller after each step.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void seg_scan_step(float& A, uint64_t F) {
  const float s = A + dpp_moved<kCtrl, kRowMask>(A);
  A = lane_in(F) ? A : s;
}

// DPP controls (gfx9): shift right by n lanes inside each row of 16, copy
// lane 15 / 31 into the following row(s), shift right by one lane across
// the whole wave.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;

// What a wave carries from one tile of its range to the next: the running
// sum of the row still open at the tile's end (when that row is one the wave
// must write), a window of 64 entries of the chunk's position table held one
// per lane, and a cursor into it with the next boundaries and shifts in
// scalar registers.
struct PullCarry {
  double open = 0.0;
  int32_t open_row = -1;           // >= 0 when the wave owes that row's sum
  int32_t jw = 0;                  // first table entry of the window
  int32_t sbw, sdw;                // lane l: sb[jw + l], sd[jw + l] (past the table: its last spare)
  int32_t jc = 0;                  // sb[jc] <= every row the wave still writes; jc - jw <= 60
  int32_t b1, b2, b3, d0, d1, d2;  // sb[jc+1..jc+3], sd[jc..jc+2]
};

__device__ __forceinline__ void load_window(const int32_t* sb, const int32_t* sd, int32_t ns, int lane,
                                            PullCarry& c) {
  const int32_t i = min(c.jw + lane, ns + kSegPad - 1);
  c.sbw = sb[i];
  c.sdw = sd[i];
}

__device__ __forceinline__ void cursor_from_window(PullCarry& c) {
  const int32_t o = c.jc - c.jw;
  c.b1 = __builtin_amdgcn_readlane(c.sbw, o + 1);
  c.b2 = __builtin_amdgcn_readlane(c.sbw, o + 2);
  c.b3 = __builtin_amdgcn_readlane(c.sbw, o + 3);
  c.d0 = __builtin_amdgcn_readlane(c.sdw, o);
  c.d1 = __builtin_amdgcn_readlane(c.sdw, o + 1);
  c.d2 = __builtin_amdgcn_readlane(c.sdw, o + 2);
}

// Moves the cursor to the range holding row r (r >= sb[jc]): the count of
// window entries at or below r, restarting the window when the cursor and
// the three boundaries after it would not fit in it.
__device__ __forceinline__ void seek_cursor(const int32_t* sb, const int32_t* sd, int32_t ns, int lane, int32_t r,
                                            PullCarry& c) {
  for (;;) {
    const int32_t cnt = __popcll(__ballot(c.sbw <= r));  // >= 1: sb[jw] <= r
    if (cnt <= kWave - 3) {
      c.jc = c.jw + cnt - 1;
      break;
    }
    c.jw += cnt - 1;  // advances by at least 61; entries past the table are INT32_MAX, so this ends
    load_window(sb, sd, ns, lane, c);
  }
  cursor_from_window(c);
}

// Sum over the tiles after tile q of the row open at q's end, up to its end
// (the first head bit that follows).
template <bool kVal>
__device__ double finish_open_row(const uint16_t* __restrict__ col16, const gc_head_word* __restrict__ heads,
                                  const float* __restrict__ vals, const float* slice, int32_t q, int lane) {
  double acc = 0.0;
  for (int32_t qq = q + 1;; ++qq) {
    const WaveTile u = load_wave_tile<kVal>(col16, heads, vals, qq, lane);
    const uint64_t hb = word_bits(u.hw);
    // position of the tile's first head (kWaveTile if none): lowest lane group with a set bit
    const uint64_t has = __ballot(hb != 0ull && (lane & 7) == 0);
    const int32_t grp = has ? (__ffsll(static_cast<long long>(has)) - 1) >> 3 : 8;
    const uint64_t gb = grp < 8 ? static_cast<uint64_t>(__shfl(static_cast<long long>(hb), grp * 8, kWave)) : 0ull;
    const int32_t p = grp < 8 ? 64 * grp + __ffsll(static_cast<long long>(gb)) - 1 : kWaveTile;
    double part = 0.0;
#pragma unroll
    for (int e = 0; e < kArcsPerLane; ++e)
      if (kArcsPerLane * lane + e < p)
        part += static_cast<double>(slice[(u.cols[e >> 1] >> (16 * (e & 1))) & 0xFFFFu] * arc_value<kVal>(u, e));
    acc += gcd::wave_sum(part);
    if (p < kWaveTile) return acc;  // bits past the last arc are set, so this ends
  }
}

// Keeps a tile's registers and gathered values allocated up to this point.
template <bool kVal>
__device__ __forceinline__ void hold_live(const WaveTile& t, const float (&x)[kArcsPerLane]) {
  asm volatile("" ::"v"(t.cols), "v"(t.hw));
  if (kVal) asm volatile("" ::"v"(t.va), "v"(t.vb));
#pragma unroll
  for (int e = 0; e < kArcsPerLane; ++e) asm volatile("" ::"v"(x[e]));
}

typedef __attribute__((address_space(3))) const float lds_float;

// The contributions this lane's 8 arcs gather from the block's slice (times
// the arc values in the valued pull). The kernel declares no static LDS, so
// its dynamic LDS (and the slice at its start) begins at LDS address 0: a
// column's byte offset is its address.
template <bool kVal>
__device__ __forceinline__ void gather_tile(const WaveTile& t, float (&x)[kArcsPerLane]) {
#pragma unroll
  for (int e = 0; e < kArcsPerLane; ++e) {
    const uint32_t col = (t.cols[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
    x[e] = *reinterpret_cast<lds_float*>(static_cast<uintptr_t>(col << 2));
    if (kVal) x[e] *= arc_value<kVal>(t, e);
  }
}

constexpr uint32_t kPushOut = 1u << 23;  // moves the staging slot of an arc that ends no row past every pass

// Byte offsets (past the store's base) of the stores k < nk of a staging
// pass: store k holds rows rs + i, i = lo + 64k + lane, written to index
// i + D0 / D1 / D2 below / from / past the range boundaries i1 and i2
// (kTwo: i2 lies among the rows written), dropped from iz on. The lane is
// compared with scalar thresholds; the store's base offset 4(lo + 64k)
// travels in the scalar offset operand, which the hardware leaves out of
// its range check, so a dropped lane's offset alone is past the resource.
template <bool kTwo>
__device__ __forceinline__ void row_offsets(uint32_t (&off)[kStageRows / kWave], int nk, int lane, int32_t lo,
                                            int32_t i1, int32_t i2, int32_t iz, int32_t D0, int32_t D1, int32_t D2) {
  constexpr int32_t kDropIndex = 1 << 29;  // (lane + kDropIndex) * 4 >= 2^31
#pragma unroll
  for (int k = 0; k < kStageRows / kWave; ++k) {
    if (k < nk) {
      const int32_t base = lo + k * kWave;
      const bool p1 = lane >= i1 - base, pz = lane >= iz - base;
      int32_t d = p1 ? D1 : D0;
      if (kTwo) d = lane >= i2 - base ? D2 : d;
      d = pz ? kDropIndex : d;
      off[k] = static_cast<uint32_t>(lane + d) << 2;
    }
  }
}

__device__ __forceinline__ void reduce_wave_tile(const WaveTile& t, const float (&x)[kArcsPerLane], int lane,
                                                 const int32_t* sb, const int32_t* sd, int32_t ns, int32_t r0,
                                                 int32_t r1, PullCarry& cr, __amdgpu_buffer_rsrc_t out,
                                                 float* stage) {
  const uint32_t wlo = t.hw[0], whi = t.hw[1];
  const int32_t wrow = static_cast<int32_t>(t.hw[2]);
  const int32_t ta = __builtin_amdgcn_readfirstlane(wrow);
  const int32_t tz = __builtin_amdgcn_readlane(wrow + __popc(wlo) + __popc(whi), kWave - 1);
  const uint32_t next_head = __builtin_amdgcn_readlane(static_cast<int32_t>(t.hw[3]), kWave - 1) & 1u;
  // rows the wave writes from this tile: those whose head is here and that
  // belong to the chunk, and the row left open by the previous tile
  const int32_t rz = min(tz, r1);
  const int32_t rmin = cr.open_row >= 0 ? cr.open_row : max(ta, r0);
  if (rmin < rz && rmin >= cr.b1) seek_cursor(sb, sd, ns, lane, rmin, cr);
  // this lane's 8 head bits and the head bit of the arc after them (bit 8)
  const int sub = lane & 7;
  const uint32_t wa = sub < 4 ? wlo : whi, wb = sub < 4 ? whi : t.hw[3];
  const uint32_t my9 = __builtin_amdgcn_alignbit(wb, wa, 8 * (sub & 3)) & 0x1FFu;
  const uint32_t my8 = my9 & 0xFFu;
  const int32_t first = wrow + (sub < 4 ? 0 : __popc(wlo)) + __popc(wa & ((1u << (8 * (sub & 3))) - 1u));
  // none[e]: all ones when arc e ends no row (the arc after it is no head)
  uint32_t none[kArcsPerLane];
#pragma unroll
  for (int e = 0; e < kArcsPerLane; ++e)
    none[e] = static_cast<uint32_t>(__builtin_amdgcn_sbfe(static_cast<int32_t>(~my9), e + 1, 1));
  // The lane's open sum in FP32: a run over its 8 arcs from the row's start
  // (or the lane's first arc) that carries over arc e - 1 (its bits masked
  // to +0.0 otherwise) when that arc ends no row.
  float run = x[0];
#pragma unroll
  for (int e = 1; e < kArcsPerLane; ++e) run = x[e] + __uint_as_float(__float_as_uint(run) & none[e - 1]);
  // Segmented inclusive scan of the lanes' open sums across the wave (FP32;
  // the flag of a lane is whether it holds a head). The flags live in a
  // scalar lane mask, widened after each step the way the DPP moves data.
  const uint64_t H = __ballot(my8 != 0u);
  float A = run;
  uint64_t F = H;
  seg_scan_step<kDppRowShr1, 0xF>(A, F);
  F |= (F << 1) & 0xFFFEFFFEFFFEFFFEull;
  seg_scan_step<kDppRowShr2, 0xF>(A, F);
  F |= (F << 2) & 0xFFFCFFFCFFFCFFFCull;
  seg_scan_step<kDppRowShr4, 0xF>(A, F);
  F |= (F << 4) & 0xFFF0FFF0FFF0FFF0ull;
  seg_scan_step<kDppRowShr8, 0xF>(A, F);
  F |= (F << 8) & 0xFF00FF00FF00FF00ull;
  seg_scan_step<kDppRowBcast15, 0xA>(A, F);
  F |= ((F & (1ull << 15)) ? 0x00000000FFFF0000ull : 0ull) | ((F & (1ull << 47)) ? 0xFFFF000000000000ull : 0ull);
  seg_scan_step<kDppRowBcast31, 0xC>(A, F);
  // lane l: the open sum at the end of lane l - 1, plus (in FP64) the sum
  // carried from earlier tiles when no lane before l holds a head
  const float c = dpp_moved<kDppWaveShr1, 0xF>(A);
  const uint64_t past_head = H ? ((~0ull << __builtin_ctzll(H)) << 1) : 0ull;
  const float with_open = static_cast<float>(static_cast<double>(c) + cr.open);
  const float carry = lane_in(past_head) ? c : with_open;
  // The rows this tile completes form one run [rs, re): the open row (if
  // the wave owes it) and every row of the chunk with its head here, except
  // the last one when it continues into the next tile. Their sums are
  // staged in LDS by row and written back so that store k of the wave holds
  // rows rs + 64k .. rs + 64k + 63 (coalesced); the position table turns a
  // row into its range-major index. Every lane issues the same stores
  // (unused ones get a dropped offset), so the compiler's count of
  // outstanding memory operations stays exact.
  const int32_t rs = rmin;
  const int32_t re = min(rz, next_head ? tz : tz - 1);
  // Staging slot of each arc: its row's offset from rs (as unsigned: rows
  // before rs wrap to huge values) when the arc ends its row, pushed out by
  // kPushOut otherwise. Every arc writes its run to the staging; those with
  // no row of the pass go to one of the wave's spare slots.
  uint32_t slot[kArcsPerLane];
  {
    uint32_t r = static_cast<uint32_t>(first - 1 - rs) + (my9 & 1u);  // offset of arc 0's row
#pragma unroll
    for (int e = 0; e < kArcsPerLane; ++e) {
      slot[e] = (none[e] & kPushOut) | r;  // r < 512, or wrapped past 2^31: the OR acts as an add
      r += 1u + none[e];
    }
  }
  // The staged runs: the same masked run again, now starting from the
  // carried sum unless arc 0 is a head (it reaches exactly the arcs before
  // the lane's first head, i.e. the end of the row carried into the lane;
  // an LDS atomic add of the carry to that row's slot costs more than these
  // instructions).
  float st[kArcsPerLane];
  {
    const uint32_t cont0 = static_cast<uint32_t>(__builtin_amdgcn_sbfe(static_cast<int32_t>(~my9), 0, 1));
    float r = x[0] + __uint_as_float(__float_as_uint(carry) & cont0);
    st[0] = r;
#pragma unroll
    for (int e = 1; e < kArcsPerLane; ++e) {
      r = x[e] + __uint_as_float(__float_as_uint(r) & none[e - 1]);
      st[e] = r;
    }
  }
  // rows at or past the cached boundary b3 (three or more ranges in one tile)
  // are stored on the slow path below; the others index with the cursor
  const int32_t i1 = cr.b1 - rs, i2 = cr.b2 - rs, iz = min(re, cr.b3) - rs;
  const int32_t D0 = rs + cr.d0, D1 = rs + cr.d1, D2 = rs + cr.d2;  // row rs + i goes to index i + D
  const uint32_t spare = kStageRows + (lane & (kStageSpare - 1));
  // Staging passes: rows [0, 384) of the run in every tile (6 stores),
  // rows [384, 512) only in tiles that complete more rows (a tile completes
  // at most 512). Every tile thus issues at least kStoresPerTile stores, the
  // count the compiler's memory waits assume.
  auto stage_pass = [&](auto pass_tag) {
    constexpr int pass = decltype(pass_tag)::value;
    constexpr uint32_t lo = pass == 0 ? 0u : static_cast<uint32_t>(kStageRows);
    constexpr int n = pass == 0 ? kStageRows : kTileRowsMax - kStageRows;  // rows of this pass
    // slots of the pass run [0, n); anything at or past n lands in
    // [n, n + 16), which this pass does not read back
    const uint32_t cap = spare - static_cast<uint32_t>(kStageRows - n);
#pragma unroll
    for (int e = 0; e < kArcsPerLane; ++e) stage[min(slot[e] - lo, cap)] = st[e];
    wave_lds_fence();
    float v[n / kWave];
#pragma unroll
    for (int k = 0; k < n / kWave; ++k) v[k] = stage[k * kWave + lane];
    // the offsets take one of two branches; the stores follow unconditionally
    // (stores inside the branches would leave the compiler unable to count
    // them on every path)
    uint32_t off[kStageRows / kWave];
    if (i2 < iz) row_offsets<true>(off, n / kWave, lane, static_cast<int32_t>(lo), i1, i2, iz, D0, D1, D2);
    else row_offsets<false>(off, n / kWave, lane, static_cast<int32_t>(lo), i1, i2, iz, D0, D1, D2);
#pragma unroll
    for (int k = 0; k < n / kWave; ++k)
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[k]), out, off[k], 4 * (static_cast<int32_t>(lo) + k * kWave), 0);
    wave_lds_fence();  // the staging is rewritten next
  };
  stage_pass(std::integral_constant<int, 0>());
  if (re - rs > kStageRows) stage_pass(std::integral_constant<int, 1>());  // uniform
  if (re > cr.b3) {  // uniform, rare: store the rows at or past b3
#pragma unroll
    for (int e = 0; e < kArcsPerLane; ++e) {
      const int32_t r = rs + static_cast<int32_t>(slot[e]);
      if (slot[e] < static_cast<uint32_t>(re - rs) && r >= cr.b3) {
        const int32_t j = seek_range(sb, cr.jc, r);
        partial_store(out, 4u * static_cast<uint32_t>(r + sd[j]), st[e]);
      }
    }
  }
  // the row open at the tile's end, if the wave writes it (lane 63 holds its
  // open sum; the earlier tiles' part joins in FP64)
  const float run63 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(run), kWave - 1));
  const float c63 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c), kWave - 1));
  const double tail = static_cast<double>((H >> 63) ? run63 : run63 + c63) + (H ? 0.0 : cr.open);
  const int32_t ro = tz - 1;  // the row of the tile's last arc
  const bool owe = !next_head && (tz > ta ? (ro >= r0 && ro < r1) : cr.open_row >= 0);
  cr.open_row = owe ? ro : -1;
  cr.open = owe ? tail : 0.0;
}

template <bool kVal>
__global__ __launch_bounds__(kLdsThreads) void k_pr_tocab_pull_lds(
    const int32_t* __restrict__ row_ptr, const uint16_t* __restrict__ col16,
    const gc_head_word* __restrict__ heads, const float* __restrict__ vals, const int32_t* __restrict__ chunk_beg,
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
  if (r0 >= r1) return;  // padding of the dispatch order (uniform)
  float* slice = lds;
  float* stage = lds + W + wid * (kStageRows + kStageSpare);  // this wave's output staging and spare slots
  int32_t* sb = reinterpret_cast<int32_t*>(lds + W + kLdsWaves * (kStageRows + kStageSpare));  // ns + 1 boundaries, then sentinels
  int32_t* sd = sb + ns + kSegPad;                    // ns shifts, then spares
  {
    const int32_t v0 = b << log2W;
    const int32_t cnt = min(W, n - v0);
    const float4* c4 = reinterpret_cast<const float4*>(c + v0);  // v0 is a multiple of W >= 2^10
    float4* s4 = reinterpret_cast<float4*>(slice);
    constexpr int kFill = gcx::kLdsMaxWidth / 4 / kLdsThreads;
    if (cnt == gcx::kLdsMaxWidth) {  // uniform: a full block of the widest kind
      // all of a thread's loads are issued before its first LDS write (one
      // memory round trip for the whole slice)
      float4 f[kFill];
#pragma unroll
      for (int k = 0; k < kFill; ++k) f[k] = c4[threadIdx.x + k * kLdsThreads];
#pragma unroll
      for (int k = 0; k < kFill; ++k) s4[threadIdx.x + k * kLdsThreads] = f[k];
    } else {
      for (int32_t i = threadIdx.x; i < (cnt >> 2); i += kLdsThreads) s4[i] = c4[i];
      for (int32_t i = (cnt & ~3) + threadIdx.x; i < cnt; i += kLdsThreads) slice[i] = c[v0 + i];
    }
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
  load_window(sb, sd, ns, lane, cr);
  cursor_from_window(cr);
  // Four tiles in registers: while one is reduced, the next one's gathers
  // and the two after it's loads are in flight; the tile just reduced is
  // refilled once its stores are issued, so the youngest memory operations
  // at every wait are tile loads. Its registers (and its gathered values)
  // are held live until then, so the compiler cannot hand them to the
  // stores as temporaries (a load into a register a pending store still
  // reads would wait for that store). Each tile issues exactly
  // kStoresPerTile stores, and dropped stores after the prologue's loads
  // give the compiler's count of memory operations after each load at
  // least its steady-state value on entry.
  int32_t q = qa;
  WaveTile t0 = load_wave_tile<kVal>(col16, heads, vals, q, lane);
  WaveTile t1 = load_wave_tile<kVal>(col16, heads, vals, min(q + 1, qz), lane);
  WaveTile t2 = load_wave_tile<kVal>(col16, heads, vals, min(q + 2, qz), lane);
  WaveTile t3 = load_wave_tile<kVal>(col16, heads, vals, min(q + 3, qz), lane);
  drop_stores(out);
  drop_stores(out);
  drop_stores(out);
  float x0[kArcsPerLane], x1[kArcsPerLane];
  gather_tile<kVal>(t0, x0);
  // Whole rounds of four tiles run in a loop with no exit inside (an exit
  // merged into the loop's back edge would make the compiler assume a path
  // with fewer memory operations and wait longer); the last nt % 4 tiles
  // follow it.
#define GC_PULL_STEP(cur, xcur, nxt, xnxt, k)                           \
  gather_tile<kVal>(nxt, xnxt);                                         \
  reduce_wave_tile(cur, xcur, lane, sb, sd, ns, r0, r1, cr, out, stage); \
  hold_live<kVal>(cur, xcur);                                           \
  cur = load_wave_tile<kVal>(col16, heads, vals, min(q + (k + 4), qz), lane);
  const int32_t nw = qz - qa + 1;
  for (int32_t round = 0; round < nw / 4; ++round) {
    GC_PULL_STEP(t0, x0, t1, x1, 0)
    GC_PULL_STEP(t1, x1, t2, x0, 1)
    GC_PULL_STEP(t2, x0, t3, x1, 2)
    GC_PULL_STEP(t3, x1, t0, x0, 3)
    q += 4;
  }
  const int32_t rest = nw % 4;
  if (rest > 0) {
    gather_tile<kVal>(t1, x1);
    reduce_wave_tile(t0, x0, lane, sb, sd, ns, r0, r1, cr, out, stage);
  }
  if (rest > 1) {
    gather_tile<kVal>(t2, x0);
    reduce_wave_tile(t1, x1, lane, sb, sd, ns, r0, r1, cr, out, stage);
  }
  if (rest > 2) reduce_wave_tile(t2, x0, lane, sb, sd, ns, r0, r1, cr, out, stage);
#undef GC_PULL_STEP
  if (cr.open_row >= 0) {  // the range's last row continues past it
    const double v = cr.open + finish_open_row<kVal>(col16, heads, vals, slice, qz, lane);
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
  double mine = 0.0, dl = 0.0;
  if (r0 < r1) {
    const double D = *u.dtotal_in;
    pull_tile(t_rowptr, t_col, c_in, r0, r1, vals,
              [&](int32_t v, double s) { mine += update_vertex(u, v, s, D, dl); });
  }
  publish_update(u, mine, dl);
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
  double mine = 0.0, dl = 0.0;
  for (int i = threadIdx.x; i < K; i += kThreads) {
    const int32_t v = v0 + i;
    if (v < u.n) mine += update_vertex(u, v, acc[i], D, dl);
  }
  publish_update(u, mine, dl);
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

// Accumulation part of the stream-layout merge for range blockIdx.x (NT
// threads), into acc[K] (FP64, LDS).
template <int K, int NT>
__device__ __forceinline__ void stream_accumulate(const int32_t* __restrict__ rstart,
                                                  const uint16_t* __restrict__ id16s,
                                                  const float* __restrict__ partial, double* acc) {
  for (int i = threadIdx.x; i < K; i += NT) acc[i] = 0.0;
  __syncthreads();
  const int32_t a = rstart[blockIdx.x], z = rstart[blockIdx.x + 1];
  const int32_t g0 = a >> 2, g1 = (z + 3) >> 2;  // 4-entry groups covering [a, z)
  const f32x4* p4 = reinterpret_cast<const f32x4*>(partial);
  const uint64_t* i4 = reinterpret_cast<const uint64_t*>(id16s);
  // kU groups of 4 entries per thread and step; the next step's loads are
  // issued before this step's LDS adds (two register sets in turn)
  constexpr int kU = 4;
  f32x4 pa[kU], pb[kU];
  uint64_t ia[kU], ib[kU];
  auto load = [&](int32_t g, f32x4 (&p)[kU], uint64_t (&id)[kU]) {
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int32_t gg = min(g + k * NT, g1 - 1);  // clamped, masked below
      p[k] = gcd::ld_stream(p4 + gg);
      id[k] = gcd::ld_stream(i4 + gg);
    }
  };
  auto add = [&](int32_t g, const f32x4 (&p)[kU], const uint64_t (&id)[kU]) {
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int32_t e0 = 4 * (g + k * NT);
      const float pv[4] = {p[k][0], p[k][1], p[k][2], p[k][3]};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (e0 + e >= a && e0 + e < z)
          atomicAdd(&acc[(id[k] >> (16 * e)) & 0xFFFFu], static_cast<double>(pv[e]));
    }
  };
  // (loads are clamped to the last group, so they need no branch and the
  // compiler's count of outstanding loads holds on every path)
  constexpr int32_t kStep = NT * kU;
  int32_t g = g0 + static_cast<int32_t>(threadIdx.x);
  if (g0 < g1) load(g, pa, ia);  // uniform
  for (; g < g1; g += 2 * kStep) {
    load(g + kStep, pb, ib);
    add(g, pa, ia);
    load(g + 2 * kStep, pa, ia);
    add(g + kStep, pb, ib);
  }
  __syncthreads();
}

// The stream-layout merge as a persistent kernel: one work-group per CU
// (two for ranges up to 8192 vertices) walks ranges j = blockIdx.x,
// blockIdx.x + gridDim.x, ... With one work-group per CU, a work-group per
// range would leave the CU idle while it clears its accumulator, waits for
// its first loads and updates its vertices; here the update of one range
// clears the accumulator as it reads it, and the first loads of the next
// range are issued before that update runs. One dangling partial per
// work-group (its ranges in order, so D stays reproducible).
template <int K, int NT = merge_threads<K>()>
__global__ __launch_bounds__(NT) void k_pr_merge_persist(const int32_t* __restrict__ rstart,
                                                         const uint16_t* __restrict__ id16s,
                                                         const float* __restrict__ partial, int32_t R, Update u) {
  __shared__ double acc[K];
  for (int i = threadIdx.x; i < K; i += NT) acc[i] = 0.0;
  __syncthreads();
  const f32x4* p4 = reinterpret_cast<const f32x4*>(partial);
  const uint64_t* i4 = reinterpret_cast<const uint64_t*>(id16s);
  constexpr int kU = 4;  // groups of 4 entries per thread and step (two register sets in turn)
  constexpr int32_t kStep = NT * kU;
  f32x4 pa[kU], pb[kU];
  uint64_t ia[kU], ib[kU];
  int32_t a = 0, z = 0, g0 = 0, g1 = 0;  // the current range's entries [a, z), 4-entry groups [g0, g1)
  auto bounds = [&](int32_t j) {
    a = rstart[j];
    z = rstart[j + 1];
    g0 = a >> 2;
    g1 = (z + 3) >> 2;
  };
  // (loads are clamped to the range's last group, so they need no branch
  // and the compiler's count of outstanding loads holds on every path)
  auto load = [&](int32_t g, f32x4 (&p)[kU], uint64_t (&id)[kU]) {
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int32_t gg = min(g + k * NT, g1 - 1);
      p[k] = gcd::ld_stream(p4 + gg);
      id[k] = gcd::ld_stream(i4 + gg);
    }
  };
  auto add = [&](int32_t g, const f32x4 (&p)[kU], const uint64_t (&id)[kU]) {
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int32_t e0 = 4 * (g + k * NT);
      const float pv[4] = {p[k][0], p[k][1], p[k][2], p[k][3]};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (e0 + e >= a && e0 + e < z) atomicAdd(&acc[(id[k] >> (16 * e)) & 0xFFFFu], static_cast<double>(pv[e]));
    }
  };
  const double D = *u.dtotal_in;
  double mine = 0.0, dl = 0.0;
  const int32_t tid = threadIdx.x;
  int32_t j = blockIdx.x;
  if (j < R) {
    bounds(j);
    if (g0 < g1) load(g0 + tid, pa, ia);  // uniform
  }
  for (; j < R; j += gridDim.x) {
    for (int32_t g = g0 + tid; g < g1; g += 2 * kStep) {
      load(g + kStep, pb, ib);
      add(g, pa, ia);
      load(g + 2 * kStep, pa, ia);
      add(g + kStep, pb, ib);
    }
    __syncthreads();
    const int32_t v0 = j * K;
    // The range's out-degrees (and previous ranks in convergence mode) are
    // loaded into registers before the next range's first partials: the
    // wait for them then does not wait for those, and the update below
    // runs on registers (a load per vertex inside it made every one of its
    // steps a memory round trip).
    constexpr int kPer = (K + NT - 1) / NT;
    int32_t deg[kPer];
    float prev[kPer];
    // vertex v0 + tid + q NT, clamped to the last vertex (those past it are not updated)
    const uint32_t last = static_cast<uint32_t>(u.n - 1 - v0);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const uint32_t o = min(static_cast<uint32_t>(tid + q * NT), last);
      const int32_t* rp = u.rowptr + v0;  // uniform base, 32-bit offsets
      deg[q] = rp[o + 1] - rp[o];
      prev[q] = 0.0f;
    }
    if (u.rank_prev) {
      const float* pp = u.rank_prev + v0;
#pragma unroll
      for (int q = 0; q < kPer; ++q) prev[q] = pp[min(static_cast<uint32_t>(tid + q * NT), last)];
    }
    const int32_t jn = j + gridDim.x;
    if (jn < R) {  // uniform: the next range's first loads, in flight during the update
      bounds(jn);
      if (g0 < g1) load(g0 + tid, pa, ia);
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int32_t i = tid + q * NT;
      if (K % NT != 0 && i >= K) break;
      const int32_t v = v0 + i;
      float cv;
      if (v < u.n) mine += update_vertex_loaded(u, v, acc[i], D, dl, cv, deg[q], prev[q]);
      acc[i] = 0.0;
    }
    __syncthreads();
  }
  publish_update<NT>(u, mine, dl);
}

// Work-groups of the persistent merge over R ranges of K vertices.
int32_t merge_persist_grid(int32_t K, int32_t R) {
  return std::max(1, std::min(R, (K >= 16384 ? 1 : 2) * g_cus));
}


// The same merge for SpMV: y[v] = the FP64 sum rounded to FP32.
template <int K, int kMergeThreads = merge_threads<K>()>
__global__ __launch_bounds__(kMergeThreads) void k_spmv_merge_stream(const int32_t* __restrict__ rstart,
                                                                     const uint16_t* __restrict__ id16s,
                                                                     const float* __restrict__ partial, int32_t n,
                                                                     float* __restrict__ y) {
  __shared__ double acc[K];
  stream_accumulate<K, kMergeThreads>(rstart, id16s, partial, acc);
  const int32_t v0 = blockIdx.x * K;
  for (int i = threadIdx.x; i < K; i += kMergeThreads)
    if (v0 + i < n) y[v0 + i] = static_cast<float>(acc[i]);
}

// Padded FP32 arc values in the partition's arc order: FP32 bit patterns or
// integers converted, zero past the last arc.
__global__ void k_stream_values(const int32_t* __restrict__ w, bool f32, int64_t m, int64_t m_pad,
                                float* __restrict__ out) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m_pad; i += stride) {
    float v = 0.0f;
    if (i < m) v = f32 ? __int_as_float(w[i]) : static_cast<float>(w[i]);
    out[i] = v;
  }
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

// Algorithm 5 with the destination block's sums in LDS: in a push partition
// block s holds every arc into destinations [sW, (s+1)W), so work-group s
// adds each of its local rows' contribution c[id_map[l]] into FP64 LDS sums
// (W <= kPushLdsMaxWidth: 128 KB), then applies the update to its whole
// range itself: no global atomics and no separate apply pass. A thread takes
// whole rows (a (source, block) pair holds few arcs). c is read from one
// buffer and the next iteration's contributions go to u.contrib, another.
// (Form used for partitions without the expanded contributions below.)
using gcx::kPushLdsMaxWidth;
constexpr int kPushLdsThreads = 1024;

__global__ __launch_bounds__(kPushLdsThreads) void k_pr_push_lds(const int32_t* __restrict__ blk_rowoff,
                                                                 const int32_t* __restrict__ row_ptr,
                                                                 const int32_t* __restrict__ id_map,
                                                                 const int32_t* __restrict__ col, int32_t log2W,
                                                                 const float* __restrict__ c, Update u) {
  extern __shared__ double acc[];  // the block's W sums
  const int32_t W = 1 << log2W;
  const int32_t v0 = static_cast<int32_t>(blockIdx.x) << log2W;
  for (int32_t i = threadIdx.x; i < W; i += kPushLdsThreads) acc[i] = 0.0;
  __syncthreads();
  const int32_t r0 = blk_rowoff[blockIdx.x], r1 = blk_rowoff[blockIdx.x + 1];
  // kRows rows per thread and step, their loads issued together (row
  // bounds and ids, then the contributions, then each row's first arc: a
  // local row has at least one); rows past r1 reuse the last row, masked
  constexpr int kRows = 4;
  for (int32_t r = r0 + threadIdx.x; r < r1; r += kRows * kPushLdsThreads) {
    int32_t b[kRows], e[kRows], id[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int32_t rk = min(r + k * kPushLdsThreads, r1 - 1);
      b[k] = row_ptr[rk];
      e[k] = row_ptr[rk + 1];
      id[k] = id_map[rk];
    }
    float x[kRows];
    int32_t c0[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      x[k] = c[id[k]];
      c0[k] = col[b[k]];
    }
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      if (r + k * kPushLdsThreads < r1) {
        const double xk = static_cast<double>(x[k]);
        atomicAdd(&acc[c0[k] - v0], xk);
        for (int32_t a = b[k] + 1; a < e[k]; ++a) atomicAdd(&acc[col[a] - v0], xk);
      }
    }
  }
  __syncthreads();
  const double D = *u.dtotal_in;
  double mine = 0.0, dl = 0.0;
  for (int32_t i = threadIdx.x; i < W; i += kPushLdsThreads) {
    const int32_t v = v0 + i;
    if (v < u.n) mine += update_vertex(u, v, acc[i], D, dl);
  }
  publish_update<kPushLdsThreads>(u, mine, dl);
}

// The TOCAB push with expanded contributions. Reading c[id_map[l]] for
// every local row l is a random 4-byte read per row, and on this GPU each
// one moves a whole cache line from the Infinity Cache or HBM (about 120
// bytes per row measured at R-MAT 24): the push spent its time there, not
// in its LDS atomics. Instead every row's contribution sits at xc[l], in row
// order, written by the work-group that produced it: after updating the
// vertices of its block (source block s = destination block s), a
// work-group keeps their new contributions in LDS and writes them to the
// run of rows in every block whose source lies in block s.

// Where the expanded contributions go (see gc_tocab_s): the range table,
// the rows' source offsets and, for short runs, the source-major list.
struct PushX {
  const int32_t* range_ptr;
  int32_t B, R, shift;  // shift = log2(W / k)
  const uint16_t* xid16;
  const int32_t* xperm;   // null: long runs, walked in place
  const int32_t* xstart;
};

// Contributions of rows r .. r + 3 (a group of four, 16-byte aligned)
// inside the run [st, en): one 16-byte store when the group lies inside it.
__device__ __forceinline__ void push_store4(float* __restrict__ xc_out, int32_t r, int32_t st, int32_t en,
                                            uint64_t id, const float* cs) {
  if (r >= st && r + 3 < en) {
    f32x4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = cs[(id >> (16 * e)) & 0xFFFFu];
    *reinterpret_cast<f32x4*>(xc_out + r) = v;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (r + e >= st && r + e < en) xc_out[r + e] = cs[(id >> (16 * e)) & 0xFFFFu];
  }
}

// Writes the contributions of source block s (cs: in LDS) to the rows of
// every block whose source lies in it; tbl: LDS room for 2B int32.
// Long runs: the run bounds go to LDS and a wave takes kU runs at a time,
// its lanes side by side along each, rows in groups of four (one 8-byte
// read of their offsets, one 16-byte store), so every lane keeps kU reads
// in flight. Short runs: threads stride over the source-major list of the
// block (a read of the row and of its offset per position).
template <int NT>
__device__ __forceinline__ void push_expand(const PushX& x, int32_t s, const float* cs, int32_t* tbl,
                                            float* __restrict__ xc_out) {
  constexpr int kWaves = NT / kWave, kU = 8;
  if (x.xperm) {  // uniform
    const int32_t q0 = x.xstart[s], q1 = x.xstart[s + 1];
    constexpr int kV = 4;  // positions per thread and step, loads issued together
    for (int32_t q = q0 + static_cast<int32_t>(threadIdx.x); q < q1; q += kV * NT) {
      int32_t r[kV];
      uint32_t o[kV];
#pragma unroll
      for (int k = 0; k < kV; ++k) {
        const int32_t qq = min(q + k * NT, q1 - 1);
        r[k] = gcd::ld_stream(x.xperm + qq);
        o[k] = gcd::ld_stream(x.xid16 + qq);
      }
#pragma unroll
      for (int k = 0; k < kV; ++k)
        if (q + k * NT < q1) xc_out[r[k]] = cs[o[k]];
    }
    return;
  }
  const int32_t B = x.B;
  int32_t* lo = tbl;
  int32_t* hi = tbl + B;
  {
    const int64_t j0 = static_cast<int64_t>(s) << x.shift;
    const int64_t j1 = min<int64_t>(x.R, (static_cast<int64_t>(s) + 1) << x.shift);
    for (int32_t b = threadIdx.x; b < B; b += NT) {
      lo[b] = x.range_ptr[j0 * B + b];
      hi[b] = x.range_ptr[j1 * B + b];
    }
  }
  __syncthreads();
  const uint64_t* x4 = reinterpret_cast<const uint64_t*>(x.xid16);
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t wid = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(threadIdx.x) / kWave);
  for (int32_t b0 = wid * kU; b0 < B; b0 += kWaves * kU) {  // uniform
    int32_t g0[kU], st[kU], en[kU], ng[kU];
    int32_t gmax = 0;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int32_t b = b0 + u;
      st[u] = b < B ? lo[b] : 0;
      en[u] = b < B ? hi[b] : 0;
      g0[u] = st[u] >> 2;  // groups of four rows covering the run
      ng[u] = en[u] > st[u] ? ((en[u] - 1) >> 2) - g0[u] + 1 : 0;
      gmax = max(gmax, ng[u]);
    }
    for (int32_t k = 0; k < gmax; k += kWave) {  // uniform
      uint64_t id[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) id[u] = gcd::ld_stream(x4 + g0[u] + min(k + lane, max(ng[u] - 1, 0)));
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (k + lane < ng[u]) push_store4(xc_out, 4 * (g0[u] + k + lane), st[u], en[u], id[u], cs);
    }
  }
}

PushX push_x(gc_tocab t) {
  return PushX{t->range_ptr, t->B, t->R, t->log2W - t->log2k, t->xid16, t->xperm, t->xstart};
}

// Dynamic LDS of the expanded push kernels: the block's FP64 sums, or its
// FP32 contributions followed by the run bounds of every block.
__host__ __device__ constexpr size_t push_x_lds(int32_t W, int32_t B) {
  return 8 * static_cast<size_t>(W) > 4 * static_cast<size_t>(W) + 8 * static_cast<size_t>(B)
             ? 8 * static_cast<size_t>(W)
             : 4 * static_cast<size_t>(W) + 8 * static_cast<size_t>(B);
}

// The expanded contributions of the starting vector: work-group s stages
// c[sW, sW + W) in LDS and writes them to the rows of source block s.
__global__ __launch_bounds__(kPushLdsThreads) void k_pr_push_expand(PushX x, int32_t log2W, int32_t n,
                                                                    const float* __restrict__ c,
                                                                    float* __restrict__ xc_out) {
  extern __shared__ float cs[];
  const int32_t W = 1 << log2W;
  const int32_t v0 = static_cast<int32_t>(blockIdx.x) << log2W;
  const int32_t cnt = min(W, n - v0);
  for (int32_t i = threadIdx.x; i < cnt; i += kPushLdsThreads) cs[i] = c[v0 + i];
  __syncthreads();
  push_expand<kPushLdsThreads>(x, blockIdx.x, cs, reinterpret_cast<int32_t*>(cs + W), xc_out);
}

// One iteration of the TOCAB push over expanded contributions: block s's
// sums in FP64 LDS, then the update of its W vertices, then their
// contributions expanded into xc_out. The sums walk the block's arcs as
// streams, 512-arc tiles per wave (8 consecutive arcs per lane): an arc's
// destination offset comes from the 16-bit column stream, its local row from
// the head bits (rows starting before the arc, counted with popcounts of the
// tile's head words), and the row's contribution from xc_in (neighbouring
// arcs read neighbouring rows, so these loads stay in cache). One thread per
// local row instead would serialise the arcs of long rows (a source with
// many arcs into the block) behind one lane while the rest of its wave waits.
__global__ __launch_bounds__(kPushLdsThreads) void k_pr_push_lds_x(
    const int32_t* __restrict__ blk_rowoff, const int32_t* __restrict__ row_ptr,
    const uint16_t* __restrict__ pcol16, const gc_head_word* __restrict__ pheads, int32_t log2W,
    const float* __restrict__ xc_in, PushX x, float* __restrict__ xc_out, Update u) {
  extern __shared__ double acc[];  // the block's W sums, then (as FP32) its W new contributions
  constexpr int kPer = kPushLdsMaxWidth / kPushLdsThreads;
  constexpr int kWaves = kPushLdsThreads / kWave;
  const int32_t W = 1 << log2W;
  const int32_t v0 = static_cast<int32_t>(blockIdx.x) << log2W;
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t wid = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(threadIdx.x) / kWave);
  for (int32_t i = threadIdx.x; i < W; i += kPushLdsThreads) acc[i] = 0.0;
  __syncthreads();
  const int32_t r0 = blk_rowoff[blockIdx.x], r1 = blk_rowoff[blockIdx.x + 1];
  const int32_t A0 = row_ptr[r0], A1 = row_ptr[r1];  // the block's arcs
  if (A1 > A0) {  // uniform
    const int32_t q1 = (A1 - 1) / kWaveTile;
    const int sub = lane & 7;  // this lane's 8 arcs are bits 8 sub .. 8 sub + 7 of its head word
    int32_t q = A0 / kWaveTile + wid;
    WaveTile cur = load_wave_tile<false>(pcol16, pheads, nullptr, min(q, q1), lane);
    for (; q <= q1; q += kWaves) {
      const uint64_t bits = word_bits(cur.hw);
      const uint32_t my8 = static_cast<uint32_t>(bits >> (8 * sub)) & 0xFFu;
      // the row of arc e: rows starting at or before it, minus one
      const int32_t base = static_cast<int32_t>(cur.hw[2]) - 1 + __popcll(bits & ((1ull << (8 * sub)) - 1ull));
      const int32_t a0 = q * kWaveTile + kArcsPerLane * lane;
      float x[kArcsPerLane];
      uint32_t d[kArcsPerLane];
#pragma unroll
      for (int e = 0; e < kArcsPerLane; ++e) {
        const bool ok = a0 + e >= A0 && a0 + e < A1;
        const int32_t row = ok ? base + __popc(my8 & ((2u << e) - 1u)) : r0;
        x[e] = xc_in[row];
        d[e] = ok ? (cur.cols[e >> 1] >> (16 * (e & 1))) & 0xFFFFu : 0xFFFFFFFFu;
      }
      cur = load_wave_tile<false>(pcol16, pheads, nullptr, min(q + kWaves, q1), lane);
#pragma unroll
      for (int e = 0; e < kArcsPerLane; ++e)
        if (d[e] != 0xFFFFFFFFu) atomicAdd(&acc[d[e]], static_cast<double>(x[e]));
    }
  }
  __syncthreads();
  const double D = *u.dtotal_in;
  double mine = 0.0, dl = 0.0;
  // the block's out-degrees (and previous ranks) in registers first, then
  // the update on them (a load per vertex inside it is a round trip per step)
  int32_t deg[kPer];
  float prev[kPer], cv[kPer];
  const uint32_t last = static_cast<uint32_t>(u.n - 1 - v0);  // v0 < n: the block has vertices
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t o = min(static_cast<uint32_t>(threadIdx.x + k * kPushLdsThreads), last);
    const int32_t* rp = u.rowptr + v0;
    deg[k] = rp[o + 1] - rp[o];
    prev[k] = 0.0f;
  }
  if (u.rank_prev) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) prev[k] = u.rank_prev[v0 + min(static_cast<uint32_t>(threadIdx.x + k * kPushLdsThreads), last)];
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int32_t i = threadIdx.x + k * kPushLdsThreads;
    cv[k] = 0.0f;
    if (i < W && v0 + i < u.n) mine += update_vertex_loaded(u, v0 + i, acc[i], D, dl, cv[k], deg[k], prev[k]);
  }
  __syncthreads();  // every sum has been read: the LDS now holds the contributions and the run bounds
  float* cs = reinterpret_cast<float*>(acc);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int32_t i = threadIdx.x + k * kPushLdsThreads;
    if (i < W) cs[i] = cv[k];
  }
  __syncthreads();
  publish_update<kPushLdsThreads>(u, mine, dl);
  push_expand<kPushLdsThreads>(x, blockIdx.x, cs, reinterpret_cast<int32_t*>(cs + W), xc_out);
}

__global__ __launch_bounds__(kThreads) void k_pr_apply(double* __restrict__ sums, Update u) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  const double D = *u.dtotal_in;
  double mine = 0.0, dl = 0.0;
  if (v < u.n) {
    const double s = sums[v];
    sums[v] = 0.0;
    mine = update_vertex(u, v, s, D, dl);
  }
  publish_update(u, mine, dl);
}

// ---- the baselines of Section 4's comparison (Base, VWC, conventional
// cache blocking), each with the same FP64 row sums and fused update ----

// Base: a straightforward pull, one lane per destination summing its
// in-arcs serially (Algorithm 1 as written).
__global__ __launch_bounds__(kThreads) void k_pr_base(const int32_t* __restrict__ t_rowptr,
                                                      const int32_t* __restrict__ t_col,
                                                      const float* __restrict__ c_in, Update u) {
  const int32_t v = blockIdx.x * kThreads + threadIdx.x;
  double mine = 0.0, dl = 0.0;
  if (v < u.n) {
    const double D = *u.dtotal_in;
    double s = 0.0;
    for (int32_t i = t_rowptr[v]; i < t_rowptr[v + 1]; ++i) s += static_cast<double>(c_in[t_col[i]]);
    mine = update_vertex(u, v, s, D, dl);
  }
  publish_update(u, mine, dl);
}

// VWC (the virtual-warp-centric mapping of Section 2.1): VW lanes per
// destination stride over its in-arcs, then reduce by lane exchanges. Each
// work-group walks vertex groups of 256 / VW with a uniform loop, so the grid
// (and the number of dangling partials) matches Base's.
template <int VW>
__global__ __launch_bounds__(kThreads) void k_pr_vwc(const int32_t* __restrict__ t_rowptr,
                                                     const int32_t* __restrict__ t_col,
                                                     const float* __restrict__ c_in, Update u) {
  constexpr int32_t kPerGroup = kThreads / VW;
  const int lane = threadIdx.x & (VW - 1);
  const double D = *u.dtotal_in;
  double mine = 0.0, dl = 0.0;
  for (int32_t v0 = blockIdx.x * kPerGroup; v0 < u.n; v0 += gridDim.x * kPerGroup) {
    const int32_t v = v0 + static_cast<int32_t>(threadIdx.x) / VW;
    double s = 0.0;
    if (v < u.n)
      for (int32_t i = t_rowptr[v] + lane; i < t_rowptr[v + 1]; i += VW) s += static_cast<double>(c_in[t_col[i]]);
#pragma unroll
    for (int o = VW / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, VW);
    if (lane == 0 && v < u.n) mine += update_vertex(u, v, s, D, dl);
  }
  publish_update(u, mine, dl);
}

// Conventional column blocking (the naive scheme Section 3.1 starts from):
// the blocks of a pull partition run one launch after another; a lane per
// local row of the block adds the row's sum over the block's arcs straight
// into sums[id_map[l]] (FP64 read-modify-write: a destination appears once
// per block and blocks do not overlap in time). The scattered updates of
// sums are the cost TOCAB's partials and merge avoid.
__global__ __launch_bounds__(kThreads) void k_pr_cb_block(const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ id_map,
                                                          const int32_t* __restrict__ col,
                                                          const float* __restrict__ c, double* __restrict__ sums,
                                                          int32_t a, int32_t b) {
  const int32_t l = a + static_cast<int32_t>(blockIdx.x) * kThreads + static_cast<int32_t>(threadIdx.x);
  if (l < b) {
    double s = 0.0;
    for (int32_t i = row_ptr[l]; i < row_ptr[l + 1]; ++i) s += static_cast<double>(c[col[i]]);
    sums[id_map[l]] += s;
  }
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
  {
    int dev = 0;
    GC_HIP_TRY(hipGetDevice(&dev));
    GC_HIP_TRY(hipDeviceGetAttribute(&g_cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  // the LDS-resident pull holds a slice of up to kLdsMaxWidth floats plus its
  // position table; the LDS push a block's kPushLdsMaxWidth FP64 sums
  GC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pr_push_lds),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 static_cast<int>(sizeof(double)) * kPushLdsMaxWidth));
  constexpr int kPushXLds = static_cast<int>(push_x_lds(kPushLdsMaxWidth, gcx::kPushExpandMaxBlocks));
  static_assert(kPushXLds <= 160 * 1024 - 1024, "expanded push LDS");
  GC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pr_push_lds_x),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kPushXLds));
  GC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pr_push_expand),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kPushXLds));
  GC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pr_tocab_pull_lds<false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds_budget(kLdsMaxWidth)));
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pr_tocab_pull_lds<true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds_budget(kLdsMaxWidth));
}

// Bytes of dynamic LDS the stream-layout pull takes for partition t.
size_t pull_lds_bytes(gc_tocab t) {
  return sizeof(float) * (static_cast<size_t>(t->W) + 2 * static_cast<size_t>(t->seg_max) + 2 * kSegPad) +
         kLdsStageBytes;
}

// SpMV over a stream-layout partition: the LDS-resident pull (valued when
// vals is given, unit values otherwise) and the range-major merge writing y.
hipError_t spmv_stream(gc_graph g, gc_tocab t, const float* x, const float* vals, float* y, hipStream_t s) {
  static const hipError_t setup = pagerank_setup();
  GC_HIP_TRY(setup);
  {
    ProfScope prof("spmv_tocab", s);
    if (t->n_chunks > 0) {
      const uint32_t bytes = static_cast<uint32_t>(sizeof(float) * (t->P + 8));
      if (vals)
        k_pr_tocab_pull_lds<true><<<t->n_chunks, kLdsThreads, pull_lds_bytes(t), s>>>(
            t->row_ptr, t->col16, t->heads, vals, t->chunk_beg, t->chunk_end, t->chunk_blk, t->chunk_j0,
            t->chunk_ns, t->seg, t->R, t->log2W, g->n, x, t->partial, bytes);
      else
        k_pr_tocab_pull_lds<false><<<t->n_chunks, kLdsThreads, pull_lds_bytes(t), s>>>(
            t->row_ptr, t->col16, t->heads, nullptr, t->chunk_beg, t->chunk_end, t->chunk_blk, t->chunk_j0,
            t->chunk_ns, t->seg, t->R, t->log2W, g->n, x, t->partial, bytes);
    }
  }
  ProfScope prof("spmv_merge", s);
  switch (t->k) {
    case 256: k_spmv_merge_stream<256><<<t->R, merge_threads<256>(), 0, s>>>(t->rstart, t->id16s, t->partial, g->n, y); break;
    case 512: k_spmv_merge_stream<512><<<t->R, merge_threads<512>(), 0, s>>>(t->rstart, t->id16s, t->partial, g->n, y); break;
    case 1024: k_spmv_merge_stream<1024><<<t->R, merge_threads<1024>(), 0, s>>>(t->rstart, t->id16s, t->partial, g->n, y); break;
    case 2048: k_spmv_merge_stream<2048><<<t->R, merge_threads<2048>(), 0, s>>>(t->rstart, t->id16s, t->partial, g->n, y); break;
    case 4096: k_spmv_merge_stream<4096><<<t->R, merge_threads<4096>(), 0, s>>>(t->rstart, t->id16s, t->partial, g->n, y); break;
    case 8192: k_spmv_merge_stream<8192><<<t->R, merge_threads<8192>(), 0, s>>>(t->rstart, t->id16s, t->partial, g->n, y); break;
    case 16384: k_spmv_merge_stream<16384><<<t->R, merge_threads<16384>(), 0, s>>>(t->rstart, t->id16s, t->partial, g->n, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The padded FP32 arc values of a weighted stream-layout partition (t->val32),
// built by the first valued SpMV over it.
hipError_t stream_values(gc_graph g, gc_tocab t, hipStream_t s) {
  if (t->val32) return hipSuccess;
  t->val32 = static_cast<float*>(dev_alloc(sizeof(float) * static_cast<size_t>(t->m_pad), s));
  if (!t->val32) return hipErrorOutOfMemory;
  k_stream_values<<<4096, kThreads, 0, s>>>(t->w, g->values_f32, t->m, t->m_pad, t->val32);
  return hipGetLastError();
}

// The comparison baselines (pagerank_ladder): Base and VWC gather over the
// whole transposed graph with two contribution buffers in turn; CB runs its
// block launches into the FP64 sums and then the push-side update.
hipError_t ladder_run(gc_graph g, gc_tocab t, int32_t method, float damping, int32_t dangling,
                      const float* rank_in, float* rank_out, int32_t iters, hipStream_t s) {
  const int32_t n = g->n;
  const bool cb = method == GC_LADDER_CB;
  Update u;
  u.d = damping;
  u.base = (1.0 - static_cast<double>(damping)) / n;
  u.inv_n = dangling == GC_DANGLING_UNIFORM ? 1.0 / n : 0.0;
  u.dpart = g->dpart;
  u.rowptr = g->rowptr;
  u.n = n;
  u.rank_out = nullptr;
  const int vgrid = (n + kThreads - 1) / kThreads;
  std::vector<int32_t> rows;  // CB: first local row of every block
  if (cb) {
    rows.resize(static_cast<size_t>(t->B) + 1);
    GC_HIP_TRY(hipMemcpyAsync(rows.data(), t->blk_rowoff, sizeof(int32_t) * rows.size(), hipMemcpyDeviceToHost, s));
    GC_HIP_TRY(hipStreamSynchronize(s));
  }
  u.dtotal_in = nullptr;
  u.contrib = g->contrib[0];
  k_pr_init<<<vgrid, kThreads, 0, s>>>(rank_in, u, cb ? g->sums : nullptr);
  k_reduce_dangling<<<1, 1024, 0, s>>>(g->dpart, vgrid, g->dtotal, nullptr, nullptr);
  GC_HIP_TRY(hipGetLastError());
  int cur = 0;
  for (int32_t it = 0; it < iters; ++it) {
    u.dtotal_in = g->dtotal + (it & 1);
    u.rank_out = (it == iters - 1) ? rank_out : nullptr;
    if (cb) {
      {
        ProfScope prof("pr_cb_blocks", s);
        for (int32_t b = 0; b < t->B; ++b) {
          const int32_t a = rows[b], z = rows[b + 1];
          if (z > a)
            k_pr_cb_block<<<(z - a + kThreads - 1) / kThreads, kThreads, 0, s>>>(t->row_ptr, t->id_map, t->col,
                                                                                g->contrib[0], g->sums, a, z);
        }
      }
      u.contrib = g->contrib[0];
      ProfScope prof("pr_apply", s);
      k_pr_apply<<<vgrid, kThreads, 0, s>>>(g->sums, u);
    } else {
      u.contrib = g->contrib[cur ^ 1];
      if (method == GC_LADDER_BASE) {
        ProfScope prof("pr_base", s);
        k_pr_base<<<vgrid, kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, g->contrib[cur], u);
      } else if (method == GC_LADDER_VWC) {
        ProfScope prof("pr_vwc", s);
        k_pr_vwc<8><<<vgrid, kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, g->contrib[cur], u);
      } else {
        ProfScope prof("pr_vwc64", s);
        k_pr_vwc<64><<<vgrid, kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, g->contrib[cur], u);
      }
      cur ^= 1;
    }
    {
      ProfScope prof("pr_dangling", s);
      k_reduce_dangling<<<1, 1024, 0, s>>>(g->dpart, vgrid, g->dtotal + ((it + 1) & 1), nullptr, nullptr);
    }
    GC_HIP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

// PageRank's working-set choice among the scheduler's actions (0 plain
// push, 1 plain pull, 2 + i TOCAB pull over parts[i]): every vertex is
// active, so the rule blocks whenever a partition is attached, over the
// width nearest the paper's 2^18; plain pull otherwise.
int32_t pagerank_fallback_action(const gc_tocab* parts, int32_t n_parts) {
  int32_t a = 1, best = INT32_MAX;
  for (int32_t j = 0; j < n_parts; ++j) {
    const int32_t d = std::abs(parts[j]->log2W - 18);
    if (d < best) {
      best = d;
      a = 2 + j;
    }
  }
  return a;
}

// Training rows of the level scheduler for PageRank, an all-active level
// whose cost does not change from one iteration to the next: for each row,
// every action runs kCollectIters iterations from the same ranks (0 plain
// push, 1 plain pull, 2 + i TOCAB pull over parts[i]), timed with HIP
// events (ms per iteration); the next row starts from the fastest action's
// output. Features: frontier = all n vertices and m arcs, level 1, prior
// time = the working-set rule's form's time per iteration (over m arcs),
// which is what pagerank_learned measures before it decides.
hipError_t collect_pagerank(gc_graph g, gc_tocab* parts, int32_t n_parts, int32_t n_rows, float* features,
                            float* times, int32_t max_rows, int32_t* rows, hipStream_t s) {
  constexpr int32_t kCollectIters = 4;
  const int32_t n = g->n;
  const int32_t K = 2 + n_parts;
  const int32_t fa = pagerank_fallback_action(parts, n_parts);
  Buf ra(sizeof(float) * n, s), rb(sizeof(float) * n, s), rbest(sizeof(float) * n, s);
  if (!ra.p || !rb.p || !rbest.p) return hipErrorOutOfMemory;
  std::vector<float> init(static_cast<size_t>(n), 1.0f / static_cast<float>(n));
  GC_HIP_TRY(hipMemcpyAsync(ra.p, init.data(), sizeof(float) * n, hipMemcpyHostToDevice, s));
  GC_HIP_TRY(hipStreamSynchronize(s));
  hipEvent_t e0, e1;
  GC_HIP_TRY(hipEventCreate(&e0));
  GC_HIP_TRY(hipEventCreate(&e1));
  hipError_t err = hipSuccess;
  int32_t r = 0;
  for (; r < n_rows && r < max_rows && err == hipSuccess; ++r) {
    float* row_t = times + static_cast<size_t>(r) * K;
    int32_t best = 0;
    for (int32_t a = 0; a < K && err == hipSuccess; ++a) {
      gc_tocab t = a >= 2 ? parts[a - 2] : nullptr;
      const int32_t dir = a == 0 ? GC_PUSH : GC_PULL;
      err = hipEventRecord(e0, s);
      if (err == hipSuccess)
        err = pagerank_run(g, t, dir, 0.85f, GC_DANGLING_UNIFORM, ra.as<float>(), rb.as<float>(), kCollectIters, s);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      row_t[a] = ms / kCollectIters;
      if (row_t[a] < row_t[best]) best = a;
      if (err == hipSuccess && best == a)
        err = hipMemcpyAsync(rbest.p, rb.p, sizeof(float) * n, hipMemcpyDeviceToDevice, s);
    }
    sched_features(n, g->m, n, g->m, 1, row_t[fa], g->m, features + static_cast<size_t>(r) * GC_SCHED_INPUTS);
    if (err == hipSuccess) err = hipMemcpyAsync(ra.p, rbest.p, sizeof(float) * n, hipMemcpyDeviceToDevice, s);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *rows = r;
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  return err;
}

hipError_t pagerank_run(gc_graph g, gc_tocab t, int32_t dir, float damping, int32_t dangling,
                        const float* rank_in, float* rank_out, int32_t iters, hipStream_t s, Converge* cv,
                        int32_t ladder, const PrBuffers* bufs) {
  const int32_t n = g->n;
  const PrBuffers buf = bufs ? *bufs : PrBuffers{{g->contrib[0], g->contrib[1]}, g->sums, g->dpart, g->dtotal,
                                                 t ? t->partial : nullptr};
  if (cv) iters = cv->max_iters;
  if (iters == 0)
    return hipMemcpyAsync(rank_out, rank_in, sizeof(float) * n, hipMemcpyDeviceToDevice, s);
  static const hipError_t setup = pagerank_setup();
  GC_HIP_TRY(setup);
  if (ladder >= 0) return ladder_run(g, t, ladder, damping, dangling, rank_in, rank_out, iters, s);
  const bool push = t ? (t->dir == GC_PUSH) : (dir == GC_PUSH);
  Update u;
  u.d = damping;
  u.base = (1.0 - static_cast<double>(damping)) / n;
  u.inv_n = dangling == GC_DANGLING_UNIFORM ? 1.0 / n : 0.0;
  u.dpart = buf.dpart;
  u.rowptr = g->rowptr;
  u.n = n;
  u.rank_out = nullptr;
  const int vgrid = (n + kThreads - 1) / kThreads;

  // contributions of rank_in and D of iteration 0 -> dtotal[0]
  u.dtotal_in = nullptr;
  u.contrib = buf.contrib[0];
  const bool expanded = push && t && t->W <= kPushLdsMaxWidth && t->xc;
  {
    ProfScope prof("pr_init", s);
    k_pr_init<<<vgrid, kThreads, 0, s>>>(rank_in, u, push && !expanded ? buf.sums : nullptr);
    if (expanded)
      k_pr_push_expand<<<t->n_sblk, kPushLdsThreads, push_x_lds(t->W, t->B), s>>>(push_x(t), t->log2W, n,
                                                                                 buf.contrib[0], t->xc);
  }
  k_reduce_dangling<<<1, 1024, 0, s>>>(buf.dpart, vgrid, buf.dtotal, nullptr, nullptr);
  GC_HIP_TRY(hipGetLastError());

  // convergence mode: iterates alternate between rank_out and rank_tmp,
  // each compared with the one before it
  float* const iterate[2] = {rank_out, cv ? g->rank_tmp : nullptr};
  if (cv) u.lpart = g->lpart;
  int cur = 0;
  for (int32_t it = 0; it < iters; ++it) {
    u.dtotal_in = buf.dtotal + (it & 1);
    double* dtotal_out = buf.dtotal + ((it + 1) & 1);
    u.rank_out = (it == iters - 1) ? rank_out : nullptr;
    if (cv) {
      u.rank_out = iterate[it & 1];
      u.rank_prev = it == 0 ? rank_in : iterate[(it - 1) & 1];
    }
    int32_t parts = vgrid;  // work-groups of the update kernel
    if (t && !push) {
      if (t->col16) {
        {
          ProfScope prof("pr_tocab_pull", s);
          if (t->n_chunks > 0)
            k_pr_tocab_pull_lds<false><<<t->n_chunks, kLdsThreads, pull_lds_bytes(t), s>>>(
                t->row_ptr, t->col16, t->heads, nullptr, t->chunk_beg, t->chunk_end, t->chunk_blk, t->chunk_j0,
                t->chunk_ns, t->seg, t->R, t->log2W, n, buf.contrib[0], buf.partial,
                static_cast<uint32_t>(sizeof(float) * (t->P + 8)));
        }
        u.contrib = buf.contrib[0];
        ProfScope prof("pr_merge", s);
        const int32_t mg = merge_persist_grid(t->k, t->R);
        switch (t->k) {
#define GC_MERGE(K) \
  case K: k_pr_merge_persist<K><<<mg, merge_threads<K>(), 0, s>>>(t->rstart, t->id16s, buf.partial, t->R, u); break;
          GC_MERGE(256) GC_MERGE(512) GC_MERGE(1024) GC_MERGE(2048) GC_MERGE(4096) GC_MERGE(8192) GC_MERGE(16384)
#undef GC_MERGE
          default: return hipErrorInvalidValue;
        }
        parts = mg;
      } else {
        {
          ProfScope prof("pr_tocab_pull", s);
          k_pr_tocab_pull<<<t->n_tiles, kThreads, 0, s>>>(t->row_ptr, t->col, t->tile_row, buf.contrib[0],
                                                          buf.partial);
        }
        u.contrib = buf.contrib[0];  // safe in place: the pull pass has finished reading c
        parts = t->R;
        ProfScope prof("pr_merge", s);
        switch (t->k) {
          case 256: launch_merge<256>(t->R, s, t->range_ptr, t->B, t->id16, buf.partial, u); break;
          case 512: launch_merge<512>(t->R, s, t->range_ptr, t->B, t->id16, buf.partial, u); break;
          case 1024: launch_merge<1024>(t->R, s, t->range_ptr, t->B, t->id16, buf.partial, u); break;
          case 2048: launch_merge<2048>(t->R, s, t->range_ptr, t->B, t->id16, buf.partial, u); break;
          case 4096: launch_merge<4096>(t->R, s, t->range_ptr, t->B, t->id16, buf.partial, u); break;
          case 8192: launch_merge<8192>(t->R, s, t->range_ptr, t->B, t->id16, buf.partial, u); break;
          case 16384: launch_merge<16384>(t->R, s, t->range_ptr, t->B, t->id16, buf.partial, u); break;
          default: return hipErrorInvalidValue;
        }
      }
    } else if (!push) {
      u.contrib = buf.contrib[cur ^ 1];
      parts = g->n_tiles_in;
      ProfScope prof("pr_plain_pull", s);
      k_pr_plain_pull<<<g->n_tiles_in, kThreads, 0, s>>>(g->t_rowptr, g->t_colidx, g->tile_row_in,
                                                         buf.contrib[cur], u);
      cur ^= 1;
    } else if (expanded) {
      u.contrib = nullptr;  // the contributions go to the rows' expanded copies only
      parts = t->B;
      ProfScope prof("pr_tocab_push", s);
      const int64_t P = push_xc_stride(t->P);
      k_pr_push_lds_x<<<t->B, kPushLdsThreads, push_x_lds(t->W, t->B), s>>>(
          t->blk_rowoff, t->row_ptr, t->pcol16, t->pheads, t->log2W, t->xc + (it & 1) * P, push_x(t),
          t->xc + ((it + 1) & 1) * P, u);
    } else if (t && t->W <= kPushLdsMaxWidth) {
      u.contrib = buf.contrib[cur ^ 1];
      parts = t->B;
      ProfScope prof("pr_tocab_push", s);
      k_pr_push_lds<<<t->B, kPushLdsThreads, sizeof(double) * static_cast<size_t>(t->W), s>>>(
          t->blk_rowoff, t->row_ptr, t->id_map, t->col, t->log2W, buf.contrib[cur], u);
      cur ^= 1;
    } else {
      if (t) {
        const int64_t P = t->P;
        if (P > 0) {
          ProfScope prof("pr_tocab_push", s);
          k_pr_push<<<static_cast<uint32_t>((P + kThreads - 1) / kThreads), kThreads, 0, s>>>(
              t->row_ptr, t->id_map, t->col, buf.contrib[0], buf.sums, P);
        }
      } else {
        ProfScope prof("pr_plain_push", s);
        k_pr_push<<<vgrid, kThreads, 0, s>>>(g->rowptr, nullptr, g->colidx, buf.contrib[0], buf.sums, n);
      }
      u.contrib = buf.contrib[0];
      ProfScope prof("pr_apply", s);
      k_pr_apply<<<vgrid, kThreads, 0, s>>>(buf.sums, u);
    }
    {
      ProfScope prof("pr_dangling", s);
      k_reduce_dangling<<<1, 1024, 0, s>>>(buf.dpart, parts, dtotal_out, u.lpart, g->ltotal);
    }
    GC_HIP_TRY(hipGetLastError());
    if (cv) {  // read this iteration's L1 change
      double delta = 0.0;
      GC_HIP_TRY(hipMemcpyAsync(&delta, g->ltotal, sizeof(double), hipMemcpyDeviceToHost, s));
      GC_HIP_TRY(hipStreamSynchronize(s));
      cv->iters = it + 1;
      cv->delta = delta;
      if (delta <= cv->tol) break;
    }
  }
  if (cv && (cv->iters & 1) == 0)  // the last iterate is in rank_tmp
    GC_HIP_TRY(hipMemcpyAsync(rank_out, g->rank_tmp, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
  return hipSuccess;
}

}  // namespace gcx
