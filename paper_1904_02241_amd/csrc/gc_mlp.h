// The level scheduler network's parameter layout and its one-wave
// inference, shared by the scheduler's own kernels and by the traversal
// kernel that ends a level (which runs the decision for the next one).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gc_device.h"
#include "graphcage.h"

namespace gcmlp {

using gcd::kWave;
constexpr int kIn = GC_SCHED_INPUTS;
constexpr int kHid = GC_SCHED_HIDDEN;

// Parameter layout: W1[64][6], b1[64], W2[64][64], b2[64], W3[K][64], b3[K].
struct Layout {
  int32_t W1, b1, W2, b2, W3, b3, total;
  __host__ __device__ explicit Layout(int32_t K) {
    W1 = 0;
    b1 = W1 + kHid * kIn;
    W2 = b1 + kHid;
    b2 = W2 + kHid * kHid;
    W3 = b2 + kHid;
    b3 = W3 + K * kHid;
    total = b3 + K;
  }
};

// Inference for one level (one wave): the K outputs for features `in`
// into out[k] (when given) and the arg-min action, or -1 if an output is
// not finite, into *choice. frange (nullable): per input the lowest, then
// the highest value seen in training; inputs are clamped into it, so a
// level outside the trained range is decided as the nearest trained one.
// W2's rows are read from w2 at a pitch of kPitch words (kHid in the
// parameter vector itself; kHid + 1 for a copy in LDS, where each lane
// reads its own row and a pitch of kHid would put all of them in one bank).
template <int kPitch = kHid>
__device__ __forceinline__ void mlp_decide(const float* __restrict__ p, const float* __restrict__ w2, int32_t K,
                                           const float (&in_raw)[kIn], const float* __restrict__ frange,
                                           int32_t* __restrict__ choice, float* __restrict__ out) {
  const Layout L(K);
  const int lane = threadIdx.x;
  float in[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) in[i] = frange ? fminf(fmaxf(in_raw[i], frange[i]), frange[kIn + i]) : in_raw[i];
  float z = p[L.b1 + lane];
#pragma unroll
  for (int i = 0; i < kIn; ++i) z += p[L.W1 + lane * kIn + i] * in[i];
  const float h1 = fmaxf(z, 0.0f);
  z = p[L.b2 + lane];
  for (int i = 0; i < kHid; ++i)
    z += w2[lane * kPitch + i] * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(h1), i));
  const float h2 = fmaxf(z, 0.0f);
  int best = -1;
  float bv = 0.0f;
  bool bad = false;
  for (int k = 0; k < K; ++k) {
    const float o = p[L.b3 + k] + static_cast<float>(gcd::wave_sum(static_cast<double>(p[L.W3 + k * kHid + lane] * h2)));
    if (out && lane == 0) out[k] = o;
    bad |= !isfinite(o);
    if (best < 0 || o < bv) {
      best = k;
      bv = o;
    }
  }
  if (lane == 0) *choice = bad ? -1 : best;
}

}  // namespace gcmlp
