// Level scheduler network on the GPU: an MLP 6 -> 64 -> 64 -> K (ReLU after
// the hidden layers, FP32) whose output k scores action k for a traversal
// level (a predicted log run time, absolute or relative to the level's
// fastest action); the scheduler runs the arg-min. Forward,
// backward, a deterministic gradient reduction and Adam (Kingma & Ba 2015)
// are all hand-written kernels.
//
// Parameter layout: W1[64][6], b1[64], W2[64][64], b2[64], W3[K][64], b3[K].

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gc_device.h"
#include "gc_internal.h"
#include "gc_mlp.h"

namespace {

using gcd::kWave;
using gcmlp::kHid;
using gcmlp::kIn;
using gcmlp::Layout;
using gcmlp::mlp_decide;

// One wave per sample, lane j = hidden unit j. Stores the outputs and, when
// asked, the hidden activations for the backward pass.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ p, int32_t K,
                                                     const float* __restrict__ x, int32_t batch,
                                                     float* __restrict__ y, float* __restrict__ h1_out,
                                                     float* __restrict__ h2_out) {
  const Layout L(K);
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t b = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (b >= batch) return;  // whole waves leave together
  float in[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) in[i] = x[b * kIn + i];
  float z = p[L.b1 + lane];
#pragma unroll
  for (int i = 0; i < kIn; ++i) z += p[L.W1 + lane * kIn + i] * in[i];
  const float h1 = fmaxf(z, 0.0f);
  z = p[L.b2 + lane];
  for (int i = 0; i < kHid; ++i) z += p[L.W2 + lane * kHid + i] * __shfl(h1, i, kWave);
  const float h2 = fmaxf(z, 0.0f);
  for (int k = 0; k < K; ++k) {
    float t = p[L.W3 + k * kHid + lane] * h2;
    t = gcd::wave_sum(static_cast<double>(t));  // fixed tree, every lane gets the sum
    if (lane == 0) y[b * K + k] = p[L.b3 + k] + t;
  }
  if (h1_out) h1_out[b * kHid + lane] = h1;
  if (h2_out) h2_out[b * kHid + lane] = h2;
}

// Per-sample error terms: dY = 2 M (Y - T) / sum(M); dZ2 = W3^T dY on
// active units; dZ1 = W2^T dZ2 on active units. One wave per sample.
__global__ __launch_bounds__(256) void k_mlp_backward(const float* __restrict__ p, int32_t K,
                                                      const float* __restrict__ y, const float* __restrict__ t,
                                                      const float* __restrict__ mask, const float* __restrict__ msum,
                                                      const float* __restrict__ h1, const float* __restrict__ h2,
                                                      int32_t batch, float* __restrict__ dy, float* __restrict__ dz2,
                                                      float* __restrict__ dz1) {
  const Layout L(K);
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t b = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (b >= batch) return;
  const float scale = *msum > 0.0f ? 2.0f / *msum : 0.0f;
  float g2 = 0.0f;
  for (int k = 0; k < K; ++k) {
    const float d = scale * mask[b * K + k] * (y[b * K + k] - t[b * K + k]);
    if (lane == 0) dy[b * K + k] = d;
    g2 += p[L.W3 + k * kHid + lane] * d;
  }
  const float a2 = h2[b * kHid + lane] > 0.0f ? g2 : 0.0f;
  dz2[b * kHid + lane] = a2;
  float g1 = 0.0f;
  for (int j = 0; j < kHid; ++j) g1 += p[L.W2 + j * kHid + lane] * __shfl(a2, j, kWave);
  dz1[b * kHid + lane] = h1[b * kHid + lane] > 0.0f ? g1 : 0.0f;
}

// Gradient of every parameter as a sum over the batch in sample order (one
// thread per parameter: deterministic, no atomics).
__global__ void k_mlp_grad(int32_t K, const float* __restrict__ x, const float* __restrict__ h1,
                           const float* __restrict__ h2, const float* __restrict__ dy, const float* __restrict__ dz2,
                           const float* __restrict__ dz1, int32_t batch, float* __restrict__ grad) {
  const Layout L(K);
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.total) return;
  double s = 0.0;
  if (q < L.b1) {
    const int j = (q - L.W1) / kIn, i = (q - L.W1) % kIn;
    for (int32_t b = 0; b < batch; ++b) s += static_cast<double>(dz1[b * kHid + j]) * x[b * kIn + i];
  } else if (q < L.W2) {
    const int j = q - L.b1;
    for (int32_t b = 0; b < batch; ++b) s += dz1[b * kHid + j];
  } else if (q < L.b2) {
    const int j = (q - L.W2) / kHid, i = (q - L.W2) % kHid;
    for (int32_t b = 0; b < batch; ++b) s += static_cast<double>(dz2[b * kHid + j]) * h1[b * kHid + i];
  } else if (q < L.W3) {
    const int j = q - L.b2;
    for (int32_t b = 0; b < batch; ++b) s += dz2[b * kHid + j];
  } else if (q < L.b3) {
    const int k = (q - L.W3) / kHid, i = (q - L.W3) % kHid;
    for (int32_t b = 0; b < batch; ++b) s += static_cast<double>(dy[b * K + k]) * h2[b * kHid + i];
  } else {
    const int k = q - L.b3;
    for (int32_t b = 0; b < batch; ++b) s += dy[b * K + k];
  }
  grad[q] = static_cast<float>(s);
}

// sum(M) and the masked mean squared error (one work-group, fixed order).
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ y, const float* __restrict__ t,
                                                  const float* __restrict__ mask, int32_t count,
                                                  float* __restrict__ msum, float* __restrict__ loss) {
  __shared__ double part[2][256 / kWave];
  double sm = 0.0, se = 0.0;
  for (int32_t i = threadIdx.x; i < count; i += 256) {
    const double d = static_cast<double>(y[i]) - t[i];
    sm += mask[i];
    se += mask[i] * d * d;
  }
  sm = gcd::wave_sum(sm);
  se = gcd::wave_sum(se);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    part[0][threadIdx.x / kWave] = sm;
    part[1][threadIdx.x / kWave] = se;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, e = 0.0;
    for (int w = 0; w < 256 / kWave; ++w) {
      a += part[0][w];
      e += part[1][w];
    }
    if (msum) *msum = static_cast<float>(a);
    if (loss) *loss = a > 0.0 ? static_cast<float>(e / a) : 0.0f;
  }
}

// Adam step t (1-based), bias-corrected, beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int32_t n, int32_t t, float lr) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mq = b1 * m[q] + (1.0f - b1) * g[q];
  const float vq = b2 * v[q] + (1.0f - b2) * g[q] * g[q];
  m[q] = mq;
  v[q] = vq;
  const float mh = mq / (1.0f - powf(b1, static_cast<float>(t)));
  const float vh = vq / (1.0f - powf(b2, static_cast<float>(t)));
  p[q] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ __launch_bounds__(kWave) void k_mlp_decide(const float* __restrict__ p, int32_t K, float f0, float f1,
                                                      float f2, float f3, float f4, float f5,
                                                      const float* __restrict__ frange, int32_t* __restrict__ choice,
                                                      float* __restrict__ out) {
  const float in[kIn] = {f0, f1, f2, f3, f4, f5};
  mlp_decide(p, p + Layout(K).W2, K, in, frange, choice, out);
}

// Lowest and highest value of each input over the training rows (one wave
// per input, fixed order).
__global__ __launch_bounds__(kWave) void k_feature_range(const float* __restrict__ x, int32_t batch,
                                                         float* __restrict__ frange) {
  const int i = blockIdx.x;
  float lo = INFINITY, hi = -INFINITY;
  for (int32_t b = threadIdx.x; b < batch; b += kWave) {
    lo = fminf(lo, x[b * kIn + i]);
    hi = fmaxf(hi, x[b * kIn + i]);
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o, kWave));
    hi = fmaxf(hi, __shfl_xor(hi, o, kWave));
  }
  if (threadIdx.x == 0) {
    frange[i] = lo;
    frange[kIn + i] = hi;
  }
}

}  // namespace

struct gc_sched_s {
  int32_t K = 0;
  int32_t n = 0;
  int32_t step = 0;
  float* params = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  int32_t* choice = nullptr;
  int32_t* choice_host = nullptr;
  float* frange = nullptr;  // [2 * inputs] training range of each input (set by sched_train)
  bool ranged = false;
};

namespace gcx {

int32_t sched_actions(gc_sched m) { return m->K; }

const float* sched_params(gc_sched m) { return m->params; }

const float* sched_range(gc_sched m) { return m->ranged ? m->frange : nullptr; }

// Decision for one level from host-computed features; -1 when the network
// gives no finite answer (the caller falls back to the heuristic).
hipError_t sched_decide(gc_sched m, const float* f, hipStream_t s, int32_t* action, float* out) {
  // m->choice holds the action, then the K outputs
  k_mlp_decide<<<1, kWave, 0, s>>>(m->params, m->K, f[0], f[1], f[2], f[3], f[4], f[5], sched_range(m),
                                   m->choice, reinterpret_cast<float*>(m->choice + 1));
  GC_HIP_TRY(hipGetLastError());
  GC_HIP_TRY(hipMemcpyAsync(m->choice_host, m->choice, sizeof(int32_t) * (1 + m->K), hipMemcpyDeviceToHost, s));
  GC_HIP_TRY(hipStreamSynchronize(s));
  *action = m->choice_host[0];
  if (out) std::memcpy(out, m->choice_host + 1, sizeof(float) * m->K);
  return hipSuccess;
}


}  // namespace gcx

namespace {

int fail_sched(int code, const char* what) {
  gcx::set_error("%s", what);
  return code;
}

bool dev_ptr(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Runs forward + loss + backward + gradient for one batch into m->grad.
hipError_t loss_grad(gc_sched m, const float* x, const float* t, const float* mask, int32_t batch, float* loss,
                     hipStream_t s) {
  const int32_t K = m->K;
  gcx::Buf y(sizeof(float) * batch * K, s), h1(sizeof(float) * batch * kHid, s), h2(sizeof(float) * batch * kHid, s),
      dy(sizeof(float) * batch * K, s), dz2(sizeof(float) * batch * kHid, s), dz1(sizeof(float) * batch * kHid, s),
      msum(sizeof(float) * 2, s);
  if (!y.p || !h1.p || !h2.p || !dy.p || !dz2.p || !dz1.p || !msum.p) return hipErrorOutOfMemory;
  const int grid = (batch + 3) / 4;
  k_mlp_forward<<<grid, 256, 0, s>>>(m->params, K, x, batch, y.as<float>(), h1.as<float>(), h2.as<float>());
  k_mlp_loss<<<1, 256, 0, s>>>(y.as<float>(), t, mask, batch * K, msum.as<float>(), loss);
  k_mlp_backward<<<grid, 256, 0, s>>>(m->params, K, y.as<float>(), t, mask, msum.as<float>(), h1.as<float>(),
                                      h2.as<float>(), batch, dy.as<float>(), dz2.as<float>(), dz1.as<float>());
  k_mlp_grad<<<(m->n + 255) / 256, 256, 0, s>>>(K, x, h1.as<float>(), h2.as<float>(), dy.as<float>(),
                                                dz2.as<float>(), dz1.as<float>(), batch, m->grad);
  GC_HIP_TRY(hipGetLastError());
  return hipStreamSynchronize(s);  // scratch is released on return
}

}  // namespace

extern "C" {

int sched_param_count(int32_t n_actions, int64_t* count) {
  if (n_actions < 1 || n_actions > kHid || !count) return fail_sched(GC_EINVAL, "sched_param_count: n_actions in [1, 64]");
  *count = Layout(n_actions).total;
  return GC_OK;
}

int sched_create(int32_t n_actions, const float* params, gc_sched* out) {
  if (!out) return fail_sched(GC_EINVAL, "sched_create: out is NULL");
  *out = nullptr;
  if (n_actions < 1 || n_actions > kHid) return fail_sched(GC_EINVAL, "sched_create: n_actions must be in [1, 64]");
  if (!params) return fail_sched(GC_EINVAL, "sched_create: NULL params");
  gc_sched m = new (std::nothrow) gc_sched_s;
  if (!m) return fail_sched(GC_ENOMEM, "sched_create: host allocation failed");
  m->K = n_actions;
  m->n = Layout(n_actions).total;
  const size_t bytes = sizeof(float) * m->n;
  m->params = static_cast<float*>(gcx::dev_alloc(bytes, nullptr));
  m->m = static_cast<float*>(gcx::dev_alloc(bytes, nullptr));
  m->v = static_cast<float*>(gcx::dev_alloc(bytes, nullptr));
  m->grad = static_cast<float*>(gcx::dev_alloc(bytes, nullptr));
  m->choice = static_cast<int32_t*>(gcx::dev_alloc(sizeof(int32_t) * (1 + kHid), nullptr));
  m->frange = static_cast<float*>(gcx::dev_alloc(sizeof(float) * 2 * kIn, nullptr));
  if (hipHostMalloc(reinterpret_cast<void**>(&m->choice_host), sizeof(int32_t) * (1 + kHid), hipHostMallocDefault) !=
      hipSuccess)
    m->choice_host = nullptr;
  if (!m->params || !m->m || !m->v || !m->grad || !m->choice || !m->frange || !m->choice_host) {
    sched_free(m);
    return fail_sched(GC_ENOMEM, "sched_create: allocation failed");
  }
  hipError_t e = hipMemcpy(m->params, params, bytes, hipMemcpyDefault);
  if (e == hipSuccess) e = hipMemset(m->m, 0, bytes);
  if (e == hipSuccess) e = hipMemset(m->v, 0, bytes);
  if (e != hipSuccess) {
    sched_free(m);
    return fail_sched(GC_EHIP, "sched_create: copy failed");
  }
  *out = m;
  return GC_OK;
}

int sched_get_params(gc_sched m, float* params, hipStream_t stream) {
  if (!m || !params) return fail_sched(GC_EINVAL, "sched_get_params: NULL argument");
  const hipError_t e = hipMemcpyAsync(params, m->params, sizeof(float) * m->n, hipMemcpyDefault, stream);
  return e == hipSuccess ? GC_OK : fail_sched(GC_EHIP, "sched_get_params: copy failed");
}

int sched_forward(gc_sched m, const float* x, int32_t batch, float* y, hipStream_t stream) {
  if (!m || !x || !y || batch < 0) return fail_sched(GC_EINVAL, "sched_forward: bad argument");
  if (!dev_ptr(x) || !dev_ptr(y)) return fail_sched(GC_EINVAL, "sched_forward: x and y must be device memory");
  if (batch == 0) return GC_OK;
  k_mlp_forward<<<(batch + 3) / 4, 256, 0, stream>>>(m->params, m->K, x, batch, y, nullptr, nullptr);
  return hipGetLastError() == hipSuccess ? GC_OK : fail_sched(GC_EHIP, "sched_forward: launch failed");
}

int sched_loss_grad(gc_sched m, const float* x, const float* t, const float* mask, int32_t batch, float* loss,
                    float* grad, hipStream_t stream) {
  if (!m || !x || !t || !mask || !loss || !grad || batch <= 0) return fail_sched(GC_EINVAL, "sched_loss_grad: bad argument");
  if (!dev_ptr(x) || !dev_ptr(t) || !dev_ptr(mask) || !dev_ptr(loss) || !dev_ptr(grad))
    return fail_sched(GC_EINVAL, "sched_loss_grad: buffers must be device memory");
  hipError_t e = loss_grad(m, x, t, mask, batch, loss, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(grad, m->grad, sizeof(float) * m->n, hipMemcpyDeviceToDevice, stream);
  return e == hipSuccess ? GC_OK : fail_sched(GC_EHIP, "sched_loss_grad: failed");
}

int sched_train(gc_sched m, const float* x, const float* t, const float* mask, int32_t batch, int32_t steps, float lr,
                float* loss_hist, hipStream_t stream) {
  if (!m || !x || !t || !mask || batch <= 0 || steps < 0 || !(lr > 0.0f))
    return fail_sched(GC_EINVAL, "sched_train: bad argument");
  if (!dev_ptr(x) || !dev_ptr(t) || !dev_ptr(mask) || (loss_hist && !dev_ptr(loss_hist)))
    return fail_sched(GC_EINVAL, "sched_train: buffers must be device memory");
  gcx::Buf scratch(sizeof(float), stream);
  if (!scratch.p) return fail_sched(GC_ENOMEM, "sched_train: allocation failed");
  k_feature_range<<<kIn, kWave, 0, stream>>>(x, batch, m->frange);
  if (hipGetLastError() != hipSuccess) return fail_sched(GC_EHIP, "sched_train: range launch failed");
  m->ranged = true;
  for (int32_t i = 0; i < steps; ++i) {
    hipError_t e = loss_grad(m, x, t, mask, batch, loss_hist ? loss_hist + i : scratch.as<float>(), stream);
    if (e != hipSuccess) return fail_sched(GC_EHIP, "sched_train: step failed");
    m->step += 1;
    k_adam<<<(m->n + 255) / 256, 256, 0, stream>>>(m->params, m->grad, m->m, m->v, m->n, m->step, lr);
    if (hipGetLastError() != hipSuccess) return fail_sched(GC_EHIP, "sched_train: adam launch failed");
  }
  return hipStreamSynchronize(stream) == hipSuccess ? GC_OK : fail_sched(GC_EHIP, "sched_train: sync failed");
}

int sched_free(gc_sched m) {
  if (!m) return fail_sched(GC_EINVAL, "sched_free: NULL model");
  (void)hipDeviceSynchronize();
  for (void* q : {static_cast<void*>(m->params), static_cast<void*>(m->m), static_cast<void*>(m->v),
                  static_cast<void*>(m->grad), static_cast<void*>(m->choice), static_cast<void*>(m->frange)})
    if (q) gcx::dev_free(q, nullptr);
  if (m->choice_host) (void)hipHostFree(m->choice_host);
  delete m;
  return GC_OK;
}

}  // extern "C"
