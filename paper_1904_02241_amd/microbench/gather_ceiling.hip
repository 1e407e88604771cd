// Memory-system ceilings of the GPU that bound the graph kernels: random
// 4-byte gathers from buffers of growing size (L2-, MALL- and HBM-resident),
// random 4-byte reads from LDS, and a streaming read. Indices are a hash
// masked to the buffer size, so every access is in bounds.
// Build: paper_1904_02241_amd/build.py; run: paper_1904_02241_amd/microbench/gather_ceiling
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <vector>
__device__ __forceinline__ uint32_t hsh(uint32_t x) { x ^= x >> 16; x *= 0x7feb352d; x ^= x >> 15; x *= 0x846ca68b; x ^= x >> 16; return x; }
__global__ void k_gather(const float* __restrict__ a, uint32_t mask, int per_thread, float* out, uint32_t seed) {
  uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0;
  #pragma unroll 16
  for (int i = 0; i < per_thread; ++i) s += a[hsh(t * 64u + i + seed) & mask];
  if (s == 12345.f) out[t] = s;
}
__global__ void k_lds(int per_thread, float* out, uint32_t lds_mask) {
  __shared__ float L[16384];
  for (int i = threadIdx.x; i < 16384; i += blockDim.x) L[i] = i;
  __syncthreads();
  uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0;
  #pragma unroll 16
  for (int i = 0; i < per_thread; ++i) s += L[hsh(t * 64u + i) & lds_mask];
  if (s == 12345.f) out[t] = s;
}
typedef int v4i __attribute__((ext_vector_type(4)));
__global__ void k_stream(const v4i* __restrict__ a, size_t n4, float* out) {
  size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  int acc = 0;
  for (size_t i = t; i < n4; i += (size_t)gridDim.x * blockDim.x) { v4i v = __builtin_nontemporal_load(a + i); acc += v.x ^ v.y ^ v.z ^ v.w; }
  if (acc == 12345) out[t] = acc;
}
int main() {
  size_t maxb = size_t(1) << 30;
  float* a; hipMalloc(&a, maxb); hipMemset(a, 0, maxb);
  float* out; hipMalloc(&out, 64 << 20);
  hipEvent_t e0, e1; hipEventCreate(&e0); hipEventCreate(&e1);
  int threads = 256, blocks = 256 * 64, per = 256;
  double total = double(threads) * blocks * per;
  for (size_t bytes : {size_t(1) << 18, size_t(1) << 20, size_t(1) << 22, size_t(1) << 24, size_t(1) << 26, size_t(1) << 27, size_t(1) << 28, size_t(1) << 30}) {
    uint32_t mask = uint32_t(bytes / 4 - 1);
    k_gather<<<blocks, threads>>>(a, mask, per, out, 1);
    hipEventRecord(e0);
    k_gather<<<blocks, threads>>>(a, mask, per, out, 7);
    hipEventRecord(e1); hipEventSynchronize(e1);
    float ms; hipEventElapsedTime(&ms, e0, e1);
    printf("gather buffer %8zu KiB: %.1f G gathers/s  (%.3f ms)\n", bytes >> 10, total / (ms * 1e-3) / 1e9, ms);
  }
  for (uint32_t m : {1023u, 8191u, 16383u}) {
    k_lds<<<blocks, threads>>>(per, out, m);
    hipEventRecord(e0);
    k_lds<<<blocks, threads>>>(per, out, m);
    hipEventRecord(e1); hipEventSynchronize(e1);
    float ms; hipEventElapsedTime(&ms, e0, e1);
    printf("lds gather range %u: %.1f G gathers/s\n", m + 1, total / (ms * 1e-3) / 1e9);
  }
  k_stream<<<256 * 16, 256>>>((const v4i*)a, maxb / 16, out);
  hipEventRecord(e0);
  k_stream<<<256 * 16, 256>>>((const v4i*)a, maxb / 16, out);
  hipEventRecord(e1); hipEventSynchronize(e1);
  float ms; hipEventElapsedTime(&ms, e0, e1);
  printf("stream read 1 GiB: %.1f GB/s\n", maxb / (ms * 1e-3) / 1e9);
  hipError_t err = hipGetLastError(); printf("err=%s\n", hipGetErrorString(err));
  return 0;
}
