// Measurement kernels: the read bandwidth of data held in the L2 caches, the bandwidth term
// of the render kernel's cache roofline (the bytes its pixels request over this rate).
#include "bh_dev.h"

namespace bh {

// Workgroup b streams `per_wg` float4 (coalesced: thread t reads elements t, t + 256, ...)
// starting at element (b * 4099) mod n of a buffer of n float4, n a power of two small
// enough to stay in every XCD's L2, wrapping around; the sum keeps the loads alive.
__global__ void __launch_bounds__(256)
    k_l2_read(const float4* __restrict__ buf, uint32_t mask, int per_wg, float* __restrict__ sink) {
  const uint32_t start = ((uint32_t)blockIdx.x * 4099u) & mask;
  float acc = 0.0f;
#pragma unroll 4
  for (int k = threadIdx.x; k < per_wg; k += 256) {
    const float4 v = buf[(start + (uint32_t)k) & mask];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc == -1.0f) sink[blockIdx.x] = acc;  // never true for the zero-filled buffer
}

hipError_t launch_l2_read(const float4* buf, int64_t n4, int per_wg, int grid, float* sink,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_l2_read, dim3(grid), dim3(256), 0, s, buf, (uint32_t)(n4 - 1), per_wg,
                     sink);
  return hipGetLastError();
}

}  // namespace bh
