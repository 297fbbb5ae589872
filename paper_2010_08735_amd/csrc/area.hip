// Area-source cube map (Section 3.3.2 "Emitted light": nebulae and galaxies stored in a
// cube map and read with anisotropic filtering).  Level 0 holds (I, I T) per texel from the
// caller's (I, T); level L + 1 is the box mean of its four children in both channels, so
// every level keeps the map's mean radiance and radiance-weighted temperature.  Layout:
// level L (size nL = n0 >> L) at texel 8 (n0^2 - nL^2), faces then rows then columns.
// Band maps (below) use the same pyramid on float4 texels.
#include "bh_dev.h"

namespace bh {

// level 0 from (I, T) pairs; flags any negative or non-finite input in *bad
__global__ void k_area_level0(const float2* __restrict__ it, int64_t n, float2* __restrict__ out,
                              int* __restrict__ bad) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float2 v = it[t];
  const bool ok = v.x >= 0.0f && v.y >= 0.0f && v.x <= 3.0e38f && v.y <= 3.0e38f;
  if (!ok) atomicOr(bad, 1);
  out[t] = ok ? make_float2(v.x, v.x * v.y) : make_float2(0.0f, 0.0f);
}

// level L + 1 (size nc / 2) from level L (size nc)
__global__ void k_area_mip(const float2* __restrict__ src, int nc, float2* __restrict__ dst) {
  const int n = nc >> 1;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 6ll * n * n) return;
  const int x = (int)(t % n), y = (int)((t / n) % n), f = (int)(t / ((int64_t)n * n));
  const float2* r0 = src + ((int64_t)f * nc + 2 * y) * nc + 2 * x;
  const float2* r1 = r0 + nc;
  const float2 a = r0[0], b = r0[1], c = r1[0], d = r1[1];
  dst[t] = make_float2(0.25f * ((a.x + b.x) + (c.x + d.x)), 0.25f * ((a.y + b.y) + (c.y + d.y)));
}

// Band maps (light of any colour, shifted through the colour-shift table): each texel holds
// the band radiances (R, G, B) as a float4 with w = 0, and the mips are box means of the
// three bands.
__global__ void k_area_level0_bands(const float4* __restrict__ rgbx, int64_t n,
                                    float4* __restrict__ out, int* __restrict__ bad) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float4 v = rgbx[t];
  const bool ok = v.x >= 0.0f && v.y >= 0.0f && v.z >= 0.0f && v.x <= 3.0e38f &&
                  v.y <= 3.0e38f && v.z <= 3.0e38f;
  if (!ok) atomicOr(bad, 1);
  out[t] = ok ? make_float4(v.x, v.y, v.z, 0.0f) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

__global__ void k_area_mip_bands(const float4* __restrict__ src, int nc, float4* __restrict__ dst) {
  const int n = nc >> 1;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 6ll * n * n) return;
  const int x = (int)(t % n), y = (int)((t / n) % n), f = (int)(t / ((int64_t)n * n));
  const float4* r0 = src + ((int64_t)f * nc + 2 * y) * nc + 2 * x;
  const float4* r1 = r0 + nc;
  const float4 a = r0[0], b = r0[1], c = r1[0], d = r1[1];
  dst[t] = make_float4(0.25f * ((a.x + b.x) + (c.x + d.x)), 0.25f * ((a.y + b.y) + (c.y + d.y)),
                       0.25f * ((a.z + b.z) + (c.z + d.z)), 0.0f);
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_area_build_bands(const float* rgbx, int n0, float4* tex, int* bad,
                                   hipStream_t s) {
  const int64_t n = 6ll * n0 * n0;
  hipLaunchKernelGGL(k_area_level0_bands, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                     (const float4*)rgbx, n, tex, bad);
  int64_t off = 0;
  for (int nc = n0; nc > 1; nc >>= 1) {
    const int64_t cnt = 6ll * nc * nc;
    const int64_t m = cnt / 4;
    hipLaunchKernelGGL(k_area_mip_bands, dim3(blocks_for(m, 256)), dim3(256), 0, s, tex + off,
                       nc, tex + off + cnt);
    off += cnt;
  }
  return hipGetLastError();
}

hipError_t launch_area_build(const float* it, int n0, float2* tex, int* bad, hipStream_t s) {
  const int64_t n = 6ll * n0 * n0;
  hipLaunchKernelGGL(k_area_level0, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                     (const float2*)it, n, tex, bad);
  int64_t off = 0;
  for (int nc = n0; nc > 1; nc >>= 1) {
    const int64_t cnt = 6ll * nc * nc;
    const int64_t m = cnt / 4;
    hipLaunchKernelGGL(k_area_mip, dim3(blocks_for(m, 256)), dim3(256), 0, s, tex + off, nc,
                       tex + off + cnt);
    off += cnt;
  }
  return hipGetLastError();
}

}  // namespace bh
