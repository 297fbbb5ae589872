// Star cube map (Section 3.3.2 "Emitted light").  Each texel of every mip level holds the
// intensity sum of the stars inside it, their intensity-weighted mean temperature and
// their intensity-weighted mean position inside the texel; mips combine the four children
// with the same rule (sum of intensities, intensity-weighted averages).  Stars that land in
// the same level-0 texel are merged by the same rule, in star-index order, so the build is
// deterministic whatever order the atomics run in.
// Face of a direction d: k = argmax |d_k| (ties to the lowest index), face 2k + (d_k < 0),
// U = d_{(k+1)%3} / |d_k|, V = d_{(k+2)%3} / |d_k| in [-1, 1].
// Stored texels: FP16 (I / scale_L, T / 1024, p_u, p_v) with a per-level power-of-two
// scale chosen from the level's largest intensity, or FP32 (I, T, p_u, p_v).
#include <algorithm>

#include "bh_dev.h"

namespace bh {

struct __align__(8) Half4 {
  _Float16 x, y, z, w;
};

__global__ void k_star_link(const float* __restrict__ dirs, const float* __restrict__ inten,
                            int64_t n, int n0, int* __restrict__ head, int* __restrict__ next,
                            float2* __restrict__ pos) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  float d0 = dirs[3 * s], d1 = dirs[3 * s + 1], d2 = dirs[3 * s + 2];
  float I = inten[s];
  float a0 = fabsf(d0), a1 = fabsf(d1), a2 = fabsf(d2);
  int k = 0;
  float m = a0;
  if (a1 > m) { k = 1; m = a1; }
  if (a2 > m) { k = 2; m = a2; }
  if (!(I > 0.0f) || !(m > 0.0f)) {
    next[s] = -2;
    return;
  }
  float dk = k == 0 ? d0 : (k == 1 ? d1 : d2);
  float da = k == 0 ? d1 : (k == 1 ? d2 : d0);
  float db = k == 0 ? d2 : (k == 1 ? d0 : d1);
  int face = 2 * k + (dk < 0.0f);
  float U = da / m, V = db / m;
  float gx = 0.5f * (U + 1.0f) * (float)n0, gy = 0.5f * (V + 1.0f) * (float)n0;
  int ix = min(max((int)floorf(gx), 0), n0 - 1);
  int iy = min(max((int)floorf(gy), 0), n0 - 1);
  pos[s] = make_float2(gx - (float)ix, gy - (float)iy);
  int key = (face * n0 + iy) * n0 + ix;
  next[s] = atomicExch(&head[key], (int)s);
}

// level 0: merge the stars of each texel in increasing star index
__global__ void k_star_reduce0(const int* __restrict__ head, const int* __restrict__ next,
                               const float* __restrict__ inten, const float* __restrict__ temp,
                               const float2* __restrict__ pos, int64_t ntex,
                               float4* __restrict__ master) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ntex) return;
  int h = head[t];
  double sI = 0, sIT = 0, sIu = 0, sIv = 0;
  int last = -1;
  while (h >= 0) {
    int best = 0x7fffffff;
    for (int c = h; c >= 0; c = next[c])
      if (c > last && c < best) best = c;
    if (best == 0x7fffffff) break;
    double I = inten[best];
    float2 p = pos[best];
    sI += I;
    sIT += I * (double)temp[best];
    sIu += I * (double)p.x;
    sIv += I * (double)p.y;
    last = best;
  }
  master[t] = sI > 0.0 ? make_float4((float)sI, (float)(sIT / sI), (float)(sIu / sI),
                                     (float)(sIv / sI))
                       : make_float4(0.f, 0.f, 0.f, 0.f);
}

// parent texel from children (0,0), (1,0), (0,1), (1,1)
__global__ void k_star_mip(const float4* __restrict__ prev, float4* __restrict__ cur, int nc) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t total = 6LL * nc * nc;
  if (t >= total) return;
  int x = (int)(t % nc), y = (int)((t / nc) % nc), f = (int)(t / ((int64_t)nc * nc));
  int np = 2 * nc;
  double sI = 0, sIT = 0, sIu = 0, sIv = 0;
  for (int c = 0; c < 4; ++c) {
    int cx = 2 * x + (c & 1), cy = 2 * y + (c >> 1);
    float4 ch = prev[((int64_t)f * np + cy) * np + cx];
    if (!(ch.x > 0.0f)) continue;
    double I = ch.x;
    sI += I;
    sIT += I * ch.y;
    sIu += I * 0.5 * ((c & 1) + (double)ch.z);
    sIv += I * 0.5 * ((c >> 1) + (double)ch.w);
  }
  cur[t] = sI > 0.0 ? make_float4((float)sI, (float)(sIT / sI), (float)(sIu / sI),
                                  (float)(sIv / sI))
                    : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Largest stored intensity of one level: grid-stride partial maxima, a wave then a
// workgroup reduction, one atomic per workgroup (I >= 0, so float order == bit order).
// Launched with 256 threads per workgroup.
__global__ void __launch_bounds__(256)
    k_star_maxI(const float4* __restrict__ lvl, int64_t count, unsigned* __restrict__ maxbits) {
  __shared__ float wmax[4];
  float v = 0.0f;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x)
    v = fmaxf(v, lvl[t].x);
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    if (m > 0.0f) atomicMax(maxbits, __float_as_uint(m));
  }
}

__global__ void k_star_pack(const float4* __restrict__ lvl, int64_t count,
                            const float* __restrict__ scale, int level, int fp16,
                            void* __restrict__ out) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= count) return;
  float4 m = lvl[t];
  if (fp16) {
    float inv = 1.0f / scale[level];
    Half4 h;
    h.x = (_Float16)(m.x * inv);
    h.y = (_Float16)(m.y * (1.0f / 1024.0f));
    h.z = (_Float16)m.z;
    h.w = (_Float16)m.w;
    ((Half4*)out)[t] = h;
  } else {
    ((float4*)out)[t] = m;
  }
}

__global__ void k_star_unpack(const void* __restrict__ in, int64_t count, float scale, int fp16,
                              float4* __restrict__ out) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= count) return;
  if (fp16) {
    Half4 h = ((const Half4*)in)[t];
    out[t] = make_float4((float)h.x * scale, (float)h.y * 1024.0f, (float)h.z, (float)h.w);
  } else {
    out[t] = ((const float4*)in)[t];
  }
}

// per-level scale: power of two so that the largest intensity maps to about 2^14
__global__ void k_star_scales(const unsigned* __restrict__ maxbits, int levels, int fp16,
                              float* __restrict__ scale) {
  int l = threadIdx.x;
  if (l >= levels) return;
  if (!fp16) {
    scale[l] = 1.0f;
    return;
  }
  float mx = __uint_as_float(maxbits[l]);
  scale[l] = mx > 0.0f ? exp2f(ceilf(log2f(mx)) - 14.0f) : 1.0f;
}

// Occupancy bits of one level: one bit per texel (stored intensity > 0), each texel row
// padded to whole 32-bit words plus one guard word, so a footprint row of at most 9
// texels is read from two consecutive words of its row that never leave the row's storage.
// Every row is stored paired with the next row of its face (the last row with an empty
// one), the two rows' words interleaved: word wi of the pair starting at row R = face nl + y
// is at 2 (R wpr + wi) for row y and 2 (R wpr + wi) + 1 for row y + 1, so one 16-byte load
// returns two consecutive words of two consecutive rows, from any starting row.
__device__ __forceinline__ bool occ_word_row(int64_t w, int nl, int wpr, int* wi, int64_t* row) {
  const int h = (int)(w & 1);
  const int64_t q = w >> 1;
  *wi = (int)(q % wpr);
  const int64_t R = q / wpr;                    // face * nl + y: the pair's first row
  const int y = (int)(R % nl) + h;
  *row = R + h;
  return y < nl;
}

__global__ void k_star_occupancy(const void* __restrict__ tex, int nl, int fp16,
                                 uint32_t* __restrict__ occ) {
  const int wpr = ((nl + 31) >> 5) + 1;
  int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t total = 6LL * 2 * nl * wpr;
  if (w >= total) return;
  int wi;
  int64_t row;
  uint32_t bits = 0;
  if (occ_word_row(w, nl, wpr, &wi, &row)) {
    for (int b = 0; b < 32; ++b) {
      int x = wi * 32 + b;
      if (x >= nl) break;
      int64_t t = row * nl + x;
      float I = fp16 ? (float)((const Half4*)tex)[t].x : ((const float4*)tex)[t].x;
      if (I > 0.0f) bits |= 1u << b;
    }
  }
  occ[w] = bits;
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_star_occupancy(const void* tex, int n0, int levels, const uint32_t* level_off,
                                 const uint32_t* occ_off, int fp16, uint32_t* occ,
                                 hipStream_t s) {
  size_t tsz = fp16 ? 8 : 16;
  for (int l = 0; l < levels; ++l) {
    int nl = n0 >> l;
    int64_t words = 6LL * 2 * nl * (((nl + 31) >> 5) + 1);
    hipLaunchKernelGGL(k_star_occupancy, dim3(blocks_for(words, 256)), dim3(256), 0, s,
                       (const void*)((const char*)tex + tsz * level_off[l]), nl, fp16,
                       occ + occ_off[l]);
  }
  return hipGetLastError();
}

// Build every level.  Scratch: head (6 n0^2 ints, pre-filled with -1), next (n ints),
// pos (n float2), master (all levels, float4), maxbits (levels uints, zeroed).
hipError_t launch_star_build(const float* dirs, const float* inten, const float* temp, int64_t n,
                             int n0, int levels, const uint32_t* level_off_host, int* head,
                             int* next, float2* pos, float4* master, unsigned* maxbits,
                             float* scale, int fp16, void* out, hipStream_t s) {
  const int B = 256;
  int64_t ntex0 = 6LL * n0 * n0;
  if (n > 0)
    hipLaunchKernelGGL(k_star_link, dim3(blocks_for(n, B)), dim3(B), 0, s, dirs, inten, n, n0,
                       head, next, pos);
  hipLaunchKernelGGL(k_star_reduce0, dim3(blocks_for(ntex0, B)), dim3(B), 0, s, head, next,
                     inten, temp, pos, ntex0, master);
  for (int l = 1; l < levels; ++l) {
    int nc = n0 >> l;
    hipLaunchKernelGGL(k_star_mip, dim3(blocks_for(6LL * nc * nc, B)), dim3(B), 0, s,
                       master + level_off_host[l - 1], master + level_off_host[l], nc);
  }
  for (int l = 0; l < levels; ++l) {
    int64_t cnt = 6LL * (n0 >> l) * (n0 >> l);
    unsigned grid = std::min(blocks_for(cnt, B), 2048u);
    hipLaunchKernelGGL(k_star_maxI, dim3(grid), dim3(B), 0, s, master + level_off_host[l], cnt,
                       maxbits + l);
  }
  hipLaunchKernelGGL(k_star_scales, dim3(1), dim3(64), 0, s, maxbits, levels, fp16, scale);
  size_t tsz = fp16 ? 8 : 16;
  for (int l = 0; l < levels; ++l) {
    int64_t cnt = 6LL * (n0 >> l) * (n0 >> l);
    hipLaunchKernelGGL(k_star_pack, dim3(blocks_for(cnt, B)), dim3(B), 0, s,
                       master + level_off_host[l], cnt, scale, l, fp16,
                       (void*)((char*)out + tsz * level_off_host[l]));
  }
  return hipGetLastError();
}

// ---- band-colour star maps (light of any colour, Section 3.4.2) --------------------------
// Each texel holds the band sums (R, G, B) of its stars and their position inside the texel
// weighted by S = R + G + B; mips combine the four children by the same rule.  Master
// texels are two float4 records (R, G, B, p_u) and (p_v, 0, 0, 0).  Stored texels: FP16
// (R / scale_L, G / scale_L, B / scale_L, p_u, p_v, 0, 0, 0) with the per-level power of
// two of the (I, T) format chosen from the level's largest band value, or the same eight
// values in FP32.
struct __align__(16) Half8 {
  _Float16 v[8];
};

__global__ void k_star_link_bands(const float* __restrict__ dirs, const float* __restrict__ rgb,
                                  int64_t n, int n0, int* __restrict__ head,
                                  int* __restrict__ next, float2* __restrict__ pos,
                                  int* __restrict__ bad) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  float d0 = dirs[3 * s], d1 = dirs[3 * s + 1], d2 = dirs[3 * s + 2];
  const float r = rgb[3 * s], g = rgb[3 * s + 1], b = rgb[3 * s + 2];
  // a negative, infinite or NaN band fails the whole build (the host reads `bad`)
  if (!(r >= 0.0f && g >= 0.0f && b >= 0.0f) || isinf(r) || isinf(g) || isinf(b))
    atomicOr(bad, 1);
  // S > 0 exactly when a band is positive
  const bool lit = r > 0.0f || g > 0.0f || b > 0.0f;
  float a0 = fabsf(d0), a1 = fabsf(d1), a2 = fabsf(d2);
  int k = 0;
  float m = a0;
  if (a1 > m) { k = 1; m = a1; }
  if (a2 > m) { k = 2; m = a2; }
  if (!lit || !(m > 0.0f)) {
    next[s] = -2;
    return;
  }
  float dk = k == 0 ? d0 : (k == 1 ? d1 : d2);
  float da = k == 0 ? d1 : (k == 1 ? d2 : d0);
  float db = k == 0 ? d2 : (k == 1 ? d0 : d1);
  int face = 2 * k + (dk < 0.0f);
  float U = da / m, V = db / m;
  float gx = 0.5f * (U + 1.0f) * (float)n0, gy = 0.5f * (V + 1.0f) * (float)n0;
  int ix = min(max((int)floorf(gx), 0), n0 - 1);
  int iy = min(max((int)floorf(gy), 0), n0 - 1);
  pos[s] = make_float2(gx - (float)ix, gy - (float)iy);
  int key = (face * n0 + iy) * n0 + ix;
  next[s] = atomicExch(&head[key], (int)s);
}

__device__ __forceinline__ void store_band_master(float4* master, int64_t t, double R, double G,
                                                  double B, double su, double sv) {
  const double S = R + G + B;
  if (S > 0.0) {
    master[2 * t] = make_float4((float)R, (float)G, (float)B, (float)(su / S));
    master[2 * t + 1] = make_float4((float)(sv / S), 0.f, 0.f, 0.f);
  } else {
    master[2 * t] = make_float4(0.f, 0.f, 0.f, 0.f);
    master[2 * t + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// level 0: merge the stars of each texel in increasing star index
__global__ void k_star_reduce0_bands(const int* __restrict__ head, const int* __restrict__ next,
                                     const float* __restrict__ rgb,
                                     const float2* __restrict__ pos, int64_t ntex,
                                     float4* __restrict__ master) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ntex) return;
  int h = head[t];
  double R = 0, G = 0, B = 0, su = 0, sv = 0;
  int last = -1;
  while (h >= 0) {
    int best = 0x7fffffff;
    for (int c = h; c >= 0; c = next[c])
      if (c > last && c < best) best = c;
    if (best == 0x7fffffff) break;
    const double r = rgb[3 * best], g = rgb[3 * best + 1], b = rgb[3 * best + 2];
    const double S = r + g + b;
    const float2 p = pos[best];
    R += r;
    G += g;
    B += b;
    su += S * (double)p.x;
    sv += S * (double)p.y;
    last = best;
  }
  store_band_master(master, t, R, G, B, su, sv);
}

// parent texel from children (0,0), (1,0), (0,1), (1,1)
__global__ void k_star_mip_bands(const float4* __restrict__ prev, float4* __restrict__ cur,
                                 int nc) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t total = 6LL * nc * nc;
  if (t >= total) return;
  int x = (int)(t % nc), y = (int)((t / nc) % nc), f = (int)(t / ((int64_t)nc * nc));
  int np = 2 * nc;
  double R = 0, G = 0, B = 0, su = 0, sv = 0;
  for (int c = 0; c < 4; ++c) {
    int cx = 2 * x + (c & 1), cy = 2 * y + (c >> 1);
    const int64_t ct = ((int64_t)f * np + cy) * np + cx;
    const float4 a = prev[2 * ct], b = prev[2 * ct + 1];
    const double S = (double)a.x + (double)a.y + (double)a.z;
    if (!(S > 0.0)) continue;
    R += a.x;
    G += a.y;
    B += a.z;
    su += S * 0.5 * ((c & 1) + (double)a.w);
    sv += S * 0.5 * ((c >> 1) + (double)b.x);
  }
  store_band_master(cur, t, R, G, B, su, sv);
}

// Largest band value of one level (as k_star_maxI)
__global__ void __launch_bounds__(256)
    k_star_maxI_bands(const float4* __restrict__ lvl, int64_t count,
                      unsigned* __restrict__ maxbits) {
  __shared__ float wmax[4];
  float v = 0.0f;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x) {
    const float4 a = lvl[2 * t];
    v = fmaxf(v, fmaxf(a.x, fmaxf(a.y, a.z)));
  }
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    if (m > 0.0f) atomicMax(maxbits, __float_as_uint(m));
  }
}

__global__ void k_star_pack_bands(const float4* __restrict__ lvl, int64_t count,
                                  const float* __restrict__ scale, int level, int fp16,
                                  void* __restrict__ out) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= count) return;
  const float4 a = lvl[2 * t], b = lvl[2 * t + 1];
  if (fp16) {
    const float inv = 1.0f / scale[level];
    Half8 h;
    h.v[0] = (_Float16)(a.x * inv);
    h.v[1] = (_Float16)(a.y * inv);
    h.v[2] = (_Float16)(a.z * inv);
    h.v[3] = (_Float16)a.w;
    h.v[4] = (_Float16)b.x;
    h.v[5] = h.v[6] = h.v[7] = (_Float16)0.0f;
    ((Half8*)out)[t] = h;
  } else {
    ((float4*)out)[2 * t] = a;
    ((float4*)out)[2 * t + 1] = b;
  }
}

// stored texels back to (R, G, B, p_u) (p_v, 0, 0, 0) records in the caller's units
__global__ void k_star_unpack_bands(const void* __restrict__ in, int64_t count, float scale,
                                    int fp16, float4* __restrict__ out) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= count) return;
  if (fp16) {
    const Half8 h = ((const Half8*)in)[t];
    out[2 * t] = make_float4((float)h.v[0] * scale, (float)h.v[1] * scale,
                             (float)h.v[2] * scale, (float)h.v[3]);
    out[2 * t + 1] = make_float4((float)h.v[4], 0.f, 0.f, 0.f);
  } else {
    out[2 * t] = ((const float4*)in)[2 * t];
    out[2 * t + 1] = ((const float4*)in)[2 * t + 1];
  }
}

// Occupancy bits of a band map (a texel is occupied when a stored band is positive);
// layout as k_star_occupancy.
__global__ void k_star_occupancy_bands(const void* __restrict__ tex, int nl, int fp16,
                                       uint32_t* __restrict__ occ) {
  const int wpr = ((nl + 31) >> 5) + 1;
  int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t total = 6LL * 2 * nl * wpr;
  if (w >= total) return;
  int wi;
  int64_t row;
  uint32_t bits = 0;
  if (occ_word_row(w, nl, wpr, &wi, &row)) {
    for (int b = 0; b < 32; ++b) {
      int x = wi * 32 + b;
      if (x >= nl) break;
      int64_t t = row * nl + x;
      bool lit;
      if (fp16) {
        const Half8 h = ((const Half8*)tex)[t];
        lit = (float)h.v[0] > 0.0f || (float)h.v[1] > 0.0f || (float)h.v[2] > 0.0f;
      } else {
        const float4 a = ((const float4*)tex)[2 * t];
        lit = a.x > 0.0f || a.y > 0.0f || a.z > 0.0f;
      }
      if (lit) bits |= 1u << b;
    }
  }
  occ[w] = bits;
}

// Build every level of a band map; scratch as launch_star_build with `master` holding two
// float4 per texel.
hipError_t launch_star_build_bands(const float* dirs, const float* rgb, int64_t n, int n0,
                                   int levels, const uint32_t* level_off_host, int* head,
                                   int* next, float2* pos, float4* master, unsigned* maxbits,
                                   float* scale, int fp16, void* out, int* bad, hipStream_t s) {
  const int B = 256;
  int64_t ntex0 = 6LL * n0 * n0;
  if (n > 0)
    hipLaunchKernelGGL(k_star_link_bands, dim3(blocks_for(n, B)), dim3(B), 0, s, dirs, rgb, n,
                       n0, head, next, pos, bad);
  hipLaunchKernelGGL(k_star_reduce0_bands, dim3(blocks_for(ntex0, B)), dim3(B), 0, s, head, next,
                     rgb, pos, ntex0, master);
  for (int l = 1; l < levels; ++l) {
    int nc = n0 >> l;
    hipLaunchKernelGGL(k_star_mip_bands, dim3(blocks_for(6LL * nc * nc, B)), dim3(B), 0, s,
                       master + 2 * (int64_t)level_off_host[l - 1],
                       master + 2 * (int64_t)level_off_host[l], nc);
  }
  for (int l = 0; l < levels; ++l) {
    int64_t cnt = 6LL * (n0 >> l) * (n0 >> l);
    unsigned grid = std::min(blocks_for(cnt, B), 2048u);
    hipLaunchKernelGGL(k_star_maxI_bands, dim3(grid), dim3(B), 0, s,
                       master + 2 * (int64_t)level_off_host[l], cnt, maxbits + l);
  }
  hipLaunchKernelGGL(k_star_scales, dim3(1), dim3(64), 0, s, maxbits, levels, fp16, scale);
  const size_t tsz = fp16 ? 16 : 32;
  for (int l = 0; l < levels; ++l) {
    int64_t cnt = 6LL * (n0 >> l) * (n0 >> l);
    hipLaunchKernelGGL(k_star_pack_bands, dim3(blocks_for(cnt, B)), dim3(B), 0, s,
                       master + 2 * (int64_t)level_off_host[l], cnt, scale, l, fp16,
                       (void*)((char*)out + tsz * level_off_host[l]));
  }
  return hipGetLastError();
}

hipError_t launch_star_occupancy_bands(const void* tex, int n0, int levels,
                                       const uint32_t* level_off, const uint32_t* occ_off,
                                       int fp16, uint32_t* occ, hipStream_t s) {
  const size_t tsz = fp16 ? 16 : 32;
  for (int l = 0; l < levels; ++l) {
    int nl = n0 >> l;
    int64_t words = 6LL * 2 * nl * (((nl + 31) >> 5) + 1);
    hipLaunchKernelGGL(k_star_occupancy_bands, dim3(blocks_for(words, 256)), dim3(256), 0, s,
                       (const void*)((const char*)tex + tsz * level_off[l]), nl, fp16,
                       occ + occ_off[l]);
  }
  return hipGetLastError();
}

hipError_t launch_star_unpack_bands(const void* in, int64_t count, float scale, int fp16,
                                    float4* out, hipStream_t s) {
  hipLaunchKernelGGL(k_star_unpack_bands, dim3(blocks_for(count, 256)), dim3(256), 0, s, in,
                     count, scale, fp16, out);
  return hipGetLastError();
}

// Content hash of a star field, the key under which its maps are shared: every star
// contributes a 64-bit mix of its index and the bit patterns of its five floats, and the
// contributions are summed with integer atomics (addition commutes, so the result does
// not depend on the order the atomics run in).  The mix is the splitmix64 finaliser.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256)
    k_star_hash(const float* __restrict__ dirs, const float* __restrict__ inten,
                const float* __restrict__ temp, int64_t n, unsigned long long* __restrict__ acc) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  uint64_t h = 0;
  if (s < n) {
    h = mix64((uint64_t)s + 0x9e3779b97f4a7c15ull);
    h = mix64(h ^ __float_as_uint(dirs[3 * s]));
    h = mix64(h ^ ((uint64_t)__float_as_uint(dirs[3 * s + 1]) << 32));
    h = mix64(h ^ __float_as_uint(dirs[3 * s + 2]));
    h = mix64(h ^ ((uint64_t)__float_as_uint(inten[s]) << 32));
    h = mix64(h ^ __float_as_uint(temp[s]));
  }
  for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o);
  if ((threadIdx.x & 63) == 0 && s - (threadIdx.x & 63) < n) atomicAdd(acc, (unsigned long long)h);
}

hipError_t launch_star_hash(const float* dirs, const float* inten, const float* temp, int64_t n,
                            unsigned long long* acc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_star_hash, dim3(blocks_for(n, 256)), dim3(256), 0, s, dirs, inten, temp,
                     n, acc);
  return hipGetLastError();
}

// Content hash of a band-colour star field: as k_star_hash over the direction and the three
// band values, from a different seed so a band field never shares a key with an (I, T) field.
__global__ void __launch_bounds__(256)
    k_star_hash_bands(const float* __restrict__ dirs, const float* __restrict__ rgb, int64_t n,
                      unsigned long long* __restrict__ acc) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  uint64_t h = 0;
  if (s < n) {
    h = mix64((uint64_t)s + 0x632be59bd9b4e019ull);
    h = mix64(h ^ __float_as_uint(dirs[3 * s]));
    h = mix64(h ^ ((uint64_t)__float_as_uint(dirs[3 * s + 1]) << 32));
    h = mix64(h ^ __float_as_uint(dirs[3 * s + 2]));
    h = mix64(h ^ ((uint64_t)__float_as_uint(rgb[3 * s]) << 32));
    h = mix64(h ^ __float_as_uint(rgb[3 * s + 1]));
    h = mix64(h ^ ((uint64_t)__float_as_uint(rgb[3 * s + 2]) << 32));
  }
  for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o);
  if ((threadIdx.x & 63) == 0 && s - (threadIdx.x & 63) < n) atomicAdd(acc, (unsigned long long)h);
}

hipError_t launch_star_hash_bands(const float* dirs, const float* rgb, int64_t n,
                                  unsigned long long* acc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_star_hash_bands, dim3(blocks_for(n, 256)), dim3(256), 0, s, dirs, rgb, n,
                     acc);
  return hipGetLastError();
}

__global__ void k_fill_int(int* p, int64_t n, int v) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_star_unpack(const void* in, int64_t count, float scale, int fp16, float4* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_star_unpack, dim3(blocks_for(count, 256)), dim3(256), 0, s, in, count,
                     scale, fp16, out);
  return hipGetLastError();
}

}  // namespace bh
