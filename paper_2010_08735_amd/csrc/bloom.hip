// Bloom (lens glare, Section 3.4.3): a point spread function approximated by small-support
// filters on the mipmaps of the final image, before tone mapping.
//
//   P_0 = I;  P_k = 2x2 box average of P_{k-1} (ceil(n/2) per axis, clamped source indices)
//   U_K = w_K P_K;  U_k = w_k P_k + up(U_{k+1});  O = w_0 I + up(U_1)
//
// up() doubles the resolution bilinearly: fine pixel x reads the coarse grid at x/2 - 1/4,
// i.e. coarse pixels (x-1)>>1 and (x+1)>>1 with weights 3/4, 1/4 (or 1/4, 3/4), clamped to
// the edge.  With weights summing to 1 an interior impulse keeps its flux.
//
// Three launches:
//   k_bloom_down  one workgroup per 64x64 image tile builds the tile's levels 1..6 in LDS
//                 (a level-k pixel depends on a 2^k x 2^k block of the image, inside one
//                 tile) and writes them (HBM-bound: reads the image once);
//   k_bloom_tail  one workgroup builds the coarse levels 7..K and their U chain, which are
//                 small (at most 120 x 68 pixels at 7680 x 4320), only when K > 7 (for
//                 K = 7 the output pass forms the U_7 values it needs from level 6);
//   k_bloom_up    one workgroup per 64x64 output tile (32x32 when encoding for display)
//                 runs the U chain for levels 6..1 over the tile plus the one-pixel halo each
//                 bilinear doubling needs, in LDS, then writes O (HBM-bound: reads the image
//                 once more, writes O), or O's display encoding (below) in place of O.
//
// Display encoding (the tone mapping that follows the glare pass; the paper prints no
// operator, so this is one reading): per colour channel c, x = exposure * c, y = 1 - exp(-x)
// (0 for x <= 0 or NaN), v = the sRGB transfer function of y (IEC 61966-2-1), 8-bit code
// floor(255 v + 1/2); alpha 255; bytes R, G, B, A.  k_tonemap applies it to a whole image.
#include "bh_dev.h"

namespace bh {

constexpr int kBloomTileLevels = 6;  // levels built inside a 64 x 64 tile

__device__ __forceinline__ float4 f4_fma(float a, float4 x, float4 y) {
  return make_float4(fmaf(a, x.x, y.x), fmaf(a, x.y, y.y), fmaf(a, x.z, y.z), fmaf(a, x.w, y.w));
}

__device__ __forceinline__ float4 box4(float4 a, float4 b, float4 c, float4 d) {
  return make_float4(0.25f * ((a.x + b.x) + (c.x + d.x)), 0.25f * ((a.y + b.y) + (c.y + d.y)),
                     0.25f * ((a.z + b.z) + (c.z + d.z)), 0.25f * ((a.w + b.w) + (c.w + d.w)));
}

// bilinear blend of the four coarse neighbours of a fine pixel (fx, fy: weights of the
// second column / row, 1/4 or 3/4)
__device__ __forceinline__ float4 blend(float4 v00, float4 v10, float4 v01, float4 v11, float fx,
                                        float fy) {
  const float gx = 1.0f - fx, gy = 1.0f - fy;
  float4 a = make_float4(gx * v00.x + fx * v10.x, gx * v00.y + fx * v10.y, gx * v00.z + fx * v10.z,
                         gx * v00.w + fx * v10.w);
  float4 b = make_float4(gx * v01.x + fx * v11.x, gx * v01.y + fx * v11.y, gx * v01.z + fx * v11.z,
                         gx * v01.w + fx * v11.w);
  return make_float4(gy * a.x + fy * b.x, gy * a.y + fy * b.y, gy * a.z + fy * b.z,
                     gy * a.w + fy * b.w);
}

// ---- display encoding ------------------------------------------------------------------------

// 8-bit code of one colour channel.  1 - exp(-x) loses ~1e-7 absolute to cancellation, which
// the linear sRGB segment (3295 codes per unit) would turn into 4e-4 codes, so below x = 1/16
// it comes from its Taylor series to x^5 (truncation below 1e-9 relative).  With hardware
// exp2 and log2 (about 1 ulp each) the value whose floor is the code stays within 2e-4 of its
// exact value.
__device__ __forceinline__ uint32_t display_code(float c, float exposure) {
  const float x = exposure * c;
  if (!(x > 0.0f)) return 0u;
  const float series =
      x * fmaf(-x, fmaf(-x, fmaf(-x, fmaf(-x, 1.0f / 120.0f, 1.0f / 24.0f), 1.0f / 6.0f), 0.5f),
               1.0f);
  const float y = x < 0.0625f ? series
                              : 1.0f - __builtin_amdgcn_exp2f(x * -1.44269504088896341f);
  const float v = y <= 0.0031308f
                      ? 12.92f * y
                      : fmaf(1.055f,
                             __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(y) * (1.0f / 2.4f)),
                             -0.055f);
  return min((uint32_t)fmaf(255.0f, v, 0.5f), 255u);  // v >= 0: truncation is the floor
}

__device__ __forceinline__ uint32_t display_pixel(float4 c, float exposure) {
  return display_code(c.x, exposure) | (display_code(c.y, exposure) << 8) |
         (display_code(c.z, exposure) << 16) | 0xff000000u;
}

__global__ void __launch_bounds__(256)
    k_tonemap(const float4* __restrict__ in, uint32_t* __restrict__ out, int64_t n,
              float exposure) {
  // two pixels per thread, one grid apart (both loads in flight before either encoding);
  // the launch has ceil(n / 512) workgroups, so i0 + step covers the rest of the image
  const int64_t step = (int64_t)gridDim.x * 256;
  const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x, i1 = i0 + step;
  const float4 a = i0 < n ? in[i0] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const float4 b = i1 < n ? in[i1] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (i0 < n) store_stream(&out[i0], display_pixel(a, exposure));
  if (i1 < n) store_stream(&out[i1], display_pixel(b, exposure));
}

// ---- level building inside one 64 x 64 tile --------------------------------------------------

// LDS holds level k of the tile at local index l for every l in [0, 64 / 2^k), also beyond
// the level's last pixel: an entry past it holds the last pixel's value (its index clamped),
// so the next level's 2x2 averages need no clamping of their own.
__global__ void __launch_bounds__(256)
    k_bloom_down(const float4* __restrict__ img, float4* __restrict__ P, BloomDev B) {
  __shared__ float4 s1[32 * 32];
  __shared__ float4 s2[16 * 16];
  const int tx = blockIdx.x % B.tiles_x, ty = blockIdx.x / B.tiles_x;
  const int m = min(B.levels, kBloomTileLevels);
  const int t = threadIdx.x;
  float4* cur = s1;
  float4* nxt = s2;
  // level 1 from the image
  {
    const int n1x = B.w[1], n1y = B.h[1];
    for (int l = t; l < 32 * 32; l += 256) {
      const int lx = l & 31, ly = l >> 5;
      const int gx = tx * 32 + lx, gy = ty * 32 + ly;
      const int cx = min(gx, n1x - 1), cy = min(gy, n1y - 1);
      const int x0 = 2 * cx, y0 = 2 * cy;
      const int x1 = min(x0 + 1, B.w[0] - 1), y1 = min(y0 + 1, B.h[0] - 1);
      const float4 v = box4(img[(size_t)y0 * B.w[0] + x0], img[(size_t)y0 * B.w[0] + x1],
                            img[(size_t)y1 * B.w[0] + x0], img[(size_t)y1 * B.w[0] + x1]);
      cur[l] = v;
      if (gx < n1x && gy < n1y) P[B.off[1] + (size_t)gy * n1x + gx] = v;
    }
  }
  __syncthreads();
  // levels 2 .. m from the previous level in LDS
  for (int k = 2; k <= m; ++k) {
    const int lside = 6 - k, side = 1 << lside, pside = side * 2;
    const int nx = B.w[k], ny = B.h[k];
    const int sx = tx * side, sy = ty * side;  // the tile's first level-k pixel
    for (int l = t; l < side * side; l += 256) {
      const int lx = l & (side - 1), ly = l >> lside;
      const int cx = min(sx + lx, nx - 1) - sx, cy = min(sy + ly, ny - 1) - sy;
      const float4 v = box4(cur[(2 * cy) * pside + 2 * cx], cur[(2 * cy) * pside + 2 * cx + 1],
                            cur[(2 * cy + 1) * pside + 2 * cx],
                            cur[(2 * cy + 1) * pside + 2 * cx + 1]);
      nxt[l] = v;
      if (sx + lx < nx && sy + ly < ny) P[B.off[k] + (size_t)(sy + ly) * nx + sx + lx] = v;
    }
    __syncthreads();
    float4* sw = cur;
    cur = nxt;
    nxt = sw;
  }
}

// levels 7 .. K and U_K .. U_7, one workgroup, a barrier between levels.  LDS: the levels live
// in shared memory (U_k overwrites P_k in place) and only U_7, which the output tiles read, goes
// to global memory; used when levels 7 .. K hold at most kBloomTailLds pixels (7680 x 4320
// needs 2685).  Otherwise the levels are kept in global memory.
constexpr int kBloomTailLds = 3072;

template <bool LDS>
__global__ void __launch_bounds__(256)
    k_bloom_tail(float4* __restrict__ P, float4* __restrict__ U, BloomDev B) {
  __shared__ float4 sl[LDS ? kBloomTailLds : 1];
  const int t = threadIdx.x;
  const int64_t base = B.off[kBloomTileLevels + 1];
  for (int k = kBloomTileLevels + 1; k <= B.levels; ++k) {
    const int nx = B.w[k], ny = B.h[k], px = B.w[k - 1], py = B.h[k - 1];
    for (int l = t; l < nx * ny; l += 256) {
      const int x = l % nx, y = l / nx;
      const int x0 = 2 * x, y0 = 2 * y, x1 = min(x0 + 1, px - 1), y1 = min(y0 + 1, py - 1);
      float4 v;
      if (!LDS || k == kBloomTileLevels + 1) {
        const float4* src = P + B.off[k - 1];
        v = box4(src[(size_t)y0 * px + x0], src[(size_t)y0 * px + x1],
                 src[(size_t)y1 * px + x0], src[(size_t)y1 * px + x1]);
      } else {
        const float4* src = sl + (B.off[k - 1] - base);
        v = box4(src[y0 * px + x0], src[y0 * px + x1], src[y1 * px + x0], src[y1 * px + x1]);
      }
      if (LDS)
        sl[B.off[k] - base + l] = v;
      else
        P[B.off[k] + l] = v;
    }
    __syncthreads();
  }
  for (int k = B.levels; k > kBloomTileLevels; --k) {
    const int nx = B.w[k], ny = B.h[k];
    const float wk = B.wt[k];
    for (int l = t; l < nx * ny; l += 256) {
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (k < B.levels) {
        const int x = l % nx, y = l / nx, cx = B.w[k + 1], cy = B.h[k + 1];
        const int xa = max((x - 1) >> 1, 0), xb = min((x + 1) >> 1, cx - 1);
        const int ya = max((y - 1) >> 1, 0), yb = min((y + 1) >> 1, cy - 1);
        const float4* c = LDS ? sl + (B.off[k + 1] - base) : U + B.off[k + 1];
        v = blend(c[ya * cx + xa], c[ya * cx + xb], c[yb * cx + xa], c[yb * cx + xb],
                  (x & 1) ? 0.25f : 0.75f, (y & 1) ? 0.25f : 0.75f);
      }
      const float4 u = f4_fma(wk, LDS ? sl[B.off[k] - base + l] : P[B.off[k] + l], v);
      if (LDS) {
        sl[B.off[k] - base + l] = u;
        if (k == kBloomTileLevels + 1) U[B.off[k] + l] = u;
      } else {
        U[B.off[k] + l] = u;
      }
    }
    __syncthreads();
  }
}

// ---- the U chain and the output, per T x T output tile ------------------------------------------
//
// A tile reads level-1 pixels T t / 2 - 1 .. T t / 2 + T / 2 (T / 2 + 2 per axis), level-2
// pixels T / 4 + 2 per axis, and so on down to 3 at level 6.  Odd levels are kept in LDS
// buffer `sa` (row stride SA), even levels in `sb` (stride SB).  Every P value a tile needs is
// loaded into registers first, so the chain of levels waits on LDS only.
template <int T, int K>
struct UpLevel {
  static constexpr int S = (K & 1) ? T / 2 + 2 : T / 4 + 2;  // LDS row stride
  // rows of the region, at most: T / 2^K + 2 while that is at least 3, then 3
  static constexpr int ROWS = T / (1 << K) + 2 < 3 ? 3 : T / (1 << K) + 2;
  static constexpr int N = (S * ROWS + 255) / 256;           // slots per thread
  static_assert(ROWS <= S, "a region's rows and columns fit the LDS row stride");
};

struct Region {
  int lox, hix, loy, hiy;
};

// P_k over the region, slot j of this thread = element threadIdx.x + 256 j of the region in
// row-major order with row stride S (entries outside the region are not loaded)
template <int T, int K>
__device__ __forceinline__ void load_p(const BloomDev& B, const float4* __restrict__ P,
                                       const Region& R, float4 (&p)[UpLevel<T, K>::N]) {
  using L = UpLevel<T, K>;
#pragma unroll
  for (int j = 0; j < L::N; ++j) {
    const int l = threadIdx.x + 256 * j;
    const int r = l / L::S, c = l - r * L::S;
    if (c <= R.hix - R.lox && r <= R.hiy - R.loy)
      p[j] = P[B.off[K] + (size_t)(R.loy + r) * B.w[K] + R.lox + c];
  }
}

// U_7 = w_7 P_7 at level-7 pixel (x, y) of a pyramid of exactly 7 levels, from level 6: the
// operations of the tail kernel, in its order, so the values are the same bits
__device__ __forceinline__ float4 u7_from_p6(const BloomDev& B, const float4* __restrict__ P,
                                             int x, int y) {
  constexpr int K = kBloomTileLevels + 1;
  const int px = B.w[K - 1], py = B.h[K - 1];
  const int x0 = 2 * x, y0 = 2 * y, x1 = min(x0 + 1, px - 1), y1 = min(y0 + 1, py - 1);
  const float4* src = P + B.off[K - 1];
  const float4 p = box4(src[(size_t)y0 * px + x0], src[(size_t)y0 * px + x1],
                        src[(size_t)y1 * px + x0], src[(size_t)y1 * px + x1]);
  return f4_fma(B.wt[K], p, make_float4(0.f, 0.f, 0.f, 0.f));
}

// The level-7 neighbourhood of a tile's level-6 region R: at most 3 x 3 pixels
__device__ __forceinline__ Region coarse_region(const BloomDev& B, const Region& R) {
  constexpr int K = kBloomTileLevels + 1;
  return Region{max((R.lox - 1) >> 1, 0), min((R.hix + 1) >> 1, B.w[K] - 1),
                max((R.loy - 1) >> 1, 0), min((R.hiy + 1) >> 1, B.h[K] - 1)};
}
constexpr int kU7Max = 16;  // >= 3 x 3

// U_7 over the coarse region C of a 7-level pyramid, one value per thread, into LDS `su7`
// (row stride 4)
__device__ __forceinline__ void fill_u7(const BloomDev& B, const float4* __restrict__ P,
                                        const Region& C, float4* su7) {
  const int t = threadIdx.x, w = C.hix - C.lox + 1, h = C.hiy - C.loy + 1;
  if (t < w * h) {
    const int x = t % w, y = t / w;
    su7[y * 4 + x] = u7_from_p6(B, P, C.lox + x, C.loy + y);
  }
}

// U_7 at the four coarse neighbours of every level-6 element of the region (only when the
// pyramid has more than 6 levels): with exactly 7, from `su7` (fill_u7, region C); with
// more, from the global U array the tail kernel wrote
template <int T>
__device__ __forceinline__ void load_u_coarse(const BloomDev& B, const float4* __restrict__ U,
                                              const Region& R, const float4* su7,
                                              const Region& C,
                                              float4 (&q)[UpLevel<T, kBloomTileLevels>::N][4]) {
  using L = UpLevel<T, kBloomTileLevels>;
  constexpr int K = kBloomTileLevels;
  const int cnx = B.w[K + 1], cny = B.h[K + 1];
  const float4* cu = U + B.off[K + 1];
  const bool direct = B.levels == K + 1;
#pragma unroll
  for (int j = 0; j < L::N; ++j) {
    // slots outside the region load a neighbour of its last element, unused: loads that
    // every lane issues keep the chain's waits on earlier loads exact
    const int l = threadIdx.x + 256 * j;
    const int r = l / L::S, c = l - r * L::S;
    const int x = R.lox + min(c, R.hix - R.lox), y = R.loy + min(r, R.hiy - R.loy);
    const int xa = max((x - 1) >> 1, 0), xb = min((x + 1) >> 1, cnx - 1);
    const int ya = max((y - 1) >> 1, 0), yb = min((y + 1) >> 1, cny - 1);
    if (direct) {
      q[j][0] = su7[(ya - C.loy) * 4 + xa - C.lox];
      q[j][1] = su7[(ya - C.loy) * 4 + xb - C.lox];
      q[j][2] = su7[(yb - C.loy) * 4 + xa - C.lox];
      q[j][3] = su7[(yb - C.loy) * 4 + xb - C.lox];
    } else {
      q[j][0] = cu[(size_t)ya * cnx + xa];
      q[j][1] = cu[(size_t)ya * cnx + xb];
      q[j][2] = cu[(size_t)yb * cnx + xa];
      q[j][3] = cu[(size_t)yb * cnx + xb];
    }
  }
}

// U_K = w_K P_K + up(U_{K+1}) over the region, into `dst`.  U_{K+1} comes from LDS (`src`,
// region Rs, stride of level K + 1) for K < 6, from the preloaded values `q` for K = 6, and
// is absent for K = levels.  The chain itself reads no global memory, so its waits cover
// only the loads it uses.
template <int T, int K>
__device__ __forceinline__ void u_level(const BloomDev& B, const float4 (&p)[UpLevel<T, K>::N],
                                        const float4 (*q)[4], const Region& R, const float4* src,
                                        const Region& Rs, float4* dst) {
  using L = UpLevel<T, K>;
  constexpr int SS = UpLevel<T, K + 1>::S;
  const float wk = B.wt[K];
#pragma unroll
  for (int j = 0; j < L::N; ++j) {
    const int l = threadIdx.x + 256 * j;
    const int r = l / L::S, c = l - r * L::S;
    if (c > R.hix - R.lox || r > R.hiy - R.loy) continue;
    const int x = R.lox + c, y = R.loy + r;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (K < B.levels) {
      float4 v00, v10, v01, v11;
      if constexpr (K == kBloomTileLevels) {
        v00 = q[j][0];
        v10 = q[j][1];
        v01 = q[j][2];
        v11 = q[j][3];
      } else {
        const int cnx = B.w[K + 1], cny = B.h[K + 1];
        const int xa = max((x - 1) >> 1, 0), xb = min((x + 1) >> 1, cnx - 1);
        const int ya = max((y - 1) >> 1, 0), yb = min((y + 1) >> 1, cny - 1);
        v00 = src[(ya - Rs.loy) * SS + xa - Rs.lox];
        v10 = src[(ya - Rs.loy) * SS + xb - Rs.lox];
        v01 = src[(yb - Rs.loy) * SS + xa - Rs.lox];
        v11 = src[(yb - Rs.loy) * SS + xb - Rs.lox];
      }
      v = blend(v00, v10, v01, v11, (x & 1) ? 0.25f : 0.75f, (y & 1) ? 0.25f : 0.75f);
    }
    dst[l] = f4_fma(wk, p[j], v);
  }
}

// Output tile edge: 64 for the linear output; 32 when the pass also encodes for display, whose
// per-pixel arithmetic (three transcendentals per channel at the end of each workgroup)
// overlaps other workgroups' memory traffic better with four times as many of them.
constexpr int kBloomUpTile = 64, kBloomUpTileDisplay = 32;

// DISPLAY: `out` receives the display encoding of O (uint32 per pixel), else O (float4)
template <int T, bool DISPLAY>
__global__ void __launch_bounds__(256)
    k_bloom_up(const float4* __restrict__ img, void* __restrict__ out,
               const float4* __restrict__ P, const float4* __restrict__ U, BloomDev B,
               float exposure) {
  constexpr int SA = UpLevel<T, 1>::S, SB = UpLevel<T, 2>::S;
  static_assert(UpLevel<T, 3>::S == SA && UpLevel<T, 4>::S == SB, "odd / even strides");
  static_assert(256 % T == 0 && T % (256 / T) == 0, "whole rows per pass, whole passes per tile");
  __shared__ float4 sa[SA * SA];
  __shared__ float4 sb[SB * SB];
  const int ntx = (B.w[0] + T - 1) / T;
  const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
  const int m = min(B.levels, kBloomTileLevels);
  // regions of levels 0 .. 6
  Region R[kBloomTileLevels + 1];
  R[0].lox = tx * T;
  R[0].hix = min(R[0].lox + T - 1, B.w[0] - 1);
  R[0].loy = ty * T;
  R[0].hiy = min(R[0].loy + T - 1, B.h[0] - 1);
#pragma unroll
  for (int k = 1; k <= kBloomTileLevels; ++k) {
    const int nx = B.w[min(k, B.levels)], ny = B.h[min(k, B.levels)];
    R[k].lox = max((R[k - 1].lox - 1) >> 1, 0);
    R[k].hix = min((R[k - 1].hix + 1) >> 1, nx - 1);
    R[k].loy = max((R[k - 1].loy - 1) >> 1, 0);
    R[k].hiy = min((R[k - 1].hiy + 1) >> 1, ny - 1);
  }
  // every P value of the chain, in flight at once (levels beyond m are not loaded)
  float4 p1[UpLevel<T, 1>::N], p2[UpLevel<T, 2>::N], p3[UpLevel<T, 3>::N],
      p4[UpLevel<T, 4>::N], p5[UpLevel<T, 5>::N], p6[UpLevel<T, 6>::N];
  if (m >= 6) load_p<T, 6>(B, P, R[6], p6);
  if (m >= 5) load_p<T, 5>(B, P, R[5], p5);
  if (m >= 4) load_p<T, 4>(B, P, R[4], p4);
  if (m >= 3) load_p<T, 3>(B, P, R[3], p3);
  if (m >= 2) load_p<T, 2>(B, P, R[2], p2);
  if (m >= 1) load_p<T, 1>(B, P, R[1], p1);
  float4 q6[UpLevel<T, 6>::N][4];
  __shared__ float4 su7[kU7Max];
  const Region C7 = coarse_region(B, R[6]);
  if (B.levels == kBloomTileLevels + 1) {  // uniform: the barrier is reached by all threads
    fill_u7(B, P, C7, su7);
    __syncthreads();
  }
  if (B.levels > kBloomTileLevels) load_u_coarse<T>(B, U, R[6], su7, C7, q6);
  // this thread's image pixels (column x, rows y0 + kRows j), in flight during the chain;
  // positions past the image's edge load the edge pixel, unused
  constexpr int kRows = 256 / T, kIt = T / kRows;
  const int x = R[0].lox + (int)(threadIdx.x % T);
  const int y0 = R[0].loy + (int)(threadIdx.x / T);
  const bool xin = x <= R[0].hix;
  float4 im[kIt];
#pragma unroll
  for (int j = 0; j < kIt; ++j)
    im[j] = img[(size_t)min(y0 + kRows * j, R[0].hiy) * B.w[0] + min(x, R[0].hix)];
  // U_k, k = m .. 1 (m is the same for the whole launch, so the barriers are uniform)
  if (m >= 6) { u_level<T, 6>(B, p6, q6, R[6], sa, R[6], sb); __syncthreads(); }
  if (m >= 5) { u_level<T, 5>(B, p5, nullptr, R[5], sb, R[6], sa); __syncthreads(); }
  if (m >= 4) { u_level<T, 4>(B, p4, nullptr, R[4], sa, R[5], sb); __syncthreads(); }
  if (m >= 3) { u_level<T, 3>(B, p3, nullptr, R[3], sb, R[4], sa); __syncthreads(); }
  if (m >= 2) { u_level<T, 2>(B, p2, nullptr, R[2], sa, R[3], sb); __syncthreads(); }
  if (m >= 1) { u_level<T, 1>(B, p1, nullptr, R[1], sb, R[2], sa); __syncthreads(); }
  // O = w_0 I + up(U_1)
  const float w0 = B.wt[0];
  if (!xin) return;
#pragma unroll
  for (int j = 0; j < kIt; ++j) {
    const int y = y0 + kRows * j;
    if (y > R[0].hiy) break;
    const size_t i = (size_t)y * B.w[0] + x;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (B.levels >= 1) {
      const int cnx = B.w[1], cny = B.h[1];
      const int xa = max((x - 1) >> 1, 0) - R[1].lox, xb = min((x + 1) >> 1, cnx - 1) - R[1].lox;
      const int ya = max((y - 1) >> 1, 0) - R[1].loy, yb = min((y + 1) >> 1, cny - 1) - R[1].loy;
      v = blend(sa[ya * SA + xa], sa[ya * SA + xb], sa[yb * SA + xa], sa[yb * SA + xb],
                (x & 1) ? 0.25f : 0.75f, (y & 1) ? 0.25f : 0.75f);
    }
    const float4 o = f4_fma(w0, im[j], v);
    if constexpr (DISPLAY)
      store_stream(&static_cast<uint32_t*>(out)[i], display_pixel(o, exposure));
    else
      store_stream(&static_cast<float4*>(out)[i], o);
  }
}

hipError_t launch_tonemap(const float4* in, uint32_t* out, int64_t n, float exposure,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_tonemap, dim3((unsigned)((n + 511) / 512)), dim3(256), 0, s, in, out, n,
                     exposure);
  return hipGetLastError();
}

// display: write the display encoding of O (exposure) to `out` (uint32 per pixel), else O
hipError_t launch_bloom(const float4* in, void* out, float4* P, float4* U, const BloomDev& B,
                        bool display, float exposure, hipStream_t s) {
  const int tiles = B.tiles_x * B.tiles_y;
  if (B.levels >= 1) {
    hipLaunchKernelGGL(k_bloom_down, dim3(tiles), dim3(256), 0, s, in, P, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // with exactly 7 levels the output pass computes the few U_7 values it needs itself
  if (B.levels > kBloomTileLevels + 1) {
    const int64_t tail = B.off[B.levels] + (int64_t)B.w[B.levels] * B.h[B.levels] -
                         B.off[kBloomTileLevels + 1];
    if (tail <= kBloomTailLds)
      hipLaunchKernelGGL(k_bloom_tail<true>, dim3(1), dim3(256), 0, s, P, U, B);
    else
      hipLaunchKernelGGL(k_bloom_tail<false>, dim3(1), dim3(256), 0, s, P, U, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int T = display ? kBloomUpTileDisplay : kBloomUpTile;
  const int ut = ((B.w[0] + T - 1) / T) * ((B.h[0] + T - 1) / T);
  if (display)
    hipLaunchKernelGGL((k_bloom_up<kBloomUpTileDisplay, true>), dim3(ut), dim3(256), 0, s, in,
                       out, P, U, B, exposure);
  else
    hipLaunchKernelGGL((k_bloom_up<kBloomUpTile, false>), dim3(ut), dim3(256), 0, s, in, out, P,
                       U, B, exposure);
  return hipGetLastError();
}

}  // namespace bh
