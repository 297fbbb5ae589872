// Device-side records and helpers shared by the libbh HIP kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bh.h"

// AOV flag bits (see include/bh.h)
#define BH_CAPTURED_BIT BH_AOV_CAPTURED
#define BH_CROSS0_BIT BH_AOV_CROSS0
#define BH_CROSS1_BIT BH_AOV_CROSS1
#define BH_STAR_ZEROED_BIT BH_AOV_STAR_ZEROED
#define BH_DEGENERATE_BIT BH_AOV_DEGENERATE
#define BH_UNFINISHED_BIT BH_AOV_UNFINISHED

namespace bh {

// mu = 4/27: maximum of u^2 (1 - u), reached at the photon sphere u = 2/3 (Section 3.3.1)
constexpr float kMu = 4.0f / 27.0f;
constexpr double kMuD = 4.0 / 27.0;
constexpr float kPi = 3.14159265358979323846f;

// ---- tables -------------------------------------------------------------------------
struct TablesDev {
  const float* D;   // d_n x d_n, row j (u coordinate) major
  const float* U;   // u_nphi x u_ne, row j (phi coordinate) major
  const float* Dt;  // time channels: e tau (regularised time) in the layouts of D and U
  const float* Ut;
  int d_n, u_ne, u_nphi, pad;
};

// ---- blackbody band table -----------------------------------------------------------
// lut[k] = (log2 L_R, log2 L_G, log2 L_B, log2(L_R + L_G + L_B)) at log2 T = x0 + k dx
struct LutDev {
  const float4* lut;
  int n;
  float x0, inv_dx, pad;
};

// ---- star map -------------------------------------------------------------------------
struct StarsDev {
  const void* tex;        // all levels, level L at element offset level_off[L]
  const float* scale;     // per-level intensity scale (FP16 format), 1 for FP32
  const uint32_t* level_off;  // texel offset of each level (<= 2^32 texels)
  const uint32_t* occ;    // occupancy bits, level L at word offset occ_off[L]
  const uint32_t* occ_off;
  int n0, levels, fp16;
  float one;              // 1.0 (a run-time constant, see the gather)
  float tw0;              // 2 / n0: width of a level-0 texel in face coordinates (n0 = 2^k)
  int bands;              // 1: band-colour texels (R, G, B, p_u, p_v), received through `ctab`
  const float4* ctab;     // colour-shift table of the context (band maps), else null
};
static_assert(sizeof(StarsDev) == 72, "the star-map record keeps the view record's layout");

// ---- area-source map (nebulae, galaxies) ----------------------------------------------
// (I, I T) per texel: radiance and radiance-weighted colour temperature; level L (size
// n0 >> L, n0 a power of two) starts at texel 8 (n0^2 - nL^2), within it face-major rows.
struct AreaDev {
  const void* tex;        // null: no area map; float2 (I, I T) texels, or float4 (R, G, B, 0)
  int n0, levels;
  float k_area;
  int bands;              // 1: band texels, received through the colour-shift table `ctab`
  const float4* ctab;     // log2 C_b at kCshiftN^3 nodes (cshift.hip)
};

// Colour-shift table (Section 3.4.2): nodes per axis (r, g, log2 D over [-3, 3])
constexpr int kCshiftN = 128;

// Gauss-Legendre nodes and weights on [-1, 1] for the table's band integrals
struct CshiftRule {
  double x[8], w[8];
};

// Optional per-view work the render kernels are specialised for (a kernel without a
// feature carries none of its code or registers): a particle disc, an area-source map.
// kFeatBands: band colours received through the colour-shift table, from an area map (then
// with kFeatArea) or a star map.
constexpr int kFeatParticles = 1, kFeatArea = 2, kFeatBands = 4;

// ---- per-view constant block (host computes it in FP64 from bh_view) -----------------
// The camera axes and the velocity direction are passed split into their parts transverse
// to the radial direction e_x' and their radial components: a beam's transverse part is then
// a sum of small, accurately computed terms, and its angle to e_x' keeps its relative
// precision even for a distant camera, whose beams are all nearly radial.
struct ViewDev {
  float rhat[3], sq1mu;   // e_x' = radial unit vector at the camera, sqrt(1 - u_c)
  float ew[3], f;         // camera axes' parts transverse to e_x' (world), focal length in pixels
  float eh[3], u_c;
  float ed[3], gamma;
  float vhat[3], vmag;    // velocity direction's part transverse to e_x', speed (static frame)
  float half_w, half_h, u_ic, u_oc;
  float inv_sq1mu, T0, T_exp, rho;
  float k_disc, k_star, T_norm, march_h;   // march_h: ray-marching step (marching only)
  int width, height, T_law, has_stars;
  StarsDev stars;
  float4* out;
  float4* aov;
  // animated disc: density_mode 1 = particles at the crossings' retarded times
  float time;             // camera coordinate time
  int density_mode, nparts, march_steps;   // march_steps: step budget (marching only)
  const float4* parts;    // 2 float4 per particle (see disc_density)
  const int* pstart;      // first particle reaching radius bin floor(r * pscale), pbins + 1
  float pscale;
  int pbins;
  // radial components of e_w, e_h, e_d and of the velocity direction.  Last in the record:
  // inserted before the star-map fields it shifted their offsets and the render measured
  // 2.6% slower at 1920x1080.
  float er[4];
  AreaDev area;
};

// the features a view uses
__host__ __device__ inline int view_features(const ViewDev& v) {
  return (v.density_mode != 0 ? kFeatParticles : 0) | (v.area.tex ? kFeatArea : 0) |
         ((v.area.tex && v.area.bands) || (v.has_stars && v.stars.bands) ? kFeatBands : 0);
}

// Bloom launch record: the image's box pyramid, levels 0 (the image) .. levels <= 16, and
// the weights w_0 .. w_levels of the mipmap filters (Section 3.4.3)
constexpr int kBloomMaxLevels = 16;
struct BloomDev {
  int w[kBloomMaxLevels + 1], h[kBloomMaxLevels + 1];  // level sizes
  int64_t off[kBloomMaxLevels + 1];  // float4 offset of level k in the pyramid arrays (k >= 1)
  float wt[kBloomMaxLevels + 1];
  int levels, tiles_x, tiles_y, pad;  // tiles: 64 x 64 image pixels each
};

// Work of the batched kernels, as runs of consecutive tiles of one view: the view's tiles
// tile0 .. tile0 + n - 1 (row-major tile order, tiles_x tiles per row) take the launch's
// flat tile indices start .. start + n - 1.  A launch lists its runs in increasing start,
// the first at 0.
struct TileRun {
  int view, tile0, start, tiles_x;
};

__device__ __forceinline__ float clampf(float x, float lo, float hi) {
  return fminf(fmaxf(x, lo), hi);
}

// Streaming stores of results the kernel never reads back (images): marked non-temporal, so
// they do not evict the tables and star-map lines the other waves still read from L2.
__device__ __forceinline__ void store_stream(float4* p, float4 v) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  const f4v x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, reinterpret_cast<f4v*>(p));
}
__device__ __forceinline__ void store_stream(uint32_t* p, uint32_t v) {
  __builtin_nontemporal_store(v, p);
}

// ---- short math for the render path ----------------------------------------------------
// Hardware square root and reciprocal (about 1 ulp each), for values whose rounding is not
// amplified afterwards.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// log(1 + x), x > -1: with u = fl(1 + x), log(u) * x / (u - 1) cancels the rounding of u.
__device__ __forceinline__ float flog1p(float x) {
  float u = 1.0f + x;
  float d = u - 1.0f;
  if (d == 0.0f) return x;
  return __builtin_amdgcn_logf(u) * 0.693147180559945309f * fdiv(x, d);
}

// sin on |x| <= pi/6: Taylor series through x^11 (remainder below 2e-11).
__device__ __forceinline__ float fsin_small(float x) {
  float s = x * x;
  return x * (1.0f + s * (-1.0f / 6.0f + s * (1.0f / 120.0f + s * (-1.0f / 5040.0f +
              s * (1.0f / 362880.0f + s * (-1.0f / 39916800.0f))))));
}

// atan2(y, x) for y >= 0 (the render path's angles lie in [0, pi]): t = min/max of |x|, |y|
// in [0, 1], atan(t) = t P(t^2) with a degree-8 P fitted by weighted least squares at
// Chebyshev nodes (max error 1.2e-7 rad in FP32), then the octant.
__device__ __forceinline__ float fatan2_pos(float y, float x) {
  float ax = fabsf(x), ay = fabsf(y);
  float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  float t = mx > 0.0f ? fdiv(mn, mx) : 0.0f;
  float s = t * t;
  float p = 0.0024567029904574156f;
  p = fmaf(p, s, -0.014401259832084179f);
  p = fmaf(p, s, 0.03978103771805763f);
  p = fmaf(p, s, -0.07234838604927063f);
  p = fmaf(p, s, 0.10498934984207153f);
  p = fmaf(p, s, -0.141612246632576f);
  p = fmaf(p, s, 0.19985905289649963f);
  p = fmaf(p, s, -0.33332598209381104f);
  p = fmaf(p, s, 0.9999998807907104f);
  float r = p * t;
  if (ay > ax) r = 1.57079632679489662f - r;
  if (x < 0.0f) r = 3.14159265358979324f - r;
  return r;
}

// bilinear fetch of a row-major table with texel k of n at unit coordinate k/(n-1),
// columns clamped to [lo, hi] (so the two halves of D are never mixed)
// Coordinates are clamped to just below the last texel (k (1 - 2^-23) < k for every k >= 1),
// so the lower texel is trunc(t), the next one exists, and the weight is fract(t); at the
// edge itself the result differs from the edge texel by 2^-23 of the last texel step.
constexpr float kBelowOne = 0.99999988f;  // 1 - 2^-23

__device__ __forceinline__ float bilinear(const float* __restrict__ t, int nx, int ny, int lo,
                                          int hi, float x, float y) {
  float tx = clampf(x * (float)(nx - 1), (float)lo, (float)hi * kBelowOne);
  float ty = clampf(y * (float)(ny - 1), 0.0f, (float)(ny - 1) * kBelowOne);
  int i0 = (int)tx, j0 = (int)ty;
  float fx = __builtin_amdgcn_fractf(tx), fy = __builtin_amdgcn_fractf(ty);
  const float* r0 = t + (__umul24((unsigned)j0, (unsigned)nx) + (unsigned)i0);  // nx, ny < 2^24
  const float* r1 = r0 + nx;
  float a = r0[0] + fx * (r0[1] - r0[0]);
  float b = r1[0] + fx * (r1[1] - r1[0]);
  return a + fy * (b - a);
}

// apsis of a ray with e^2 < mu (Section 3.3.1, eq. uapsis)
__device__ __forceinline__ float apsis_f(float e2) {
  float a = clampf(e2 * (2.0f / kMu) - 1.0f, -1.0f, 1.0f);
  return 1.0f / 3.0f + 2.0f / 3.0f * fsin_small(asinf(a) * (1.0f / 3.0f));
}

// D(e, u) through the Appendix A mapping, read from `tab` (T.D, or the time channel T.Dt,
// which shares its layout).  udot = du/dphi at (e, u) on the ray.  For
// e^2 < mu the row coordinate y = 1 - sqrt(1 - u/u_a) is evaluated as
// 1 - sqrt(udot^2 / (e^2 + u u_a (1 - u_a - u))): the two are equal because
// udot^2 = (u_a - u)(u_2 - u)(u - u_3) with u_2 + u_3 = 1 - u_a and u_2 u_3 = -e^2 / u_a,
// and the second form has no cancellation when the camera sits near the apsis.
__device__ __forceinline__ float lookup_D(const TablesDev& T, const float* tab, float e2,
                                          float u, float ua, float udot) {
  const int n = T.d_n;
  if (e2 < kMu) {
    float x = 0.5f - fsqrt(-flog1p(-e2 * (1.0f / kMu)) * (1.0f / 50.0f));
    float den = e2 + u * ua * (1.0f - ua - u);
    float s2 = den > 0.0f ? fminf(fdiv(udot * udot, den), 1.0f) : 0.0f;
    float y = 1.0f - fsqrt(s2);
    return bilinear(tab, n, n, 0, n / 2 - 1, x, y);
  }
  float x = 0.5f + fsqrt(-flog1p(-kMu / e2) * (1.0f / 50.0f));
  float dz = u - 2.0f / 3.0f;
  const float s23 = 0.816496580927726f, s13 = 0.577350269189626f;
  float y = (s23 + copysignf(fsqrt(fabsf(dz)), dz)) * (1.0f / (s23 + s13));
  return bilinear(tab, n, n, n / 2, n - 1, x, y);
}

// D(e, u_a) for e^2 < mu: the apsis is the last row (y = 1) of the left half
__device__ __forceinline__ float lookup_D_apsis(const TablesDev& T, const float* tab, float e2) {
  const int n = T.d_n, hi = n / 2 - 1;
  float x = 0.5f - fsqrt(-flog1p(-e2 * (1.0f / kMu)) * (1.0f / 50.0f));
  float tx = clampf(x * (float)(n - 1), 0.0f, (float)hi * kBelowOne);
  int i0 = (int)tx;
  float fx = __builtin_amdgcn_fractf(tx);
  const float* r = tab + (__umul24((unsigned)(n - 1), (unsigned)n) + (unsigned)i0);
  return r[0] + fx * (r[1] - r[0]);
}

// U(e, phi) through the Appendix A mapping, read from `tab` (T.U or the time channel T.Ut)
__device__ __forceinline__ float lookup_U(const TablesDev& T, const float* tab, float e2, float e,
                                          float phi) {
  float x = fdiv(1.0f, 1.0f + 6.0f * e2);
  // (1 + 6 e^3) / (1 + e^2) written so that it cannot overflow for nearly radial rays
  float y = phi * (1.0f / 3.0f) * (6.0f * e + fdiv(1.0f - 6.0f * e, 1.0f + e2));
  return bilinear(tab, T.u_ne, T.u_nphi, 0, T.u_ne - 1, x, y);
}

// band radiances (R, G, B, sum) at temperature T from the log-log band table
__device__ __forceinline__ float4 band_lookup(const LutDev& L, float T) {
  if (!(T > 0.0f)) return make_float4(0.f, 0.f, 0.f, 0.f);
  float x = (__log2f(T) - L.x0) * L.inv_dx;
  if (x < 0.0f) return make_float4(0.f, 0.f, 0.f, 0.f);
  x = fminf(x, (float)L.n + 1024.0f);  // keeps the index conversion defined for T = inf
  int k = min((int)x, L.n - 2);
  float fr = x - (float)k;  // > 1 above the table: linear extrapolation in log-log
  float4 a = L.lut[k], b = L.lut[k + 1];
  // hardware 2^x (about 1 ulp; results below 2^-126 flush to zero)
  return make_float4(__builtin_amdgcn_exp2f(a.x + fr * (b.x - a.x)),
                     __builtin_amdgcn_exp2f(a.y + fr * (b.y - a.y)),
                     __builtin_amdgcn_exp2f(a.z + fr * (b.z - a.z)),
                     __builtin_amdgcn_exp2f(a.w + fr * (b.w - a.w)));
}

}  // namespace bh
