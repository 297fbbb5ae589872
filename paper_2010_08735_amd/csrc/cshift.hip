// Colour-shift table for light of any colour (Section 3.4.2), built on the device in FP64.
//
// Received spectral radiance is D^5 I(D lambda) for emitted I and frequency ratio D.  Each
// band chromaticity (r, g) (bands R 600-700 nm, G 500-600, B 400-500, b = 1 - r - g) stands
// for one spectrum I = B_T (1 - a1 A1 - a2 A2): B_T the blackbody whose blue-to-red band
// ratio is b / r (bisection on log T over [1e3, 1e6] K, clamped at the ends), A1 and A2
// Gaussian absorption bands at 450 and 650 nm of width 30 nm, and a1, a2 in [-8, 1] the
// solution of the two linear conditions R(I) = r S(I), G(I) = g S(I).  Node (i, j, k) holds
// log2 of C_b = D^5 int_b I(D lambda) / int_{400}^{700} I, at r = i / 127, g = j / 127
// (projected onto r + g <= 1), log2 D = -3 + 6 k / 127, each C_b raised to 2^-100 first;
// layout ((i 128 + j) 128 + k), float4 (log2 C_R, log2 C_G, log2 C_B, 0).
// Band integrals: 32 equal panels of 8-point Gauss-Legendre per band (the spectrum may
// change sign, so no relative-tolerance adaptivity); the Planck factor varies by at most
// ~2 e-folds per panel down to D T = 125 K, where the rule is exact to rounding.
#include "bh_dev.h"

namespace bh {

namespace {

constexpr double kHc = 6.62607015e-34 * 299792458.0;   // h c
constexpr double kHc2 = 6.62607015e-34 * 299792458.0 * 299792458.0;
constexpr double kKb = 1.380649e-23;
constexpr double kAbsMu0 = 450e-9, kAbsMu1 = 650e-9, kAbsSigma = 30e-9;
constexpr double kCctLo = 1000.0, kCctHi = 1.0e6;
constexpr int kPanels = 32;
// band edges, R then G then B
__constant__ double kBandLo[3] = {600e-9, 500e-9, 400e-9};

__device__ double planck_d(double lam, double T) {
  const double x = kHc / (lam * kKb * T);
  if (x > 700.0) return 0.0;
  const double l2 = lam * lam;
  return 2.0 * kHc2 / (l2 * l2 * lam) / expm1(x);
}

__device__ double gauss_abs(double lam, double mu) {
  const double z = (lam - mu) * (1.0 / kAbsSigma);
  return exp(-0.5 * z * z);
}

// integral of f over band b (100 nm) by the composite rule
template <typename F>
__device__ double band_integral(const CshiftRule& q, int b, F f) {
  const double h = 100e-9 / kPanels;
  double s = 0.0;
  for (int p = 0; p < kPanels; ++p) {
    const double mid = kBandLo[b] + (p + 0.5) * h;
    double ps = 0.0;
#pragma unroll
    for (int n = 0; n < 8; ++n) ps += q.w[n] * f(mid + 0.5 * h * q.x[n]);
    s += 0.5 * h * ps;
  }
  return s;
}

__device__ double blue_over_red(const CshiftRule& q, double T) {
  const auto bb = [T](double l) { return planck_d(l, T); };
  return band_integral(q, 2, bb) / band_integral(q, 0, bb);
}

}  // namespace

// one thread per chromaticity node: (T, a1, a2, band sum of the spectrum)
__global__ void k_cshift_spectra(CshiftRule q, double4* __restrict__ spec) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kCshiftN * kCshiftN) return;
  double r = (double)(t / kCshiftN) / (kCshiftN - 1), g = (double)(t % kCshiftN) / (kCshiftN - 1);
  if (r + g > 1.0) {
    const double s = r + g;
    r /= s;
    g /= s;
  }
  const double b = fmax(1.0 - r - g, 0.0);
  double T;
  if (b <= blue_over_red(q, kCctLo) * r) {
    T = kCctLo;
  } else if (b >= blue_over_red(q, kCctHi) * r) {
    T = kCctHi;
  } else {
    double lo = log(kCctLo), hi = log(kCctHi);
    for (int it = 0; it < 64; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (blue_over_red(q, exp(mid)) * r < b)
        lo = mid;
      else
        hi = mid;
    }
    T = exp(0.5 * (lo + hi));
  }
  double P[3], Q1[3], Q2[3];
  for (int k = 0; k < 3; ++k) {
    P[k] = band_integral(q, k, [T](double l) { return planck_d(l, T); });
    Q1[k] = band_integral(q, k, [T](double l) { return planck_d(l, T) * gauss_abs(l, kAbsMu0); });
    Q2[k] = band_integral(q, k, [T](double l) { return planck_d(l, T) * gauss_abs(l, kAbsMu1); });
  }
  const double sP = P[0] + P[1] + P[2], s1 = Q1[0] + Q1[1] + Q1[2], s2 = Q2[0] + Q2[1] + Q2[2];
  // a1 (r s1 - Q1_R) + a2 (r s2 - Q2_R) = r sP - P_R; the same with g and the G band
  const double m00 = r * s1 - Q1[0], m01 = r * s2 - Q2[0], y0 = r * sP - P[0];
  const double m10 = g * s1 - Q1[1], m11 = g * s2 - Q2[1], y1 = g * sP - P[1];
  const double det = m00 * m11 - m01 * m10, scale = fabs(m00 * m11) + fabs(m01 * m10);
  double a1 = 0.0, a2 = 0.0;
  if (scale > 0.0 && fabs(det) > 1e-12 * scale) {
    a1 = fmin(fmax((y0 * m11 - m01 * y1) / det, -8.0), 1.0);
    a2 = fmin(fmax((m00 * y1 - y0 * m10) / det, -8.0), 1.0);
  }
  spec[t] = make_double4(T, a1, a2, sP - a1 * s1 - a2 * s2);
}

// one thread per node (i, j, k): log2 of the shifted band radiances per unit emitted sum
__global__ void k_cshift_table(CshiftRule q, const double4* __restrict__ spec,
                               float4* __restrict__ tab) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kCshiftN * kCshiftN * kCshiftN) return;
  const double4 s = spec[t / kCshiftN];
  const int k = t % kCshiftN;
  const double D = exp2(-3.0 + 6.0 * k / (kCshiftN - 1));
  const double D5 = D * D * D * D * D;
  const double T = s.x, a1 = s.y, a2 = s.z, den = s.w;
  const auto shifted = [=](double l) {
    const double lp = D * l;
    return D5 * planck_d(lp, T) * (1.0 - a1 * gauss_abs(lp, kAbsMu0) - a2 * gauss_abs(lp, kAbsMu1));
  };
  float out[3];
  for (int b = 0; b < 3; ++b) {
    double v = den > 0.0 ? band_integral(q, b, shifted) / den : 0.0;
    v = fmax(v, 0x1p-100);
    out[b] = (float)log2(v);
  }
  tab[t] = make_float4(out[0], out[1], out[2], 0.0f);
}

hipError_t launch_cshift_build(const CshiftRule& q, double4* spec, float4* tab, hipStream_t s) {
  const int nc = kCshiftN * kCshiftN, nt = kCshiftN * kCshiftN * kCshiftN;
  hipLaunchKernelGGL(k_cshift_spectra, dim3((nc + 63) / 64), dim3(64), 0, s, q, spec);
  hipLaunchKernelGGL(k_cshift_table, dim3((nt + 255) / 256), dim3(256), 0, s, q,
                     (const double4*)spec, tab);
  return hipGetLastError();
}

}  // namespace bh
