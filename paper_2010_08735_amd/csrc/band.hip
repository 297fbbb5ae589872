// Blackbody band table.  Disc emission is a blackbody at T(u) (Section 3.3.3) and, for
// blackbodies, Doppler shift plus beaming reduce to the temperature shift T -> (nu/nu') T
// (Section 3.4.2), so a received colour is the band radiance of a blackbody at D T.
// Colour model: Planck spectral radiance integrated over the box bands R = 600-700 nm,
// G = 500-600 nm, B = 400-500 nm (W m^-2 sr^-1), stored as log2 on a log2 T grid and
// interpolated linearly in log-log space by band_lookup().  Built once per context in
// FP64 by composite Simpson quadrature (1024 panels per band).
#include "bh_dev.h"

namespace bh {

__device__ double planck64(double lambda, double T) {
  const double h = 6.62607015e-34, c = 299792458.0, k = 1.380649e-23;
  double x = h * c / (lambda * k * T);
  if (x > 700.0) return 0.0;
  double l2 = lambda * lambda;
  return 2.0 * h * c * c / (l2 * l2 * lambda) / expm1(x);
}

__device__ double band_simpson(double lo, double hi, double T) {
  const int n = 1024;
  double hstep = (hi - lo) / n;
  double s = planck64(lo, T) + planck64(hi, T);
  for (int i = 1; i < n; ++i) s += (i & 1 ? 4.0 : 2.0) * planck64(lo + i * hstep, T);
  return s * hstep / 3.0;
}

__global__ void k_band_lut(float4* __restrict__ lut, int n, float x0, float dx) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double T = exp2((double)x0 + k * (double)dx);
  double r = band_simpson(600e-9, 700e-9, T);
  double g = band_simpson(500e-9, 600e-9, T);
  double b = band_simpson(400e-9, 500e-9, T);
  const double tiny = 1e-300;
  lut[k] = make_float4((float)log2(fmax(r, tiny)), (float)log2(fmax(g, tiny)),
                       (float)log2(fmax(b, tiny)), (float)log2(fmax(r + g + b, tiny)));
}

__global__ void k_band_eval(LutDev L, const float* __restrict__ temps, int64_t n,
                            float* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float4 v = band_lookup(L, temps[i]);
  out[3 * i] = v.x;
  out[3 * i + 1] = v.y;
  out[3 * i + 2] = v.z;
}

hipError_t launch_band_lut(float4* lut, int n, float x0, float dx, hipStream_t s) {
  hipLaunchKernelGGL(k_band_lut, dim3((n + 63) / 64), dim3(64), 0, s, lut, n, x0, dx);
  return hipGetLastError();
}

hipError_t launch_band_eval(const LutDev& L, const float* temps, int64_t n, float* out,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L, temps,
                     n, out);
  return hipGetLastError();
}

}  // namespace bh
