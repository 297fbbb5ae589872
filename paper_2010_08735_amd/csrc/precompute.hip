// Table precompute on the GPU: integrate the photon orbit equation u'' = 3/2 u^2 - u
// (Section 3.3, eq. rayequation) for rays coming from infinity (u = 0, du/dphi = e) and
// record, at the Appendix A texel centres k/(N-1):
//   D(e, u)   = phi - atan2(u, du/dphi) on the incoming branch   (Algorithm 1, Precompute)
//   U(e, phi) = u for 0 <= phi < pi, 1 once the ray has fallen in (Section 3.3.3).
// One thread integrates one e column with classic RK4 in phi.  Precision: FP64 while
// |u - 2/3| < band (near the photon sphere, where the deflection diverges and errors grow
// exponentially with each turn), FP32 elsewhere with Kahan-compensated state updates.
// Values between steps come from cubic Hermite interpolation (u and du/dphi are both
// known at every step), in the variable that is smooth for each table half:
//   - D, e^2 < mu: in y = 1 - s with s = (du/dphi) / sqrt(u_a (u_2 - u)(u - u_3)), the
//     Appendix A row coordinate, which passes smoothly through the apsis (y = 1);
//   - D, e^2 > mu: u is monotone, so phi(u_j) is found by inverting the Hermite cubic;
//   - U: directly in phi.
// Time channels (Algorithm 1 Precompute also stores t, dt/dphi = e / (u^2 - u^3)): the
// time since infinity diverges, so the tables hold e tau with the regularised time
// tau = t - ln(u/(1-u)) + 1/u (+ const), whose rate is dtau/dphi = 1 / (e + du/dphi) on both
// branches (e - du/dphi = u^2 (1 - u) / (e + du/dphi) on a ray with invariant e^2).  tau is
// integrated with the same RK4 stages and read out with the same Hermite interpolation.
#include "bh_dev.h"

namespace bh {

enum { kTabFP32 = 0, kTabBand = 1, kTabAll = 2 };

__device__ __forceinline__ double accel64(double u) { return 1.5 * u * u - u; }
__device__ __forceinline__ float accel32(float u) { return 1.5f * u * u - u; }

__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  float y = x - c;
  float t = s + y;
  c = (t - s) - y;
  s = t;
}

// State of one column integration, switching between FP64 and compensated FP32.
struct Integrator {
  double e2;            // the column's conserved (du/dphi)^2 + u^2 (1 - u)
  double e;             // its square root
  double u, w, tau;     // FP64 state (valid when in64)
  float uf, wf, cu, cw; // FP32 state, true value = uf - cu (Kahan)
  float tf, ct;         // FP32 regularised time, true value = tf - ct
  bool in64;
  int mode;
  double band;

  __device__ bool want64(double uu) const {
    return mode == kTabAll || (mode == kTabBand && fabs(uu - 2.0 / 3.0) < band);
  }
  __device__ void init(double u0, double w0) {
    u = u0;
    w = w0;
    tau = 0.0;
    uf = (float)u0;
    wf = (float)w0;
    cu = (float)((double)uf - u0);
    cw = (float)((double)wf - w0);
    tf = 0.0f;
    ct = 0.0f;
    in64 = want64(u0);
  }
  __device__ double get_u() const { return in64 ? u : (double)uf - (double)cu; }
  __device__ double get_w() const { return in64 ? w : (double)wf - (double)cw; }
  __device__ double get_tau() const { return in64 ? tau : (double)tf - (double)ct; }
  __device__ void step(double h) {
    double uc = get_u();
    bool w64 = want64(uc);
    if (w64 != in64) {
      if (w64) {
        // entering the FP64 band: keep u and re-derive |du/dphi| from the exact invariant,
        // so FP32 rounding of e^2 is not amplified by the unstable orbit near u = 2/3
        u = uc;
        double wc = get_w();
        tau = get_tau();
        double w2 = e2 - uc * uc * (1.0 - uc);
        w = w2 > 0.0 ? copysign(sqrt(w2), wc) : 0.0;
      } else {
        uf = (float)u;
        cu = (float)((double)uf - u);
        wf = (float)w;
        cw = (float)((double)wf - w);
        tf = (float)tau;
        ct = (float)((double)tf - tau);
      }
      in64 = w64;
    }
    if (in64) {
      double k1u = w, k1w = accel64(u);
      double k2u = w + 0.5 * h * k1w, k2w = accel64(u + 0.5 * h * k1u);
      double k3u = w + 0.5 * h * k2w, k3w = accel64(u + 0.5 * h * k2u);
      double k4u = w + h * k3w, k4w = accel64(u + h * k3u);
      tau += h / 6.0 * (1.0 / (e + k1u) + 2.0 / (e + k2u) + 2.0 / (e + k3u) + 1.0 / (e + k4u));
      u += h / 6.0 * (k1u + 2.0 * k2u + 2.0 * k3u + k4u);
      w += h / 6.0 * (k1w + 2.0 * k2w + 2.0 * k3w + k4w);
    } else {
      float hf = (float)h;
      float k1u = wf, k1w = accel32(uf);
      float k2u = wf + 0.5f * hf * k1w, k2w = accel32(uf + 0.5f * hf * k1u);
      float k3u = wf + 0.5f * hf * k2w, k3w = accel32(uf + 0.5f * hf * k2u);
      float k4u = wf + hf * k3w, k4w = accel32(uf + hf * k3u);
      float ef = (float)e;
      kahan_add(tf, ct, hf / 6.0f * (1.0f / (ef + k1u) + 2.0f / (ef + k2u) + 2.0f / (ef + k3u) +
                                     1.0f / (ef + k4u)));
      kahan_add(uf, cu, hf / 6.0f * (k1u + 2.0f * k2u + 2.0f * k3u + k4u));
      kahan_add(wf, cw, hf / 6.0f * (k1w + 2.0f * k2w + 2.0f * k3w + k4w));
    }
  }
};

__device__ __forceinline__ double hermite(double t, double f0, double d0, double f1, double d1,
                                          double hh) {
  double t2 = t * t, t3 = t2 * t;
  return (2 * t3 - 3 * t2 + 1) * f0 + (t3 - 2 * t2 + t) * hh * d0 + (-2 * t3 + 3 * t2) * f1 +
         (t3 - t2) * hh * d1;
}
__device__ __forceinline__ double hermite_dt(double t, double f0, double d0, double f1,
                                             double d1, double hh) {
  double t2 = t * t;
  return (6 * t2 - 6 * t) * f0 + (3 * t2 - 4 * t + 1) * hh * d0 + (-6 * t2 + 6 * t) * f1 +
         (3 * t2 - 2 * t) * hh * d1;
}

__device__ double d_col_e2(int n, int i) {
  double x = (double)i / (n - 1);
  if (i < n / 2) {
    double a = 0.5 - x;
    return -kMuD * expm1(-50.0 * a * a);
  }
  double a = x - 0.5;
  return kMuD / (-expm1(-50.0 * a * a));
}

constexpr int kMaxSteps = 4000000;

__global__ void __launch_bounds__(64) k_precompute_D(float* __restrict__ D,
                                                     float* __restrict__ Dt, int n, int mode,
                                                     double band, double step) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double e2 = d_col_e2(n, i);
  const double e = sqrt(e2);
  const double h = step / (1.0 + e);
  Integrator I;
  I.mode = mode;
  I.band = band;
  I.e2 = e2;
  I.e = e;
  I.init(0.0, e);
  D[i] = 0.0f;  // u = 0 at phi = 0: D = 0 - atan2(0, e)
  Dt[i] = 0.0f;
  int j = 1;
  if (i < n / 2) {
    // roots u_a < u_2 of u^3 - u^2 + e^2 (u_3 < 0): closed form and sum/product of roots
    double ua = 1.0 / 3.0 + 2.0 / 3.0 * sin(asin(fmin(2.0 * e2 / kMuD - 1.0, 1.0)) / 3.0);
    double ssum = 1.0 - ua, prod = -e2 / ua;
    double disc = sqrt(ssum * ssum - 4.0 * prod);
    double u2 = 0.5 * (ssum + disc), u3 = 0.5 * (ssum - disc);
    double yp = 0.0, fp = 0.0, dp, tp = 0.0, dtp;
    {
      // derivatives at the start (u = 0, w = e): s = w / g, g(0) = e
      double g = e, gp = ua * (u2 + u3) / (2.0 * g);
      double dsdphi = (0.0 * g - e * e * gp) / (g * g);  // accel(0) = 0
      double dDdphi = 1.0 - (e * e) / (e * e);            // = 0 at u = 0
      dp = dDdphi / (-dsdphi);
      dtp = (0.5 / e) / (-dsdphi);                         // dtau/dphi = 1 / (2e) at u = 0
    }
    for (int k = 1; k < kMaxSteps && j < n; ++k) {
      I.step(h);
      double u = I.get_u(), w = I.get_w(), phi = k * h;
      double g2 = ua * (u2 - u) * (u - u3);
      double g = sqrt(fmax(g2, 1e-300));
      double y = 1.0 - w / g;
      double acc = accel64(u);
      double gp = ua * (u2 + u3 - 2.0 * u) / (2.0 * g);
      double dydphi = -(acc * g - w * w * gp) / g2;
      double f = phi - atan2(u, w);
      double dfdphi = 1.0 - (w * w - u * acc) / (u * u + w * w);
      double d = dfdphi / dydphi;
      double tv = I.get_tau(), dtv = (1.0 / (e + w)) / dydphi;
      while (j < n) {
        double yj = (double)j / (n - 1);
        if (yj > y) break;
        double hh = y - yp;
        double t = hh > 0.0 ? (yj - yp) / hh : 1.0;
        D[(size_t)j * n + i] = (float)hermite(t, fp, dp, f, d, hh);
        Dt[(size_t)j * n + i] = (float)(e * hermite(t, tp, dtp, tv, dtv, hh));
        ++j;
      }
      yp = y;
      fp = f;
      dp = d;
      tp = tv;
      dtp = dtv;
    }
    for (; j < n; ++j) {  // not reached in practice
      D[(size_t)j * n + i] = (float)fp;
      Dt[(size_t)j * n + i] = (float)(e * tp);
    }
  } else {
    const double a = sqrt(2.0 / 3.0), b = sqrt(1.0 / 3.0);
    double phip = 0.0, up = 0.0, wp = e, taup = 0.0;
    for (int k = 1; k < kMaxSteps && j < n; ++k) {
      I.step(h);
      double u = I.get_u(), w = I.get_w(), phi = k * h, tau = I.get_tau();
      while (j < n) {
        double z = (double)j / (n - 1) * (a + b) - a;
        double uj = 2.0 / 3.0 + (z >= 0 ? z * z : -z * z);
        if (j == n - 1) uj = 1.0;
        if (uj > u) break;
        double hh = phi - phip;
        double t = (u > up) ? (uj - up) / (u - up) : 1.0;
        for (int it = 0; it < 8; ++it) {
          double r = hermite(t, up, wp, u, w, hh) - uj;
          double dr = hermite_dt(t, up, wp, u, w, hh);
          if (dr > 0.0) t -= r / dr;
          t = fmin(fmax(t, 0.0), 1.0);
        }
        double ph = phip + t * hh;
        double wj = sqrt(fmax(e2 - uj * uj * (1.0 - uj), 0.0));
        D[(size_t)j * n + i] = (float)(ph - atan2(uj, wj));
        Dt[(size_t)j * n + i] =
            (float)(e * hermite(t, taup, 1.0 / (e + wp), tau, 1.0 / (e + w), hh));
        ++j;
      }
      phip = phi;
      up = u;
      wp = w;
      taup = tau;
    }
  }
}

__global__ void __launch_bounds__(64) k_precompute_U(float* __restrict__ U,
                                                     float* __restrict__ Ut, int ne, int nphi,
                                                     int mode, double band, double step) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  if (i == 0) {  // e -> infinity: u = e phi along phi = y / (2e), i.e. u = y / 2; e tau -> 0
    for (int j = 0; j < nphi; ++j) {
      U[(size_t)j * ne] = 0.5f * (float)j / (float)(nphi - 1);
      Ut[(size_t)j * ne] = 0.0f;
    }
    return;
  }
  if (i == ne - 1) {
    // e = 0: the ray stays at infinity (u = 0) along phi = 3y; e tau tends to tan(phi/2)
    // on a straight ray before its closest point (phi = pi/2), 2/sin(phi) - cot(phi/2) after
    for (int j = 0; j < nphi; ++j) {
      double phi = 3.0 * (double)j / (nphi - 1);
      U[(size_t)j * ne + i] = 0.0f;
      Ut[(size_t)j * ne + i] =
          (float)(phi <= 0.5 * M_PI ? tan(0.5 * phi) : 2.0 / sin(phi) - 1.0 / tan(0.5 * phi));
    }
    return;
  }
  double x = (double)i / (ne - 1);
  double e2 = (1.0 / x - 1.0) / 6.0;
  double e = sqrt(e2);
  double scale = 3.0 * (1.0 + e2) / (1.0 + 6.0 * e2 * e);  // phi_j = scale * y_j
  double h = step / (1.0 + e);
  Integrator I;
  I.mode = mode;
  I.band = band;
  I.e2 = e2;
  I.e = e;
  I.init(0.0, e);
  U[i] = 0.0f;
  Ut[i] = 0.0f;
  int j = 1;
  double phip = 0.0, up = 0.0, wp = e, taup = 0.0;
  bool fallen = false;
  for (int k = 1; k < kMaxSteps && j < nphi; ++k) {
    I.step(h);
    double u = I.get_u(), w = I.get_w(), phi = k * h, tau = I.get_tau();
    while (j < nphi) {
      double phij = scale * (double)j / (nphi - 1);
      if (phij > phi) break;
      double hh = phi - phip;
      double t = (phij - phip) / hh;
      double v = hermite(t, up, wp, u, w, hh);
      U[(size_t)j * ne + i] = (float)fmin(fmax(v, 0.0), 1.0);
      Ut[(size_t)j * ne + i] =
          (float)(e * hermite(t, taup, 1.0 / (e + wp), tau, 1.0 / (e + w), hh));
      ++j;
    }
    if (u >= 1.0) {
      fallen = true;
      break;
    }
    phip = phi;
    up = u;
    wp = w;
    taup = tau;
  }
  if (fallen)
    for (; j < nphi; ++j) {
      U[(size_t)j * ne + i] = 1.0f;
      Ut[(size_t)j * ne + i] = 0.0f;
    }
}

hipError_t launch_precompute(float* D, float* Dt, int d_n, float* U, float* Ut, int u_ne,
                             int u_nphi, int mode, double band, double step, hipStream_t s) {
  hipLaunchKernelGGL(k_precompute_D, dim3((d_n + 63) / 64), dim3(64), 0, s, D, Dt, d_n, mode,
                     band, step);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_precompute_U, dim3((u_ne + 63) / 64), dim3(64), 0, s, U, Ut, u_ne,
                     u_nphi, mode, band, step);
  return hipGetLastError();
}

}  // namespace bh
