/*
 * Light of any colour under the Doppler and beaming effects (Section 3.4.2): the colour-shift
 * table C(xy, D).  TEST INFRASTRUCTURE ONLY (bh_oracle.h).
 *
 * Received spectral radiance is D^5 I(D lambda) for emitted I and frequency ratio
 * D = nu / nu' (I / nu^3 is invariant; per unit wavelength this is the fifth power).  For a
 * blackbody that is the blackbody at D T.  For any other colour the paper picks one
 * spectrum per chromaticity, a blackbody at the correlated colour temperature T times
 * (1 - a1 A1 - a2 A2) with two fixed absorption spectra, solves a1, a2 from the
 * chromaticity (a linear system), and tabulates the received colour per unit emitted
 * colour sum over chromaticity and D.
 *
 * Readings (the paper prints neither the absorption spectra nor colour-matching data):
 *  - colour is the band model of emission.c (R 600-700 nm, G 500-600, B 400-500 nm);
 *    a chromaticity is (r, g) = (R, G) / S, S = R + G + B, b = 1 - r - g;
 *  - A1, A2 are Gaussian absorption bands exp(-(lambda - mu)^2 / (2 s^2)), mu = 450 nm
 *    (blue) and 650 nm (red), s = 30 nm, defined at every wavelength;
 *  - the correlated temperature is that of the blackbody with the same blue-to-red band
 *    ratio b / r (increasing in T, towards 4.45 in the Rayleigh-Jeans limit), by bisection
 *    on log T over [1000 K, 10^6 K]; T = 1000 K when b <= rho(1000) r, else T = 10^6 K
 *    when b >= rho(10^6) r;
 *  - a1, a2 make the band chromaticity of the spectrum (r, g): R(I) - r S(I) = 0 and
 *    G(I) - g S(I) = 0, linear in a1, a2 (Cramer's rule; a1 = a2 = 0 if singular), then
 *    each is clamped to [-8, 1]: at most full absorption, so the spectrum stays
 *    non-negative (A1 + A2 <= 1 + 2e-10), and at most a ninefold boost; a chromaticity
 *    that needs more (far from the blackbody locus) gets the clamped spectrum's colour;
 *  - a chromaticity off the triangle is projected onto it: negative parts to 0, then
 *    (r, g) / (r + g) if r + g > 1;
 *  - C_b(r, g, D) = D^5 int_b I(D lambda) d lambda / int_{400 nm}^{700 nm} I(lambda)
 *    d lambda, set to 0 where negative; the received colour of emitted (R, G, B) is S C.
 * For a blackbody chromaticity a1 = a2 = 0 and C_b = L_b(D T) / sum L(T): the band
 * model's temperature shift.
 *
 * Table: log2 C_b at nodes r_i = i / (nr - 1), g_j = j / (ng - 1), log2 D_k = -3 + 6 k /
 * (nd - 1) (128^3 nodes in use), each C_b first raised to at least 2^-100; layout
 * ((i ng + j) nd + k) * 3.  A lookup interpolates the log2 values trilinearly, linearly in
 * r and g and, between the two D nodes around D, linearly in 1 / D (the Wien factor
 * exp(-h c / (lambda k D T)) is then followed exactly); r, g and log2 D are clamped to
 * the node range first; it returns 2^value.
 * Parity: pinned by the chromaticity a spectrum reproduces at D = 1, by the blackbody
 * limit against emission.c's band integrals, by the correlated temperature of blackbody
 * colours, and by the table's nodes.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>

#include "bh_oracle.h"
#include "oracle_internal.h"

static const double MU_ABS[2] = {450e-9, 650e-9};
static const double S_ABS = 30e-9;
static const double T_LO = 1000.0, T_HI = 1.0e6;
static const double EDGES[4] = {700e-9, 600e-9, 500e-9, 400e-9};  /* R, G, B bands */

double orc_absorption(int k, double lambda) {
  double x = (lambda - MU_ABS[k]) / S_ABS;
  return exp(-0.5 * x * x);
}

typedef struct {
  double T, a1, a2, D, D5;
  int weight;  /* 0: the spectrum, 1: B_T A1, 2: B_T A2 */
} spec_t;

static double spec_cb(double lambda, void* vc) {
  const spec_t* s = (const spec_t*)vc;
  double lp = s->D * lambda;
  double B = orc_planck(lp, s->T);
  if (s->weight == 1) return B * orc_absorption(0, lp);
  if (s->weight == 2) return B * orc_absorption(1, lp);
  return s->D5 * B * (1.0 - s->a1 * orc_absorption(0, lp) - s->a2 * orc_absorption(1, lp));
}

/* fixed panels: the spectrum may change sign, so its band integrals may cancel; 32
   panels of 3.125 nm keep the Gauss-Legendre rule exact to rounding for the Planck factor
   down to D T = 125 K (exponent at most ~2 per panel) */
static double band_int(spec_t* s, int b) {
  return orc_integrate_panels(spec_cb, s, EDGES[b + 1], EDGES[b], 32);
}

void orc_chroma_project(double r, double g, double out[2]) {
  r = r > 0.0 ? r : 0.0;
  g = g > 0.0 ? g : 0.0;
  if (r + g > 1.0) {
    double s = r + g;
    r /= s;
    g /= s;
  }
  out[0] = r;
  out[1] = g;
}

static double blue_red(double T) {
  double L[3];
  orc_band_radiance(T, L);
  return L[2] / L[0];
}

double orc_band_cct(double r, double g) {
  double c[2];
  orc_chroma_project(r, g, c);
  r = c[0];
  g = c[1];
  double b = 1.0 - r - g;
  if (b < 0.0) b = 0.0;
  if (b <= blue_red(T_LO) * r) return T_LO;
  if (b >= blue_red(T_HI) * r) return T_HI;
  double lo = log(T_LO), hi = log(T_HI);
  for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
    double mid = 0.5 * (lo + hi);
    if (blue_red(exp(mid)) * r < b)
      lo = mid;
    else
      hi = mid;
  }
  return exp(0.5 * (lo + hi));
}

void orc_spectrum_of(double r, double g, double out[3]) {
  double c[2];
  orc_chroma_project(r, g, c);
  r = c[0];
  g = c[1];
  double T = orc_band_cct(r, g);
  double P[3], Q1[3], Q2[3];
  spec_t s = {T, 0.0, 0.0, 1.0, 1.0, 0};
  for (int b = 0; b < 3; ++b) P[b] = band_int(&s, b);
  s.weight = 1;
  for (int b = 0; b < 3; ++b) Q1[b] = band_int(&s, b);
  s.weight = 2;
  for (int b = 0; b < 3; ++b) Q2[b] = band_int(&s, b);
  double sP = P[0] + P[1] + P[2], sQ1 = Q1[0] + Q1[1] + Q1[2], sQ2 = Q2[0] + Q2[1] + Q2[2];
  /* a1 (r sQ1 - Q1_R) + a2 (r sQ2 - Q2_R) = r sP - P_R, and the same with g and G */
  double m00 = r * sQ1 - Q1[0], m01 = r * sQ2 - Q2[0], y0 = r * sP - P[0];
  double m10 = g * sQ1 - Q1[1], m11 = g * sQ2 - Q2[1], y1 = g * sP - P[1];
  double det = m00 * m11 - m01 * m10;
  double scale = fabs(m00 * m11) + fabs(m01 * m10);
  out[0] = T;
  out[1] = out[2] = 0.0;
  if (fabs(det) > 1e-12 * scale && scale > 0.0) {
    out[1] = fmin(fmax((y0 * m11 - m01 * y1) / det, -8.0), 1.0);
    out[2] = fmin(fmax((m00 * y1 - y0 * m10) / det, -8.0), 1.0);
  }
}

void orc_color_shift(double r, double g, double D, double out[3]) {
  double sp[3];
  orc_spectrum_of(r, g, sp);
  spec_t s = {sp[0], sp[1], sp[2], 1.0, 1.0, 0};
  double den = band_int(&s, 0) + band_int(&s, 1) + band_int(&s, 2);
  s.D = D;
  s.D5 = D * D * D * D * D;
  for (int b = 0; b < 3; ++b) {
    double v = den > 0.0 ? band_int(&s, b) / den : 0.0;
    out[b] = v > 0.0 ? v : 0.0;
  }
}

/* the nodes of row i (r = i / (nr - 1)) */
static void table_row(int32_t i, int32_t nr, int32_t ng, int32_t nd, double* out) {
  const double floor_ = ldexp(1.0, -100);
  for (int32_t j = 0; j < ng; ++j) {
    double r = (double)i / (nr - 1), g = (double)j / (ng - 1);
    double sp[3];
    orc_spectrum_of(r, g, sp);
    spec_t s = {sp[0], sp[1], sp[2], 1.0, 1.0, 0};
    double den = band_int(&s, 0) + band_int(&s, 1) + band_int(&s, 2);
    for (int32_t k = 0; k < nd; ++k) {
      double D = exp2(-3.0 + 6.0 * k / (nd - 1));
      s.D = D;
      s.D5 = D * D * D * D * D;
      double* o = out + 3 * (((int64_t)i * ng + j) * nd + k);
      for (int b = 0; b < 3; ++b) {
        double v = den > 0.0 ? band_int(&s, b) / den : 0.0;
        o[b] = log2(v > floor_ ? v : floor_);
      }
    }
  }
}

typedef struct {
  int32_t nr, ng, nd, next;
  double* out;
  pthread_mutex_t mu;
} tjob;

static void* table_worker(void* p) {
  tjob* j = (tjob*)p;
  for (;;) {
    pthread_mutex_lock(&j->mu);
    int32_t i = j->next++;
    pthread_mutex_unlock(&j->mu);
    if (i >= j->nr) return NULL;
    table_row(i, j->nr, j->ng, j->nd, j->out);
  }
}

void orc_cshift_table(int32_t nr, int32_t ng, int32_t nd, double* out, int nthreads) {
  tjob j = {nr, ng, nd, 0, out, PTHREAD_MUTEX_INITIALIZER};
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  pthread_t th[64];
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, table_worker, &j);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

static double coord(double x, int32_t n, int32_t* i0) {
  x = fmin(fmax(x, 0.0), (double)(n - 1));
  int32_t i = (int32_t)floor(x);
  if (i > n - 2) i = n - 2;
  *i0 = i;
  return x - i;
}

void orc_cshift_lookup(const double* tab, int32_t nr, int32_t ng, int32_t nd, double r,
                       double g, double D, double out[3]) {
  int32_t i, j, k;
  double fx = coord(r * (nr - 1), nr, &i);
  double fy = coord(g * (ng - 1), ng, &j);
  double ld = fmin(fmax(log2(D), -3.0), 3.0);
  coord((ld + 3.0) / 6.0 * (nd - 1), nd, &k);
  double i0 = exp2(-(-3.0 + 6.0 * k / (nd - 1))), i1 = exp2(-(-3.0 + 6.0 * (k + 1) / (nd - 1)));
  double fz = (exp2(-ld) - i0) / (i1 - i0);
  fz = fmin(fmax(fz, 0.0), 1.0);
  for (int b = 0; b < 3; ++b) {
    double v = 0.0;
    for (int c = 0; c < 8; ++c) {
      int di = c & 1, dj = (c >> 1) & 1, dk = (c >> 2) & 1;
      double w = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy) * (dk ? fz : 1.0 - fz);
      v += w * tab[3 * (((int64_t)(i + di) * ng + (j + dj)) * nd + (k + dk)) + b];
    }
    out[b] = exp2(v);
  }
}
