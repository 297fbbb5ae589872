/*
 * Blackbody band radiances and the star cubemap.  TEST INFRASTRUCTURE ONLY (bh_oracle.h).
 *
 * Colour model.  The disc emits as a blackbody at temperature T(u) (Section 3.3.3
 * "Emitted light"), and for blackbodies the Doppler shift plus beaming reduce to the
 * temperature shift T -> (nu/nu') T (Section 3.4.2).  Reading: instead of CIE XYZ and the
 * C(xy, D) table (whose colour-matching data and absorption spectra are not given), colour
 * is the Planck spectral radiance integrated over three box bands, R = 600-700 nm,
 * G = 500-600 nm, B = 400-500 nm, in W m^-2 sr^-1.
 *
 * Star cubemap (Section 3.3.2, "Emitted light", first bullet).  Each texel of each mip
 * level holds (I, T, p_u, p_v): the intensity sum of the stars inside it, their
 * intensity-weighted mean temperature and their intensity-weighted mean position inside
 * the texel in [0, 1)^2.  Mip levels combine the four children with the same rule (sum of
 * intensities, intensity-weighted averages).  Readings: stars that fall into the same
 * level-0 texel are merged with the mip rule; the weighted mean temperature stands in for
 * the colour sum; the position is stored, not derived from a colour hash.
 * Face of a unit direction d: k = argmax |d_k| (ties to the lowest index), face index
 * 2k + (d_k < 0), face coordinates U = d_{(k+1)%3} / |d_k|, V = d_{(k+2)%3} / |d_k|
 * (the +z example of the paper, U = d_x / d_z, extended to all faces).
 * Layout: level L (size n0 >> L) starts after all lower levels; within a level
 * ((face * nL + y) * nL + x) * 4 doubles.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "bh_oracle.h"
#include "oracle_internal.h"

static const double H_PLANCK = 6.62607015e-34;
static const double C_LIGHT = 299792458.0;
static const double K_BOLTZ = 1.380649e-23;

double orc_planck(double lambda, double T) {
  if (!(T > 0.0)) return 0.0;
  double x = H_PLANCK * C_LIGHT / (lambda * K_BOLTZ * T);
  double l5 = lambda * lambda * lambda * lambda * lambda;
  double pref = 2.0 * H_PLANCK * C_LIGHT * C_LIGHT / l5;
  if (x > 700.0) return 0.0;
  return pref / expm1(x);
}

static double planck_cb(double lambda, void* ctx) { return orc_planck(lambda, *(double*)ctx); }

void orc_band_radiance(double T, double out[3]) {
  static const double edges[4] = {700e-9, 600e-9, 500e-9, 400e-9};
  for (int b = 0; b < 3; ++b)
    out[b] = orc_integrate(planck_cb, &T, edges[b + 1], edges[b], 1e-13);
}

/* ---- cubemap ---------------------------------------------------------------------- */

static int levels_of(int32_t n0) {
  int l = 0;
  while ((n0 >> l) >= 1) ++l;
  return l;
}

int64_t orc_cubemap_texels(int32_t n0) {
  int64_t t = 0;
  for (int l = 0; (n0 >> l) >= 1; ++l) t += 6LL * (n0 >> l) * (n0 >> l);
  return t;
}

/* level-0 texel of direction d: face, column, row and the position inside the texel in
   [0, 1)^2; 0 for the zero vector */
static int star_texel(const double* d, int32_t n0, int64_t* t, double* fu, double* fv) {
  int k = 0;
  if (fabs(d[1]) > fabs(d[k])) k = 1;
  if (fabs(d[2]) > fabs(d[k])) k = 2;
  double m = fabs(d[k]);
  if (!(m > 0.0)) return 0;
  int face = 2 * k + (d[k] < 0.0);
  double U = d[(k + 1) % 3] / m, V = d[(k + 2) % 3] / m;
  double gx = 0.5 * (U + 1.0) * n0, gy = 0.5 * (V + 1.0) * n0;
  int64_t ix = (int64_t)floor(gx), iy = (int64_t)floor(gy);
  if (ix < 0) ix = 0;
  if (ix > n0 - 1) ix = n0 - 1;
  if (iy < 0) iy = 0;
  if (iy > n0 - 1) iy = n0 - 1;
  *t = ((int64_t)face * n0 + iy) * n0 + ix;
  *fu = gx - ix;
  *fv = gy - iy;
  return 1;
}

/* Band-colour star map (light of any colour, spectrum.c): each texel holds the band sums
 * (R, G, B) of its stars and their position inside the texel weighted by S = R + G + B;
 * mips combine the four children by the same rule.  Layout as the (I, T) map with 5
 * doubles per texel: (R, G, B, p_u, p_v).  Stars with S = 0 are left out; a negative or
 * non-finite band returns 2. */
int orc_cubemap_build_bands(const float* dirs, const float* rgb, int64_t n, int32_t n0,
                            double* tex) {
  if (n0 < 1 || (n0 & (n0 - 1))) return 1;
  for (int64_t s = 0; s < 3 * n; ++s)
    if (!(rgb[s] >= 0.0f) || isinf(rgb[s])) return 2;
  int nl = levels_of(n0);
  int64_t total = orc_cubemap_texels(n0);
  memset(tex, 0, sizeof(double) * 5 * total);
  double* acc = (double*)calloc((size_t)6 * n0 * n0 * 5, sizeof(double));
  if (!acc) return 3;
  for (int64_t s = 0; s < n; ++s) {
    double d[3] = {dirs[3 * s], dirs[3 * s + 1], dirs[3 * s + 2]};
    double c[3] = {rgb[3 * s], rgb[3 * s + 1], rgb[3 * s + 2]};
    double S = c[0] + c[1] + c[2];
    int64_t t;
    double fu, fv;
    if (!(S > 0.0) || !star_texel(d, n0, &t, &fu, &fv)) continue;
    double* a = acc + t * 5;
    for (int b = 0; b < 3; ++b) a[b] += c[b];
    a[3] += S * fu;
    a[4] += S * fv;
  }
  for (int64_t t = 0; t < 6LL * n0 * n0; ++t) {
    const double* a = acc + t * 5;
    double* o = tex + t * 5;
    double S = a[0] + a[1] + a[2];
    if (S > 0.0) {
      for (int b = 0; b < 3; ++b) o[b] = a[b];
      o[3] = a[3] / S;
      o[4] = a[4] / S;
    }
  }
  free(acc);
  int64_t off_prev = 0;
  for (int l = 1; l < nl; ++l) {
    int32_t np = n0 >> (l - 1), nc = n0 >> l;
    int64_t off = off_prev + 6LL * np * np;
    for (int f = 0; f < 6; ++f)
      for (int32_t y = 0; y < nc; ++y)
        for (int32_t x = 0; x < nc; ++x) {
          double sc[3] = {0, 0, 0}, su = 0, sv = 0;
          for (int c = 0; c < 4; ++c) {
            int cx = 2 * x + (c & 1), cy = 2 * y + (c >> 1);
            const double* ch = tex + (off_prev + ((int64_t)f * np + cy) * np + cx) * 5;
            double S = ch[0] + ch[1] + ch[2];
            if (!(S > 0.0)) continue;
            for (int b = 0; b < 3; ++b) sc[b] += ch[b];
            su += S * 0.5 * ((c & 1) + ch[3]);
            sv += S * 0.5 * ((c >> 1) + ch[4]);
          }
          double S = sc[0] + sc[1] + sc[2];
          double* o = tex + (off + ((int64_t)f * nc + y) * nc + x) * 5;
          if (S > 0.0) {
            for (int b = 0; b < 3; ++b) o[b] = sc[b];
            o[3] = su / S;
            o[4] = sv / S;
          }
        }
    off_prev = off;
  }
  return 0;
}

int orc_cubemap_build(const float* dirs, const float* inten, const float* temp, int64_t n,
                      int32_t n0, double* tex) {
  if (n0 < 1 || (n0 & (n0 - 1))) return 1;
  int nl = levels_of(n0);
  int64_t total = orc_cubemap_texels(n0);
  memset(tex, 0, sizeof(double) * 4 * total);
  /* level 0: accumulate sums I, I*T, I*(x + p_u), I*(y + p_v) ... in star order */
  double* acc = (double*)calloc((size_t)6 * n0 * n0 * 4, sizeof(double));
  if (!acc) return 2;
  for (int64_t s = 0; s < n; ++s) {
    double d[3] = {dirs[3 * s], dirs[3 * s + 1], dirs[3 * s + 2]};
    double I = inten[s], T = temp[s];
    int64_t t;
    double fu, fv;
    if (!(I > 0.0) || !star_texel(d, n0, &t, &fu, &fv)) continue;
    double* a = acc + t * 4;
    a[0] += I;
    a[1] += I * T;
    a[2] += I * fu;
    a[3] += I * fv;
  }
  for (int64_t t = 0; t < 6LL * n0 * n0; ++t) {
    double* a = acc + t * 4;
    double* o = tex + t * 4;
    if (a[0] > 0.0) {
      o[0] = a[0];
      o[1] = a[1] / a[0];
      o[2] = a[2] / a[0];
      o[3] = a[3] / a[0];
    }
  }
  free(acc);
  /* mips: children (0,0), (1,0), (0,1), (1,1) of each parent */
  int64_t off_prev = 0;
  for (int l = 1; l < nl; ++l) {
    int32_t np = n0 >> (l - 1), nc = n0 >> l;
    int64_t off = off_prev + 6LL * np * np;
    for (int f = 0; f < 6; ++f)
      for (int32_t y = 0; y < nc; ++y)
        for (int32_t x = 0; x < nc; ++x) {
          double sI = 0, sIT = 0, sIu = 0, sIv = 0;
          for (int c = 0; c < 4; ++c) {
            int cx = 2 * x + (c & 1), cy = 2 * y + (c >> 1);
            const double* ch = tex + (off_prev + ((int64_t)f * np + cy) * np + cx) * 4;
            if (!(ch[0] > 0.0)) continue;
            sI += ch[0];
            sIT += ch[0] * ch[1];
            sIu += ch[0] * 0.5 * ((c & 1) + ch[2]);
            sIv += ch[0] * 0.5 * ((c >> 1) + ch[3]);
          }
          double* o = tex + (off + ((int64_t)f * nc + y) * nc + x) * 4;
          if (sI > 0.0) {
            o[0] = sI;
            o[1] = sIT / sI;
            o[2] = sIu / sI;
            o[3] = sIv / sI;
          }
        }
    off_prev = off;
  }
  return 0;
}
