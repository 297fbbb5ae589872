/*
 * Extended (area) sources: a radiance cube map sampled over the pixel's footprint.
 * TEST INFRASTRUCTURE ONLY (bh_oracle.h).
 *
 * Section 3.3.2 ("Emitted light") stores nebulae and galaxies in a cube map read with
 * anisotropic texture filtering over the beam's footprint, and Section 3.4.1 notes that
 * the lensing amplification Omega/Omega' does not apply to them (their radiance is
 * carried unchanged along the beam).  The paper leaves the filter to the texture hardware;
 * the readings below fix one, and the exact footprint mean it approximates.
 *
 * Map.  Each level-0 texel holds a radiance I and a colour temperature T (blackbody
 * colour, the band model of emission.c).  Stored per level: (I, I T).  Level L + 1 is the
 * mean of its four children in both channels (a box pyramid of an intensive quantity, so
 * every level has the same map mean).  Layout as the star cubemap: level L after all lower
 * levels, ((face * nL + y) * nL + x) * 2 doubles; faces and (U, V) as in emission.c.
 * Band maps (light of any colour, spectrum.c) hold the band radiances (R, G, B) per texel
 * instead: 3 doubles per texel, the same pyramid and filters on all three channels.
 *
 * Footprint (reading).  The pixel's beam covers the parallelogram of directions
 * p(w, h) = d' + w d_w d' + h d_h d', (w, h) in [-1/2, 1/2]^2, with the same fine quad
 * differences d_w d', d_h d' as the star filter; the pixel receives the mean of the map
 * over it, uniform in (w, h) (a box pixel).
 *
 * Exact mean (orc_area_exact).  With the level-0 map piecewise constant (nearest texel),
 * the mean is a sum over texels of value x area of the set of (w, h) whose direction falls
 * in that texel.  p is affine in (w, h), so on face k with sign s the conditions
 * s p_k >= |p_a|, |p_b| and (2 i / n0 - 1) s p_k <= p_a < (2 (i + 1) / n0 - 1) s p_k (and
 * the same for rows with p_b) are half-planes in (w, h): each texel's set is the unit
 * square clipped by at most eight half-planes, a convex polygon whose area is exact.
 *
 * Anisotropic filter (orc_area_filter), the method's approximation of that mean, in the
 * manner of texture hardware: the footprint's two axes d_w d', d_h d' are measured in
 * level-0 texels on the face of d' (the face Jacobian of the star filter, Euclidean
 * length); the longer is the major axis.  Probes sit at the centres of an N_maj x N_min
 * grid over the parallelogram, spaced no closer than half a level-0 texel: with
 * s = max(l_min / 2, 1/2), N_maj = clamp(ceil(l_maj / s), 1, 16) along the major axis and
 * N_min = clamp(ceil(l_min / s), 1, 2) across it (for l_min >= 1 that is
 * ceil(2 l_maj / l_min) by 2; a footprint below a texel takes a single probe, as texture
 * hardware does when magnifying); all probes read level
 * lambda = log2(max(l_maj / N_maj, l_min / N_min)) - 1 (one level sharper than the probe
 * spacing), clamped to [0, levels - 1], trilinearly: bilinear on levels floor(lambda) and
 * floor(lambda) + 1, mixed by the fraction.  Bilinear reads take the face of the probe's
 * own direction (so a footprint may span cube edges), texel centres at
 * ((x + 1/2) 2 / nL - 1), coordinates clamped to the face's outermost texel centres.  The
 * result is the mean over the probes.
 * Parity: orc_area_exact is pinned by closed forms (constant maps, footprints inside one
 * texel, a split across a cube edge) and by brute-force sampling; orc_area_filter by a
 * constant map, maps linear in U on a face (reproduced exactly), and its distance to the
 * exact mean on smooth maps.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "bh_oracle.h"

static int area_levels(int32_t n0) {
  int l = 0;
  while ((n0 >> l) >= 1) ++l;
  return l;
}

int64_t orc_area_texels(int32_t n0) {
  int64_t t = 0;
  for (int l = 0; (n0 >> l) >= 1; ++l) t += 6LL * (n0 >> l) * (n0 >> l);
  return t;
}

static int64_t level_offset(int32_t n0, int L) {
  int64_t off = 0;
  for (int l = 0; l < L; ++l) off += 6LL * (n0 >> l) * (n0 >> l);
  return off;
}

/* levels 1 .. of an nch-channel map whose level 0 is filled: box means of four children */
static void build_mips(int32_t n0, int nch, double* levels) {
  int nl = area_levels(n0);
  for (int L = 1; L < nl; ++L) {
    int32_t nc = n0 >> (L - 1), nL = n0 >> L;
    const double* src = levels + nch * level_offset(n0, L - 1);
    double* dst = levels + nch * level_offset(n0, L);
    for (int f = 0; f < 6; ++f)
      for (int32_t y = 0; y < nL; ++y)
        for (int32_t x = 0; x < nL; ++x)
          for (int c = 0; c < nch; ++c) {
            double s = 0.0;
            for (int dy = 0; dy < 2; ++dy)
              for (int dx = 0; dx < 2; ++dx)
                s += src[nch * (((int64_t)f * nc + 2 * y + dy) * nc + 2 * x + dx) + c];
            dst[nch * (((int64_t)f * nL + y) * nL + x) + c] = 0.25 * s;
          }
  }
}

int orc_area_build(const float* it, int32_t n0, double* levels) {
  if (n0 < 1 || (n0 & (n0 - 1))) return 1;
  int64_t n = 6LL * n0 * n0;
  for (int64_t t = 0; t < n; ++t) {
    double I = it[2 * t], T = it[2 * t + 1];
    if (!(I >= 0.0) || !(T >= 0.0)) return 2;
    levels[2 * t] = I;
    levels[2 * t + 1] = I * T;
  }
  build_mips(n0, 2, levels);
  return 0;
}

int orc_area_build_bands(const float* rgbx, int32_t n0, double* levels) {
  if (n0 < 1 || (n0 & (n0 - 1))) return 1;
  int64_t n = 6LL * n0 * n0;
  for (int64_t t = 0; t < n; ++t)
    for (int c = 0; c < 3; ++c) {
      double v = rgbx[4 * t + c];
      if (!(v >= 0.0) || isinf(v)) return 2;
      levels[3 * t + c] = v;
    }
  build_mips(n0, 3, levels);
  return 0;
}

/* face of a direction: k = argmax |p_k| (ties to the lowest index), face 2k + (p_k < 0) */
static int face_of(const double* p, int* k, double* U, double* V) {
  int kk = 0;
  if (fabs(p[1]) > fabs(p[kk])) kk = 1;
  if (fabs(p[2]) > fabs(p[kk])) kk = 2;
  double m = fabs(p[kk]);
  *k = kk;
  *U = p[(kk + 1) % 3] / m;
  *V = p[(kk + 2) % 3] / m;
  return 2 * kk + (p[kk] < 0.0);
}

/* bilinear read of the nch channels of level L at direction p */
static void bilinear(const double* levels, int nch, int32_t n0, int L, const double* p,
                     double* out) {
  int k;
  double U, V;
  int f = face_of(p, &k, &U, &V);
  int32_t nL = n0 >> L;
  const double* t = levels + nch * (level_offset(n0, L) + (int64_t)f * nL * nL);
  if (nL == 1) {
    for (int c = 0; c < nch; ++c) out[c] = t[c];
    return;
  }
  double x = 0.5 * (U + 1.0) * nL - 0.5, y = 0.5 * (V + 1.0) * nL - 0.5;
  x = fmin(fmax(x, 0.0), nL - 1.0);
  y = fmin(fmax(y, 0.0), nL - 1.0);
  int32_t i0 = (int32_t)floor(x), j0 = (int32_t)floor(y);
  if (i0 > nL - 2) i0 = nL - 2;
  if (j0 > nL - 2) j0 = nL - 2;
  double fx = x - i0, fy = y - j0;
  for (int c = 0; c < nch; ++c) {
    double a = t[nch * ((int64_t)j0 * nL + i0) + c];
    double b = t[nch * ((int64_t)j0 * nL + i0 + 1) + c];
    double d = t[nch * ((int64_t)(j0 + 1) * nL + i0) + c];
    double e = t[nch * ((int64_t)(j0 + 1) * nL + i0 + 1) + c];
    out[c] = (1.0 - fy) * ((1.0 - fx) * a + fx * b) + fy * ((1.0 - fx) * d + fx * e);
  }
}

/* length in level-0 texels of the face-coordinate change along direction change a */
static double axis_texels(const double* d, const double* a, int32_t n0) {
  int k;
  double U, V;
  face_of(d, &k, &U, &V);
  double m = fabs(d[k]), sg = d[k] < 0.0 ? -1.0 : 1.0;
  double dU = (a[(k + 1) % 3] - U * sg * a[k]) / m;
  double dV = (a[(k + 2) % 3] - V * sg * a[k]) / m;
  return 0.5 * n0 * sqrt(dU * dU + dV * dV);
}

static void filter_n(const double* levels, int nch, int32_t n0, const double* d,
                     const double* dw, const double* dh, double* out) {
  int nl = area_levels(n0);
  double la = axis_texels(d, dw, n0), lb = axis_texels(d, dh, n0);
  const double *maj = dw, *mn = dh;
  double lmaj = la, lmin = lb;
  if (lb > la) {
    maj = dh;
    mn = dw;
    lmaj = lb;
    lmin = la;
  }
  double spc = fmax(0.5 * lmin, 0.5);
  double r = ceil(lmaj / spc);
  int nmaj = r < 1.0 ? 1 : (r > 16.0 ? 16 : (int)r);
  int nmin = lmin / spc > 1.0 ? 2 : 1;
  double s = fmax(lmaj / nmaj, lmin / nmin);
  double lam = s > 0.0 ? log2(s) - 1.0 : 0.0;
  lam = fmin(fmax(lam, 0.0), (double)(nl - 1));
  int L0 = (int)floor(lam);
  int L1 = L0 + 1 < nl ? L0 + 1 : L0;
  double fr = lam - L0;
  double sum[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < nmaj; ++a)
    for (int b = 0; b < nmin; ++b) {
      double ta = (a + 0.5) / nmaj - 0.5, tb = (b + 0.5) / nmin - 0.5;
      double p[3], v0[3], v1[3];
      for (int i = 0; i < 3; ++i) p[i] = d[i] + ta * maj[i] + tb * mn[i];
      bilinear(levels, nch, n0, L0, p, v0);
      bilinear(levels, nch, n0, L1, p, v1);
      for (int c = 0; c < nch; ++c) sum[c] += (1.0 - fr) * v0[c] + fr * v1[c];
    }
  for (int c = 0; c < nch; ++c) out[c] = sum[c] / (nmaj * nmin);
}

void orc_area_filter(const double* levels, int32_t n0, const double* d, const double* dw,
                     const double* dh, double* A, double* B) {
  double o[2];
  filter_n(levels, 2, n0, d, dw, dh, o);
  *A = o[0];
  *B = o[1];
}

void orc_area_filter_bands(const double* levels, int32_t n0, const double* d, const double* dw,
                           const double* dh, double out[3]) {
  filter_n(levels, 3, n0, d, dw, dh, out);
}

/* ---- exact footprint mean ------------------------------------------------------------ */

#define MAXV 24

typedef struct {
  int n;
  double w[MAXV], h[MAXV];
} poly;

/* keep the part of P where c0 + c1 w + c2 h >= 0 (Sutherland-Hodgman, one edge) */
static void clip(const poly* P, double c0, double c1, double c2, poly* Q) {
  Q->n = 0;
  for (int i = 0; i < P->n; ++i) {
    int j = (i + 1) % P->n;
    double fi = c0 + c1 * P->w[i] + c2 * P->h[i];
    double fj = c0 + c1 * P->w[j] + c2 * P->h[j];
    if (fi >= 0.0 && Q->n < MAXV) {
      Q->w[Q->n] = P->w[i];
      Q->h[Q->n] = P->h[i];
      Q->n++;
    }
    if ((fi >= 0.0) != (fj >= 0.0) && Q->n < MAXV) {
      double t = fi / (fi - fj);
      Q->w[Q->n] = P->w[i] + t * (P->w[j] - P->w[i]);
      Q->h[Q->n] = P->h[i] + t * (P->h[j] - P->h[i]);
      Q->n++;
    }
  }
}

static double area_of(const poly* P) {
  double s = 0.0;
  for (int i = 0; i < P->n; ++i) {
    int j = (i + 1) % P->n;
    s += P->w[i] * P->h[j] - P->w[j] * P->h[i];
  }
  return 0.5 * fabs(s);
}

/* coefficients (c0, c1, c2) of component i of p(w, h) = d + w dw + h dh */
static void comp(const double* d, const double* dw, const double* dh, int i, double c[3]) {
  c[0] = d[i];
  c[1] = dw[i];
  c[2] = dh[i];
}

static void exact_n(const double* levels, int nch, int32_t n0, const double* d,
                    const double* dw, const double* dh, double* out) {
  double sum[3] = {0.0, 0.0, 0.0};
  poly sq = {4, {-0.5, 0.5, 0.5, -0.5}, {-0.5, -0.5, 0.5, 0.5}};
  for (int f = 0; f < 6; ++f) {
    int k = f / 2, a = (k + 1) % 3, b = (k + 2) % 3;
    double s = (f & 1) ? -1.0 : 1.0;
    double pk[3], pa[3], pb[3];
    comp(d, dw, dh, k, pk);
    comp(d, dw, dh, a, pa);
    comp(d, dw, dh, b, pb);
    for (int i = 0; i < 3; ++i) pk[i] *= s; /* s p_k */
    /* face region: s p_k - p_a >= 0, s p_k + p_a >= 0, and the same with p_b */
    poly P = sq, Q;
    clip(&P, pk[0] - pa[0], pk[1] - pa[1], pk[2] - pa[2], &Q);
    clip(&Q, pk[0] + pa[0], pk[1] + pa[1], pk[2] + pa[2], &P);
    clip(&P, pk[0] - pb[0], pk[1] - pb[1], pk[2] - pb[2], &Q);
    clip(&Q, pk[0] + pb[0], pk[1] + pb[1], pk[2] + pb[2], &P);
    if (P.n < 3 || area_of(&P) <= 0.0) continue;
    /* texel ranges from the vertices' (U, V) (linear-fractional: extremes at vertices) */
    double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
    for (int i = 0; i < P.n; ++i) {
      double den = pk[0] + pk[1] * P.w[i] + pk[2] * P.h[i];
      if (!(den > 0.0)) continue;
      double U = (pa[0] + pa[1] * P.w[i] + pa[2] * P.h[i]) / den;
      double V = (pb[0] + pb[1] * P.w[i] + pb[2] * P.h[i]) / den;
      umin = fmin(umin, U);
      umax = fmax(umax, U);
      vmin = fmin(vmin, V);
      vmax = fmax(vmax, V);
    }
    if (umin > umax) continue;
    int32_t i0 = (int32_t)floor(0.5 * (umin + 1.0) * n0), i1 = (int32_t)floor(0.5 * (umax + 1.0) * n0);
    int32_t j0 = (int32_t)floor(0.5 * (vmin + 1.0) * n0), j1 = (int32_t)floor(0.5 * (vmax + 1.0) * n0);
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    if (i1 > n0 - 1) i1 = n0 - 1;
    if (j1 > n0 - 1) j1 = n0 - 1;
    const double* tex = levels + nch * (int64_t)f * n0 * n0;
    for (int32_t i = i0; i <= i1; ++i) {
      /* column i: (2i/n0 - 1) s p_k <= p_a <= (2(i+1)/n0 - 1) s p_k; the outermost columns
         reach the face edge, already enforced */
      double lo = 2.0 * i / n0 - 1.0, hi = 2.0 * (i + 1) / n0 - 1.0;
      poly C = P, C2;
      if (i > 0) {
        clip(&C, pa[0] - lo * pk[0], pa[1] - lo * pk[1], pa[2] - lo * pk[2], &C2);
        C = C2;
      }
      if (i < n0 - 1) {
        clip(&C, hi * pk[0] - pa[0], hi * pk[1] - pa[1], hi * pk[2] - pa[2], &C2);
        C = C2;
      }
      if (C.n < 3) continue;
      for (int32_t j = j0; j <= j1; ++j) {
        double vlo = 2.0 * j / n0 - 1.0, vhi = 2.0 * (j + 1) / n0 - 1.0;
        poly R = C, R2;
        if (j > 0) {
          clip(&R, pb[0] - vlo * pk[0], pb[1] - vlo * pk[1], pb[2] - vlo * pk[2], &R2);
          R = R2;
        }
        if (j < n0 - 1) {
          clip(&R, vhi * pk[0] - pb[0], vhi * pk[1] - pb[1], vhi * pk[2] - pb[2], &R2);
          R = R2;
        }
        if (R.n < 3) continue;
        double ar = area_of(&R);
        const double* t = tex + nch * ((int64_t)j * n0 + i);
        for (int c = 0; c < nch; ++c) sum[c] += ar * t[c];
      }
    }
  }
  for (int c = 0; c < nch; ++c) out[c] = sum[c];
}

void orc_area_exact(const double* levels, int32_t n0, const double* d, const double* dw,
                    const double* dh, double* A, double* B) {
  double o[2];
  exact_n(levels, 2, n0, d, dw, dh, o);
  *A = o[0];
  *B = o[1];
}

void orc_area_exact_bands(const double* levels, int32_t n0, const double* d, const double* dw,
                          const double* dh, double out[3]) {
  exact_n(levels, 3, n0, d, dw, dh, out);
}
