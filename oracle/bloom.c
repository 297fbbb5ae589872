/*
 * Bloom (lens glare, Section 3.4.3): a point spread function
 * approximated by small-support filters on the mipmaps of the final image, applied before
 * tone mapping.  TEST INFRASTRUCTURE ONLY (see bh_oracle.h).
 *
 * The paper names the filters' idea only; this is its reading, computed here in plain
 * loops over whole images in FP64:
 *   P_0 = I, the linear RGBA image (W x H, row-major);
 *   P_k = the 2 x 2 box average of P_{k-1}, of size ceil(n / 2) per axis, source indices
 *         clamped to the last row / column (k = 1 .. K);
 *   U_K = w_K P_K;  U_k = w_k P_k + up(U_{k+1}) for k = K-1 .. 1;
 *   O   = w_0 I + up(U_1)  (for K = 0: O = w_0 I);
 * up() doubles the resolution by bilinear interpolation: fine pixel x reads the coarse
 * grid at x / 2 - 1/4 (pixel centres at half-integers), coarse indices clamped to the
 * edge.  The weights w_0 .. w_K shape the point spread function; with sum 1 an interior
 * impulse keeps its flux and a linear image is reproduced.
 */
#include <stdlib.h>
#include <string.h>

#include "bh_oracle.h"

static int half_up(int n) { return (n + 1) / 2; }

static int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

/* 2 x 2 box average with clamped source indices */
static void box_down(const double* src, int w, int h, double* dst, int w2, int h2) {
  for (int y = 0; y < h2; ++y)
    for (int x = 0; x < w2; ++x)
      for (int c = 0; c < 4; ++c) {
        double s = 0.0;
        for (int b = 0; b < 2; ++b)
          for (int a = 0; a < 2; ++a)
            s += src[((size_t)clampi(2 * y + b, h) * w + clampi(2 * x + a, w)) * 4 + c];
        dst[((size_t)y * w2 + x) * 4 + c] = 0.25 * s;
      }
}

/* bilinear value of the coarse image (cw x ch) at fine pixel (x, y) */
static void up_at(const double* cs, int cw, int ch, int x, int y, double out[4]) {
  /* coarse coordinate x / 2 - 1/4: the two coarse neighbours and the weight of the upper */
  int x0 = (x - 1) >> 1, y0 = (y - 1) >> 1; /* floor((x - 1) / 2) */
  double fx = (x & 1) ? 0.25 : 0.75, fy = (y & 1) ? 0.25 : 0.75;
  int xa = clampi(x0, cw), xb = clampi(x0 + 1, cw), ya = clampi(y0, ch), yb = clampi(y0 + 1, ch);
  for (int c = 0; c < 4; ++c) {
    double v00 = cs[((size_t)ya * cw + xa) * 4 + c], v10 = cs[((size_t)ya * cw + xb) * 4 + c];
    double v01 = cs[((size_t)yb * cw + xa) * 4 + c], v11 = cs[((size_t)yb * cw + xb) * 4 + c];
    out[c] = (1 - fy) * ((1 - fx) * v00 + fx * v10) + fy * ((1 - fx) * v01 + fx * v11);
  }
}

int orc_bloom(const double* in, int32_t width, int32_t height, int32_t levels,
              const double* weights, double* out) {
  if (width < 1 || height < 1 || levels < 0 || levels > 16) return 1;
  int K = levels;
  int ws[17], hs[17];
  double* P[17];
  double* U[17];
  ws[0] = width;
  hs[0] = height;
  P[0] = (double*)in;
  for (int k = 1; k <= K; ++k) {
    ws[k] = half_up(ws[k - 1]);
    hs[k] = half_up(hs[k - 1]);
    P[k] = (double*)malloc(sizeof(double) * 4 * (size_t)ws[k] * hs[k]);
    U[k] = (double*)malloc(sizeof(double) * 4 * (size_t)ws[k] * hs[k]);
    box_down(P[k - 1], ws[k - 1], hs[k - 1], P[k], ws[k], hs[k]);
  }
  for (int k = K; k >= 1; --k) {
    for (int y = 0; y < hs[k]; ++y)
      for (int x = 0; x < ws[k]; ++x) {
        double u[4] = {0, 0, 0, 0};
        if (k < K) up_at(U[k + 1], ws[k + 1], hs[k + 1], x, y, u);
        for (int c = 0; c < 4; ++c) {
          size_t i = ((size_t)y * ws[k] + x) * 4 + c;
          U[k][i] = weights[k] * P[k][i] + u[c];
        }
      }
  }
  for (int y = 0; y < height; ++y)
    for (int x = 0; x < width; ++x) {
      double u[4] = {0, 0, 0, 0};
      if (K >= 1) up_at(U[1], ws[1], hs[1], x, y, u);
      for (int c = 0; c < 4; ++c) {
        size_t i = ((size_t)y * width + x) * 4 + c;
        out[i] = weights[0] * in[i] + u[c];
      }
    }
  for (int k = 1; k <= K; ++k) {
    free(P[k]);
    free(U[k]);
  }
  return 0;
}
