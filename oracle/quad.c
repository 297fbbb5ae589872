/*
 * Adaptive Gauss-Legendre quadrature used by the oracle's table mode and band radiances.
 * TEST INFRASTRUCTURE ONLY (see bh_oracle.h).
 *
 * The 12-point nodes are generated at start-up by Newton iteration on the Legendre
 * polynomial P_12 (three-term recurrence); no tabulated constants.  Pinned by
 * orc_quad_poly_check (exact for polynomials up to degree 23) and by the scipy/mpmath
 * comparisons in the test suite.
 */
#include <math.h>
#include <pthread.h>

#include "bh_oracle.h"
#include "oracle_internal.h"

#define GL_N 12
static double gl_x[GL_N], gl_w[GL_N];
static pthread_once_t gl_once = PTHREAD_ONCE_INIT;

static void legendre(int n, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x;
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *p = p1;
  *dp = n * (x * p1 - p0) / (x * x - 1.0);
}

static void gl_init(void) {
  for (int i = 0; i < GL_N; ++i) {
    double x = cos(M_PI * (i + 0.75) / (GL_N + 0.5));
    double p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(GL_N, x, &p, &dp);
      double dx = p / dp;
      x -= dx;
      if (fabs(dx) < 1e-17) break;
    }
    legendre(GL_N, x, &p, &dp);
    gl_x[i] = x;
    gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

static double gl_rule(orc_fn f, void* ctx, double a, double b) {
  double m = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
  for (int i = 0; i < GL_N; ++i) s += gl_w[i] * f(m + h * gl_x[i], ctx);
  return s * h;
}

/* Each half gets half the tolerance, but never less than floor_tol (a fixed fraction of
 * the whole integral): below that, differences are rounding noise and refining further
 * would only multiply the work. */
static double adapt(orc_fn f, void* ctx, double a, double b, double whole, double tol,
                    double floor_tol, int depth) {
  double m = 0.5 * (a + b);
  double l = gl_rule(f, ctx, a, m), r = gl_rule(f, ctx, m, b);
  if (depth >= 40 || fabs(l + r - whole) <= fmax(tol, floor_tol)) return l + r;
  return adapt(f, ctx, a, m, l, 0.5 * tol, floor_tol, depth + 1) +
         adapt(f, ctx, m, b, r, 0.5 * tol, floor_tol, depth + 1);
}

double orc_integrate(orc_fn f, void* ctx, double a, double b, double rel_tol) {
  pthread_once(&gl_once, gl_init);
  if (b == a) return 0.0;
  double whole = gl_rule(f, ctx, a, b);
  double tol = rel_tol * fabs(whole);
  if (tol < 1e-300) tol = 1e-300;
  return adapt(f, ctx, a, b, whole, tol, 1e-15 * fabs(whole), 0);
}

double orc_integrate_panels(orc_fn f, void* ctx, double a, double b, int panels) {
  pthread_once(&gl_once, gl_init);
  double s = 0.0, h = (b - a) / panels;
  for (int i = 0; i < panels; ++i) s += gl_rule(f, ctx, a + i * h, a + (i + 1) * h);
  return s;
}

static double poly(double x, void* ctx) { return pow(x, *(int*)ctx); }

double orc_quad_poly_check(int degree) {
  pthread_once(&gl_once, gl_init);
  /* single 12-point rule on [0, 1]: exact for degree <= 23 */
  double got = gl_rule(poly, &degree, 0.0, 1.0);
  return got - 1.0 / (degree + 1.0);
}
