/*
 * Ray marching: the ablation the paper measures its tables against (Section 5, method M3
 * of Table 1): TraceRay is replaced by a numerical integration of the orbit equation
 * u'' = 3/2 u^2 - u (Section 3.3, eq. rayequation) with a bounded number of steps, and
 * everything else is left as it is.  TEST INFRASTRUCTURE ONLY (see bh_oracle.h).
 *
 * The paper states the equation and the step budget only.  This is its reading:
 *  - the state is (u, w = du/dphi), starting from (u_c, -u_c cot delta) at phi = 0, the
 *    start of Algorithm 1;
 *  - classic fourth-order Runge-Kutta in phi with the constant step h = 2 pi / N and at most
 *    N steps, so that the march covers one full turn of the beam plane;
 *  - inside a step u(phi) is the cubic Hermite interpolant of the two end states (values
 *    and slopes), which keeps the events at the integrator's order:
 *      escape  -- u ends a step below 0: delta' is the angle of the first root of the
 *                 cubic in the step;
 *      capture -- u ends a step at or above 1 (the horizon);
 *      disc    -- at each disc-plane angle alpha + m pi the step passes (m = 0, 1, ...,
 *                 strictly ahead of the camera, as in exact mode) the cubic gives u; the
 *                 crossing counts when u_oc <= u <= u_ic; it lies after the apsis
 *                 when the beam started inward and the cubic's slope there is negative;
 *  - a ray that has neither escaped nor been captured after N steps is unfinished and is
 *    drawn as captured (it wound more than once around the hole).
 * There is no shortcut for rays that cannot escape: every ray is integrated, except beams
 * within 1e-6 of the radius (|cot delta| >= 1e6), which move along r only: outward they
 * escape at delta' = delta, inward they fall in.
 */
#include <math.h>
#include <string.h>

#include "bh_oracle.h"
#include "oracle_internal.h"

static inline double acc(double u, double gr) { return 1.5 * gr * u * u - u; }

/* one classic Runge-Kutta step of (u, w)' = (w, 3/2 gr u^2 - u) */
static void rk4(double* u, double* w, double h, double gr) {
  double u1 = *u, w1 = *w, a1 = acc(u1, gr);
  double u2 = u1 + 0.5 * h * w1, w2 = w1 + 0.5 * h * a1, a2 = acc(u2, gr);
  double u3 = u1 + 0.5 * h * w2, w3 = w1 + 0.5 * h * a2, a3 = acc(u3, gr);
  double u4 = u1 + h * w3, w4 = w1 + h * a3, a4 = acc(u4, gr);
  *u = u1 + h / 6.0 * (w1 + 2.0 * w2 + 2.0 * w3 + w4);
  *w = w1 + h / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4);
}

void orc_march_state(double u0, double w0, double h, int32_t k, double gr, double* u,
                     double* w) {
  *u = u0;
  *w = w0;
  for (int32_t i = 0; i < k; ++i) rk4(u, w, h, gr);
}

/* cubic Hermite interpolant on [0, h] of values p0, p1 and slopes m0, m1, at s */
static double herm(double p0, double m0, double p1, double m1, double h, double s) {
  double t = s / h, t2 = t * t, t3 = t2 * t;
  return (2 * t3 - 3 * t2 + 1) * p0 + (t3 - 2 * t2 + t) * h * m0 + (-2 * t3 + 3 * t2) * p1 +
         (t3 - t2) * h * m1;
}

/* its slope d/ds */
static double hermd(double p0, double m0, double p1, double m1, double h, double s) {
  double t = s / h, t2 = t * t;
  return ((6 * t2 - 6 * t) * p0 + (-6 * t2 + 6 * t) * p1) / h + (3 * t2 - 4 * t + 1) * m0 +
         (3 * t2 - 2 * t) * m1;
}

double orc_hermite(double p0, double m0, double p1, double m1, double h, double s) {
  return herm(p0, m0, p1, m1, h, s);
}

/* the smallest root in [0, h] of the Hermite cubic, given p0 >= 0 > p1: split [0, 1] at
 * the roots of the cubic's derivative into monotone pieces, take the first piece whose
 * ends differ in sign, and bisect it */
double orc_hermite_first_root(double p0, double m0, double p1, double m1, double h) {
  /* in t = s / h the slopes scale by h; p(t) = c3 t^3 + c2 t^2 + c1 t + p0 */
  double a = h * m0, b = h * m1;
  double c3 = 2 * p0 + a - 2 * p1 + b, c2 = -3 * p0 - 2 * a + 3 * p1 - b, c1 = a;
  double cuts[4] = {0.0, 1.0, 1.0, 1.0};
  int nc = 1;
  /* derivative 3 c3 t^2 + 2 c2 t + c1 */
  double qa = 3 * c3, qb = 2 * c2, qc = c1;
  double r[2];
  int nr = 0;
  if (fabs(qa) > 1e-300) {
    double disc = qb * qb - 4 * qa * qc;
    if (disc > 0) {
      double sq = sqrt(disc);
      double q = -0.5 * (qb + (qb >= 0 ? sq : -sq));
      r[nr++] = q / qa;
      if (q != 0.0) r[nr++] = qc / q;
    }
  } else if (fabs(qb) > 1e-300) {
    r[nr++] = -qc / qb;
  }
  if (nr == 2 && r[0] > r[1]) {
    double x = r[0];
    r[0] = r[1];
    r[1] = x;
  }
  for (int i = 0; i < nr; ++i)
    if (r[i] > 0.0 && r[i] < 1.0) cuts[nc++] = r[i];
  cuts[nc++] = 1.0;
  for (int i = 0; i + 1 < nc; ++i) {
    double lo = cuts[i], hi = cuts[i + 1];
    double flo = herm(p0, a, p1, b, 1.0, lo), fhi = herm(p0, a, p1, b, 1.0, hi);
    if (flo == 0.0) return lo * h;
    if ((flo > 0) == (fhi > 0) && fhi != 0.0) continue;
    for (int it = 0; it < 200 && hi - lo > 1e-17; ++it) {
      double mid = 0.5 * (lo + hi);
      double fm = herm(p0, a, p1, b, 1.0, mid);
      if ((fm > 0) == (flo > 0)) {
        lo = mid;
        flo = fm;
      } else {
        hi = mid;
      }
    }
    return 0.5 * (lo + hi) * h;
  }
  return h; /* p1 < 0 guarantees a sign change: not reached */
}

int orc_march_ray(double u_c, double delta, double alpha, double u_ic, double u_oc,
                  int32_t nsteps, double gr, orc_ray* o) {
  memset(o, 0, sizeof(*o));
  if (nsteps < 1) return 1;
  double sd = sin(delta), cd = cos(delta);
  double u = u_c, w;
  if (sd <= 1e-6 * fabs(cd)) {
    /* within 1e-6 of the radius (|cot delta| >= 1e6) the beam moves along r only: a fixed
     * step in phi cannot follow its slope, and radial beams are not deflected */
    if (cd > 0.0) {
      o->delta_prime = delta;
    } else {
      o->captured = 1;
      o->delta_prime = INFINITY;
    }
    return 0;
  }
  w = -u_c * cd / sd;
  const double h = 2.0 * M_PI / nsteps;
  const int inward = w > 0.0; /* an apsis (largest u) can lie ahead */
  int m = 0;
  double phi_d = alpha;
  if (!(phi_d > 0.0)) {
    m = 1;
    phi_d = alpha + M_PI;
  }
  double phi = 0.0;
  for (int32_t n = 0; n < nsteps; ++n) {
    double un = u, wn = w;
    rk4(&un, &wn, h, gr);
    double end = h; /* the part of the step the ray really travels */
    int escaped = un < 0.0;
    if (escaped) end = orc_hermite_first_root(u, w, un, wn, h);
    while (phi_d <= phi + end) {
      double ud = herm(u, w, un, wn, h, phi_d - phi);
      if (ud >= u_oc && ud <= u_ic && o->n_cross < 4) {
        o->u_cross[o->n_cross] = ud;
        o->phi_cross[o->n_cross] = phi_d;
        /* after the apsis: the beam started inward and u now decreases */
        o->branch[o->n_cross] = inward && hermd(u, w, un, wn, h, phi_d - phi) < 0.0;
        o->n_cross++;
      }
      ++m;
      phi_d = alpha + m * M_PI;
    }
    o->steps = n + 1;
    if (escaped) {
      o->delta_prime = phi + end;
      return 0;
    }
    phi += h;
    u = un;
    w = wn;
    if (u >= 1.0) {
      o->captured = 1;
      o->delta_prime = INFINITY;
      return 0;
    }
  }
  o->captured = 1;
  o->unfinished = 1;
  o->delta_prime = INFINITY;
  return 0;
}
