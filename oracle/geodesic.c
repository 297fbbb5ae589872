/*
 * Exact-mode ray tracing: adaptive integration of the photon orbit equation.
 * TEST INFRASTRUCTURE ONLY (see bh_oracle.h).
 *
 * Orbit equation (Section 3.3, eq. rayequation), in the ray's own plane with u = 1/r:
 *     (du/dphi)^2 = e^2 - u^2 (1 - u)   =>   u'' = 3/2 u^2 - u.
 * The beam starts at the camera (phi = 0) with u = 1/p^r and du/dphi = -u cot(delta)
 * (Algorithm 1, TraceRay, first line).  It escapes when u returns to 0 while decreasing
 * (escape angle delta' = phi at that point, Section 3.3.2 "Escape angle"), is captured
 * when u reaches 1 (the horizon), and meets the disc plane at phi = alpha + m pi
 * (Section 3.3.3 "Intersections"); a crossing counts when u_oc <= u <= u_ic.
 *
 * Integrator: Dormand-Prince 5(4) with local error control (rtol 1e-12, atol 1e-14 e);
 * disc-plane angles are hit exactly by clipping the step; the escape point is located by
 * Newton iteration on the step length.  gr = 0 drops the 3/2 u^2 term (flat space), which
 * reduces rays to straight lines u = u_c sin(delta - phi) / sin(delta).
 *
 * Coordinate time rides along as a quadrature, dt/dphi = e / (u^2 (1 - u)) (the motion
 * constants of Section 3.1; Algorithm 1 Precompute integrates the same rate), so each
 * crossing also carries the time the light takes from it to the camera.  In flat space
 * the rate is e / u^2, the distance travelled along the straight line.
 */
#include <math.h>
#include <string.h>

#include "bh_oracle.h"
#include "oracle_internal.h"

/* Dormand & Prince (1980) RK5(4)7M coefficients */
static const double A21 = 1.0 / 5.0;
static const double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
static const double A41 = 44.0 / 45.0, A42 = -56.0 / 15.0, A43 = 32.0 / 9.0;
static const double A51 = 19372.0 / 6561.0, A52 = -25360.0 / 2187.0, A53 = 64448.0 / 6561.0,
                    A54 = -212.0 / 729.0;
static const double A61 = 9017.0 / 3168.0, A62 = -355.0 / 33.0, A63 = 46732.0 / 5247.0,
                    A64 = 49.0 / 176.0, A65 = -5103.0 / 18656.0;
static const double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0,
                    B5 = -2187.0 / 6784.0, B6 = 11.0 / 84.0;
static const double E1 = 35.0 / 384.0 - 5179.0 / 57600.0, E3 = 500.0 / 1113.0 - 7571.0 / 16695.0,
                    E4 = 125.0 / 192.0 - 393.0 / 640.0, E5 = -2187.0 / 6784.0 + 92097.0 / 339200.0,
                    E6 = 11.0 / 84.0 - 187.0 / 2100.0, E7 = -1.0 / 40.0;

static inline double accel(double u, double gr) { return gr * 1.5 * u * u - u; }
static inline double trate(double u, double e, double gr) {
  return e / (u * u * (1.0 - gr * u));
}

/* one step of size h from (u, w); returns the 5th-order state and the error estimate,
 * and the increment of the coordinate time (5th order) in *dt */
static void dopri(double u, double w, double h, double gr, double e, double* u5, double* w5,
                  double* eu, double* ew, double* dt) {
  double k1u = w, k1w = accel(u, gr);
  double u2 = u + h * (A21 * k1u), w2 = w + h * (A21 * k1w);
  double k2u = w2, k2w = accel(u2, gr);
  double u3 = u + h * (A31 * k1u + A32 * k2u), w3 = w + h * (A31 * k1w + A32 * k2w);
  double k3u = w3, k3w = accel(u3, gr);
  double u4 = u + h * (A41 * k1u + A42 * k2u + A43 * k3u);
  double w4 = w + h * (A41 * k1w + A42 * k2w + A43 * k3w);
  double k4u = w4, k4w = accel(u4, gr);
  double uu5 = u + h * (A51 * k1u + A52 * k2u + A53 * k3u + A54 * k4u);
  double ww5 = w + h * (A51 * k1w + A52 * k2w + A53 * k3w + A54 * k4w);
  double k5u = ww5, k5w = accel(uu5, gr);
  double u6 = u + h * (A61 * k1u + A62 * k2u + A63 * k3u + A64 * k4u + A65 * k5u);
  double w6 = w + h * (A61 * k1w + A62 * k2w + A63 * k3w + A64 * k4w + A65 * k5w);
  double k6u = w6, k6w = accel(u6, gr);
  double un = u + h * (B1 * k1u + B3 * k3u + B4 * k4u + B5 * k5u + B6 * k6u);
  double wn = w + h * (B1 * k1w + B3 * k3w + B4 * k4w + B5 * k5w + B6 * k6w);
  double k7u = wn, k7w = accel(un, gr);
  if (dt)
    *dt = h * (B1 * trate(u, e, gr) + B3 * trate(u3, e, gr) + B4 * trate(u4, e, gr) +
               B5 * trate(uu5, e, gr) + B6 * trate(u6, e, gr));
  *u5 = un;
  *w5 = wn;
  *eu = h * (E1 * k1u + E3 * k3u + E4 * k4u + E5 * k5u + E6 * k6u + E7 * k7u);
  *ew = h * (E1 * k1w + E3 * k3w + E4 * k4w + E5 * k5w + E6 * k6w + E7 * k7w);
}

#define RTOL 1e-12
#define ATOL_REL 1e-14 /* absolute tolerance relative to the ray's scale e */

void orc_integrate_ray(double u0, double w0, double alpha, double u_ic, double u_oc,
                       double gr, orc_ray* o) {
  memset(o, 0, sizeof(*o));
  double u = u0, w = w0, phi = 0.0, t = 0.0;
  double h = 1e-3 / (1.0 + fabs(w0));
  /* u and du/dphi are bounded by the invariant e = sqrt(w^2 + u^2 (1-u)) away from the
   * horizon, so tolerances scale with it (weak-field rays far away have tiny u) */
  double escale = sqrt(w0 * w0 + u0 * u0 * fabs(1.0 - gr * u0));
  const double e_inv = escale;  /* the ray's invariant e, rate of the coordinate time */
  if (!(escale > 0.0)) escale = 1.0;
  const double atol = ATOL_REL * fmin(escale, 1.0);
  int passed_apsis = 0;
  /* disc-plane angles alpha + m pi strictly ahead of the camera */
  int m = 0;
  double phi_d = alpha;
  if (!(phi_d > 0.0)) {
    m = 1;
    phi_d = alpha + M_PI;
  }
  const double phi_max = 200.0 * M_PI;
  for (;;) {
    if (phi > phi_max) {
      o->captured = 1;
      o->delta_prime = INFINITY;
      return;
    }
    double hh = h;
    int hit_disc = 0;
    if (phi + hh >= phi_d) {
      hh = phi_d - phi;
      hit_disc = 1;
    }
    double un, wn, eu, ew, dtn;
    dopri(u, w, hh, gr, e_inv, &un, &wn, &eu, &ew, &dtn);
    double su = atol + RTOL * fmax(fabs(u), fabs(un));
    double sw = atol + RTOL * fmax(fabs(w), fabs(wn));
    double err = fmax(fabs(eu) / su, fabs(ew) / sw);
    double fac = err > 0.0 ? 0.9 * pow(err, -0.2) : 5.0;
    if (fac > 5.0) fac = 5.0;
    if (fac < 0.2) fac = 0.2;
    if (err > 1.0) {
      h = hh * fac;
      continue;
    }
    if (un < 0.0) {
      /* escaped inside this step: solve u(phi + s) = 0 for the step length s */
      double s = hh * u / (u - un);
      for (int it = 0; it < 60; ++it) {
        double us, ws, e1, e2;
        dopri(u, w, s, gr, e_inv, &us, &ws, &e1, &e2, NULL);
        double ds = us / ws;
        s -= ds;
        if (fabs(ds) < 1e-16 * (1.0 + s)) break;
      }
      o->delta_prime = phi + s;
      o->captured = 0;
      o->steps++;
      return;
    }
    phi = hit_disc ? phi_d : phi + hh;
    if (w >= 0.0 && wn < 0.0) passed_apsis = 1;
    u = un;
    w = wn;
    t += dtn;
    o->steps++;
    if (hit_disc) {
      if (u >= u_oc && u <= u_ic && o->n_cross < 4) {
        o->u_cross[o->n_cross] = u;
        o->phi_cross[o->n_cross] = phi;
        o->branch[o->n_cross] = passed_apsis;
        o->t_cross[o->n_cross] = t;
        o->n_cross++;
      }
      ++m;
      phi_d = alpha + m * M_PI;
    }
    if (u >= 1.0) {
      o->captured = 1;
      o->delta_prime = INFINITY;
      return;
    }
    h = hh * fac;
  }
}

int orc_trace_exact(double u_c, double delta, double alpha, double u_ic, double u_oc,
                    double gr, orc_ray* o) {
  double sd = sin(delta), cd = cos(delta);
  if (sd < 1e-12) {
    /* radial beam: no rotation of the ray plane is defined; outward escapes undeflected */
    memset(o, 0, sizeof(*o));
    if (cd > 0.0) {
      o->delta_prime = delta;
    } else {
      o->captured = 1;
      o->delta_prime = INFINITY;
    }
    return 0;
  }
  orc_integrate_ray(u_c, -u_c * cd / sd, alpha, u_ic, u_oc, gr, o);
  return 0;
}

/* Apsis of a ray with e^2 < mu (Section 3.3.1, eq. uapsis). */
double orc_apsis(double e2) {
  return 1.0 / 3.0 + 2.0 / 3.0 * sin(asin(2.0 * e2 / ORC_MU - 1.0) / 3.0);
}

/* Total deflection of a ray coming from infinity with inverse impact parameter e:
 * integrate from u = 0, du/dphi = e until it leaves again; deflection = phi_total - pi. */
double orc_deflection(double e) {
  orc_ray r;
  orc_integrate_ray(0.0, e, 1e300, 0.0, 1.0, 1.0, &r);
  if (r.captured) return INFINITY;
  return r.delta_prime - M_PI;
}

/* u at rotated angle phi along the ray that starts at (u0, w0); NaN if it escapes or is
 * captured first.  Uses the same integrator with the "disc" event placed at phi. */
double orc_u_at_phi(double u0, double w0, double phi, double gr) {
  orc_ray r;
  orc_integrate_ray(u0, w0, phi, INFINITY, -INFINITY, gr, &r);
  if (r.n_cross < 1) return NAN;
  return r.u_cross[0];
}
