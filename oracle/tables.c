/*
 * Table mode: deflection table D(e, u) and intersection table U(e, phi) filled by
 * quadrature of the first integral at the texel centres, and the paper's TraceRay
 * procedure reading them.  TEST INFRASTRUCTURE ONLY (see bh_oracle.h).
 *
 * What the tables hold (Section 3.3.2 "Escape angle", Section 3.3.3 "Intersections",
 * Algorithm 1 Precompute), for a ray coming from infinity with inverse impact parameter e
 * (phi measured from its start at infinity):
 *   phi(u)   = integral_0^u dv / sqrt(e^2 - v^2 (1 - v))      (incoming branch)
 *   D(e, u)  = phi(u) - atan2(u, du/dphi)                        (deflection so far)
 *   U(e, phi)= u on that ray, for 0 <= phi < pi; past the apsis by the reflection
 *              phi -> 2 phi_a - phi (Section 3.3.1); u = 1 once the ray has fallen in.
 *
 * Texel mapping (Appendix A).  Reading used here: the unit-square coordinates 0 and 1
 * are the first and last texel centres, texel k of N sits at k / (N - 1), so that the
 * apsis row (y = 1) and the e -> 0 / e -> infinity columns are stored exactly.
 *   D, e^2 < mu : x = 1/2 - sqrt(-log(1 - e^2/mu) / 50),  y = 1 - sqrt(1 - u/u_a)
 *   D, e^2 > mu : x = 1/2 + sqrt(-log(1 - mu/e^2) / 50),
 *                 y = (sqrt(2/3) + sign(u - 2/3) sqrt|u - 2/3|) / (sqrt(2/3) + sqrt(1/3))
 *   U           : x = 1 / (1 + 6 e^2),  y = (phi / 3) (1 + 6 e^3) / (1 + e^2)
 * Reading: the two halves of D meet at x = 1/2 where e -> 0 and e -> infinity; bilinear
 * interpolation never mixes the halves (clamped within each half).
 *
 * Layout: D[j * d_n + i] (row j: u coordinate, column i: e coordinate),
 *         U[j * u_ne + i] (row j: phi coordinate, column i: e coordinate).
 *
 * Time channels (Algorithm 1 Precompute stores t beside D and U, with dt/dphi =
 * e / (u^2 - u^3), Section 3.3.3 "Intersections").  On a ray from infinity t diverges, and
 * only differences along one ray are used.  With w = |du/dphi| = sqrt(e^2 - u^2 (1 - u)):
 *   dt/du = e / (u^2 (1 - u) w) = 1 / (w (e + w)) + S'(u),  S(u) = ln(u / (1 - u)) - 1/u,
 * (because 1/u^2 + 1/u + 1/(1 - u) = 1 / (u^2 (1 - u)) and e - w = u^2 (1 - u) / (e + w)),
 * so t = tau + S(u) + const with the finite regularised time
 *   tau(u) = integral_0^u dv / (w (e + w))                      (incoming branch).
 * tau grows like 1/e for small e (tau ~ tan(phi/2) / e on a nearly straight ray), so the
 * tables hold e tau, which stays finite on the e -> 0 edge of U and interpolates well
 * (reading: the paper stores t itself).  Dt and Ut hold e tau at the same texel centres
 * as D and U.  Past the apsis (U only), t = 2 t_a - t_in(u) gives
 * tau = 2 tau_a + 2 S(u_a) - tau_in(u) - 2 S(u).  On the e = 0 column of U the limit is
 * tan(phi/2) before the apsis (phi = pi/2) and 2/sin(phi) - cot(phi/2) after it.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#include "bh_oracle.h"
#include "oracle_internal.h"

#define QTOL 1e-13

/* roots of v^3 - v^2 + e^2 = 0 for e^2 < mu: u_a (smallest positive, paper's closed form)
 * and the other two from the sum and the product of the roots */
static void cubic_roots(double e2, double* ua, double* u2, double* u3) {
  *ua = orc_apsis(e2);
  double s = 1.0 - *ua;         /* u2 + u3 */
  double p = -e2 / *ua;         /* u2 * u3 */
  double d = sqrt(s * s - 4.0 * p);
  *u2 = 0.5 * (s + d);
  *u3 = 0.5 * (s - d);
}

/* ---- incoming branch for e^2 < mu, in the variable s = sqrt(1 - u/u_a) --------------- */
typedef struct { double ua, u2, u3; } lo_ctx;

static double lo_integrand(double s, void* c) {
  const lo_ctx* k = (const lo_ctx*)c;
  double v = k->ua * (1.0 - s * s);
  return 2.0 * sqrt(k->ua) / sqrt((k->u2 - v) * (v - k->u3));
}

/* phi at s (s = 1 at infinity, s = 0 at the apsis) */
static double lo_phi(const lo_ctx* k, double s) {
  return orc_integrate(lo_integrand, (void*)k, s, 1.0, QTOL);
}

/* sqrt(e^2 - u^2 (1-u)) written with the factorisation, accurate near the apsis */
static double lo_udot(const lo_ctx* k, double s) {
  double v = k->ua * (1.0 - s * s);
  return sqrt(k->ua) * s * sqrt((k->u2 - v) * (v - k->u3));
}

/* ---- incoming branch for e^2 >= mu, in u directly ------------------------------------- */
typedef struct { double e2; } hi_ctx;

static double hi_integrand(double v, void* c) {
  double e2 = ((const hi_ctx*)c)->e2;
  return 1.0 / sqrt(e2 - v * v * (1.0 - v));
}

static double hi_phi_between(double e2, double a, double b) {
  hi_ctx k = {e2};
  /* split at the photon sphere, where the integrand peaks when e^2 is close to mu */
  const double ps = 2.0 / 3.0;
  if (a < ps && b > ps)
    return orc_integrate(hi_integrand, &k, a, ps, QTOL) +
           orc_integrate(hi_integrand, &k, ps, b, QTOL);
  return orc_integrate(hi_integrand, &k, a, b, QTOL);
}

/* ---- regularised time tau ----------------------------------------------------------------- */
typedef struct { lo_ctx k; double e; } lo_tctx;

static double lo_tau_integrand(double s, void* c) {
  const lo_tctx* q = (const lo_tctx*)c;
  return lo_integrand(s, (void*)&q->k) / (q->e + lo_udot(&q->k, s));
}

/* tau between s and s_prev (s < s_prev) on the incoming branch, e^2 < mu */
static double lo_tau_between(const lo_tctx* q, double s, double s_prev) {
  return orc_integrate(lo_tau_integrand, (void*)q, s, s_prev, QTOL);
}

static double hi_tau_integrand(double v, void* c) {
  double e2 = ((const hi_ctx*)c)->e2;
  double w = sqrt(e2 - v * v * (1.0 - v));
  return 1.0 / (w * (sqrt(e2) + w));
}

static double hi_tau_between(double e2, double a, double b) {
  hi_ctx k = {e2};
  const double ps = 2.0 / 3.0;
  if (a < ps && b > ps)
    return orc_integrate(hi_tau_integrand, &k, a, ps, QTOL) +
           orc_integrate(hi_tau_integrand, &k, ps, b, QTOL);
  return orc_integrate(hi_tau_integrand, &k, a, b, QTOL);
}

/* singular part of the time along a ray: t = tau + S(u) + const */
double orc_time_singular(double u) { return log(u / (1.0 - u)) - 1.0 / u; }

/* tau(u) on the incoming branch of the ray with invariant e^2 (0 <= u, below the apsis
 * when e^2 < mu) */
double orc_tau_in(double e2, double u) {
  if (!(u > 0.0)) return 0.0;
  if (e2 < ORC_MU) {
    lo_tctx q;
    cubic_roots(e2, &q.k.ua, &q.k.u2, &q.k.u3);
    q.e = sqrt(e2);
    double r = 1.0 - u / q.k.ua;
    double s = r > 0.0 ? sqrt(r) : 0.0;
    return lo_tau_between(&q, s, 1.0);
  }
  return hi_tau_between(e2, 0.0, u);
}

/* ---- texel centres ---------------------------------------------------------------------- */
static double d_col_e2(int32_t n, int32_t i) {
  double x = (double)i / (n - 1);
  if (i < n / 2) {
    double a = 0.5 - x;
    return -ORC_MU * expm1(-50.0 * a * a);
  }
  double a = x - 0.5;
  return ORC_MU / (-expm1(-50.0 * a * a));
}

static double d_row_u_hi(int32_t n, int32_t j) {
  double y = (double)j / (n - 1);
  double z = y * (sqrt(2.0 / 3.0) + sqrt(1.0 / 3.0)) - sqrt(2.0 / 3.0);
  return 2.0 / 3.0 + (z >= 0.0 ? z * z : -z * z);
}

static double u_col_e2(int32_t ne, int32_t i) {
  double x = (double)i / (ne - 1);
  return (1.0 / x - 1.0) / 6.0; /* +inf at i = 0 */
}

/* one D column */
static void fill_D_column(int32_t n, int32_t i, double* D) {
  double e2 = d_col_e2(n, i);
  if (i < n / 2) {
    lo_ctx k;
    cubic_roots(e2, &k.ua, &k.u2, &k.u3);
    double phi = 0.0, s_prev = 1.0;
    for (int32_t j = 0; j < n; ++j) {
      double y = (double)j / (n - 1);
      double s = 1.0 - y; /* sqrt(1 - u_j/u_a) for u_j = u_a (1 - (1-y)^2) */
      phi += orc_integrate(lo_integrand, &k, s, s_prev, QTOL);
      s_prev = s;
      double u = k.ua * (1.0 - s * s);
      D[(size_t)j * n + i] = phi - atan2(u, lo_udot(&k, s));
    }
  } else {
    double phi = 0.0, u_prev = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      double u = d_row_u_hi(n, j);
      phi += hi_phi_between(e2, u_prev, u);
      u_prev = u;
      D[(size_t)j * n + i] = phi - atan2(u, sqrt(e2 - u * u * (1.0 - u)));
    }
  }
}

/* one column of Dt (tau at the D texel centres) */
static void fill_Dt_column(int32_t n, int32_t i, double* Dt) {
  double e2 = d_col_e2(n, i);
  if (i < n / 2) {
    lo_tctx q;
    cubic_roots(e2, &q.k.ua, &q.k.u2, &q.k.u3);
    q.e = sqrt(e2);
    double tau = 0.0, s_prev = 1.0;
    for (int32_t j = 0; j < n; ++j) {
      double s = 1.0 - (double)j / (n - 1);
      tau += lo_tau_between(&q, s, s_prev);
      s_prev = s;
      Dt[(size_t)j * n + i] = q.e * tau;
    }
  } else {
    double tau = 0.0, u_prev = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      double u = d_row_u_hi(n, j); /* the last row is the horizon u = 1: tau stays finite */
      tau += hi_tau_between(e2, u_prev, u);
      u_prev = u;
      Dt[(size_t)j * n + i] = sqrt(e2) * tau;
    }
  }
}

/* u on a ray from infinity at rotated angle phi_t (0 <= phi_t < pi) */
static double u_at_phi(double e2, double phi_t) {
  if (e2 < ORC_MU) {
    lo_ctx k;
    cubic_roots(e2, &k.ua, &k.u2, &k.u3);
    double phi_a = lo_phi(&k, 0.0);
    if (phi_t > phi_a) phi_t = 2.0 * phi_a - phi_t; /* reflection about the apsis */
    if (phi_t <= 0.0) return 0.0;
    double lo = 0.0, hi = 1.0; /* phi decreases with s */
    for (int it = 0; it < 64; ++it) {
      double mid = 0.5 * (lo + hi);
      if (lo_phi(&k, mid) > phi_t) lo = mid; else hi = mid;
    }
    double s = 0.5 * (lo + hi);
    return k.ua * (1.0 - s * s);
  }
  double phi_fall = hi_phi_between(e2, 0.0, 1.0);
  if (phi_t >= phi_fall) return 1.0;
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 64; ++it) {
    double mid = 0.5 * (lo + hi);
    if (hi_phi_between(e2, 0.0, mid) < phi_t) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* tau at the U texel (i, j): on the incoming branch tau_in(u(phi)); past the apsis the
 * reflection formula; 0 on the e -> infinity and e = 0 columns and after a fall-in */
static double ut_entry(int32_t ne, int32_t nphi, int32_t i, int32_t j) {
  double y = (double)j / (nphi - 1);
  if (i == 0) return 0.0;       /* e -> infinity: e tau ~ u / (2 e) -> 0 */
  if (i == ne - 1) {            /* e -> 0: phi = 3 y */
    double phi = 3.0 * y;
    if (phi <= 0.5 * M_PI) return tan(0.5 * phi);
    return 2.0 / sin(phi) - 1.0 / tan(0.5 * phi);
  }
  double e2 = u_col_e2(ne, i);
  double e = sqrt(e2);
  double phi = 3.0 * y * (1.0 + e2) / (1.0 + 6.0 * e2 * e);
  double u = u_at_phi(e2, phi);
  if (e2 < ORC_MU) {
    lo_ctx k;
    cubic_roots(e2, &k.ua, &k.u2, &k.u3);
    double phi_a = lo_phi(&k, 0.0);
    if (phi > phi_a) {
      double tau_a = orc_tau_in(e2, k.ua);
      return e * (2.0 * tau_a + 2.0 * orc_time_singular(k.ua) - orc_tau_in(e2, u) -
                  2.0 * orc_time_singular(u));
    }
    return e * orc_tau_in(e2, u);
  }
  if (u >= 1.0) return 0.0;
  return e * orc_tau_in(e2, u);
}

static double u_entry(int32_t ne, int32_t nphi, int32_t i, int32_t j, double* e2o,
                      double* phio) {
  double y = (double)j / (nphi - 1);
  if (i == 0) { /* e -> infinity: u = e phi + O(1/e^2) along phi = y / (2e) */
    *e2o = INFINITY;
    *phio = 0.0;
    return 0.5 * y;
  }
  double e2 = u_col_e2(ne, i);
  double e = sqrt(e2);
  double phi = 3.0 * y * (1.0 + e2) / (1.0 + 6.0 * e2 * e);
  *e2o = e2;
  *phio = phi;
  if (i == ne - 1) return 0.0; /* e = 0: the ray stays at infinity */
  return u_at_phi(e2, phi);
}

typedef struct {
  int32_t d_n, u_ne, u_nphi;
  double *D, *U;
  int next;
  pthread_mutex_t mu;
  int time;  /* fill tau (Dt, Ut) instead of D, U */
} tab_job;

static void* tab_worker(void* p) {
  tab_job* jb = (tab_job*)p;
  int total = (jb->D ? jb->d_n : 0) + (jb->U ? jb->u_ne : 0);
  for (;;) {
    pthread_mutex_lock(&jb->mu);
    int c = jb->next++;
    pthread_mutex_unlock(&jb->mu);
    if (c >= total) break;
    if (jb->D && c < jb->d_n) {
      if (jb->time)
        fill_Dt_column(jb->d_n, c, jb->D);
      else
        fill_D_column(jb->d_n, c, jb->D);
    } else {
      int i = c - (jb->D ? jb->d_n : 0);
      for (int32_t j = 0; j < jb->u_nphi; ++j) {
        double e2, phi;
        jb->U[(size_t)j * jb->u_ne + i] = jb->time ? ut_entry(jb->u_ne, jb->u_nphi, i, j)
                                                   : u_entry(jb->u_ne, jb->u_nphi, i, j, &e2, &phi);
      }
    }
  }
  return NULL;
}

int orc_tables(int32_t d_n, int32_t u_ne, int32_t u_nphi, double* D, double* U, int nthreads) {
  if ((D && (d_n < 4 || d_n % 2)) || (U && (u_ne < 2 || u_nphi < 2))) return 1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  tab_job jb = {d_n, u_ne, u_nphi, D, U, 0, PTHREAD_MUTEX_INITIALIZER, 0};
  pthread_t th[256];
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, tab_worker, &jb);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  return 0;
}

int orc_tables_time(int32_t d_n, int32_t u_ne, int32_t u_nphi, double* Dt, double* Ut,
                    int nthreads) {
  if ((Dt && (d_n < 4 || d_n % 2)) || (Ut && (u_ne < 2 || u_nphi < 2))) return 1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  tab_job jb = {d_n, u_ne, u_nphi, Dt, Ut, 0, PTHREAD_MUTEX_INITIALIZER, 1};
  pthread_t th[256];
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, tab_worker, &jb);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  return 0;
}

int orc_table_entry_D(int32_t n, int32_t i, int32_t j, double* value, double* e2o, double* uo) {
  if (n < 4 || n % 2 || i < 0 || i >= n || j < 0 || j >= n) return 1;
  double* col = (double*)calloc((size_t)n * n, sizeof(double));
  if (!col) return 2;
  fill_D_column(n, i, col);
  *value = col[(size_t)j * n + i];
  free(col);
  double e2 = d_col_e2(n, i);
  *e2o = e2;
  if (i < n / 2) {
    double y = (double)j / (n - 1);
    *uo = orc_apsis(e2) * (1.0 - (1.0 - y) * (1.0 - y));
  } else {
    *uo = d_row_u_hi(n, j);
  }
  return 0;
}

int orc_table_entry_U(int32_t ne, int32_t nphi, int32_t i, int32_t j, double* value,
                      double* e2o, double* phio) {
  if (ne < 2 || nphi < 2 || i < 0 || i >= ne || j < 0 || j >= nphi) return 1;
  *value = u_entry(ne, nphi, i, j, e2o, phio);
  return 0;
}

/* ---- TraceRay (Algorithm 1) --------------------------------------------------------- */

static double bilinear(const double* T, int32_t nx, int32_t ny, int32_t lo, int32_t hi,
                       double x, double y) {
  double tx = x * (nx - 1), ty = y * (ny - 1);
  if (tx < lo) tx = lo;
  if (tx > hi) tx = hi;
  if (ty < 0) ty = 0;
  if (ty > ny - 1) ty = ny - 1;
  int32_t i0 = (int32_t)floor(tx), j0 = (int32_t)floor(ty);
  if (i0 > hi - 1) i0 = hi - 1;
  if (j0 > ny - 2) j0 = ny - 2;
  double fx = tx - i0, fy = ty - j0;
  const double* r0 = T + (size_t)j0 * nx;
  const double* r1 = r0 + nx;
  return (1 - fy) * ((1 - fx) * r0[i0] + fx * r0[i0 + 1]) +
         fy * ((1 - fx) * r1[i0] + fx * r1[i0 + 1]);
}

/* D(e, u) through the Appendix A mapping; ua is used for e^2 < mu */
static double lookup_D(const double* D, int32_t n, double e2, double u, double ua) {
  double x, y;
  if (e2 < ORC_MU) {
    x = 0.5 - sqrt(-log1p(-e2 / ORC_MU) / 50.0);
    double q = u / ua;
    if (q > 1.0) q = 1.0;
    y = 1.0 - sqrt(1.0 - q);
    return bilinear(D, n, n, 0, n / 2 - 1, x, y);
  }
  x = 0.5 + sqrt(-log1p(-ORC_MU / e2) / 50.0);
  double dz = u - 2.0 / 3.0;
  y = (sqrt(2.0 / 3.0) + (dz >= 0 ? sqrt(dz) : -sqrt(-dz))) / (sqrt(2.0 / 3.0) + sqrt(1.0 / 3.0));
  return bilinear(D, n, n, n / 2, n - 1, x, y);
}

static double lookup_U(const double* U, int32_t ne, int32_t nphi, double e2, double phi) {
  double e = sqrt(e2);
  double x = 1.0 / (1.0 + 6.0 * e2);
  double y = phi / 3.0 * (1.0 + 6.0 * e2 * e) / (1.0 + e2);
  return bilinear(U, ne, nphi, 0, ne - 1, x, y);
}

static double fmod_floor(double a, double m) { return a - m * floor(a / m); }

/* TraceRay with the time channels (Dt, Ut may be NULL: no times).  The retarded time of a
 * crossing is the coordinate time the light takes from the crossing to the camera:
 * crossing 0: s (t_0 - t), crossing 1: 2 t_a - t - t_1 (Algorithm 1), with t = tau + S(u)
 * read from the tables at the camera (t), the apsis (t_a) and the crossings. */
int orc_trace_table_t(const double* D, const double* Dt, int32_t n, const double* U,
                      const double* Ut, int32_t ne, int32_t nphi, double u, double delta,
                      double alpha, double u_ic, double u_oc, orc_ray* o) {
  memset(o, 0, sizeof(*o));
  double udot = -u * cos(delta) / sin(delta);
  double e2 = udot * udot + u * u * (1.0 - u);
  if (e2 < ORC_MU && u > 2.0 / 3.0) {
    o->captured = 1;
    o->delta_prime = INFINITY;
    return 0;
  }
  int s = udot >= 0.0 ? 1 : -1;
  double ua = e2 < ORC_MU ? orc_apsis(e2) : 0.0;
  double Dl = lookup_D(D, n, e2, u, ua);
  double Da = 0.0, phi_a = INFINITY;
  if (e2 < ORC_MU) {
    Da = lookup_D(D, n, e2, ua, ua);
    phi_a = Da + M_PI / 2.0;
  }
  /* times at the camera and the apsis on the incoming branch */
  double t_cam = 0.0, t_a = 0.0;
  const double ie = 1.0 / sqrt(e2);  /* the tables hold e tau */
  if (Dt) {
    t_cam = lookup_D(Dt, n, e2, u, ua) * ie + orc_time_singular(u);
    if (e2 < ORC_MU) t_a = lookup_D(Dt, n, e2, ua, ua) * ie + orc_time_singular(ua);
  }
  double phi = Dl + (s == 1 ? M_PI - delta : delta) + s * alpha;
  double phi0 = fmod_floor(phi, M_PI);
  double u0 = lookup_U(U, ne, nphi, e2, phi0);
  int sg = (u0 > u) - (u0 < u);
  if (phi0 < phi_a && u_oc <= u0 && u0 <= u_ic && sg == s) {
    o->u_cross[o->n_cross] = u0;
    o->phi_cross[o->n_cross] = alpha + phi - phi0;
    o->branch[o->n_cross] = 0;
    if (Ut) o->t_cross[o->n_cross] = s * (lookup_U(Ut, ne, nphi, e2, phi0) * ie +
                                          orc_time_singular(u0) - t_cam);
    o->n_cross++;
  }
  if (e2 < ORC_MU && s == 1) {
    phi = 2.0 * phi_a - phi;
    double phi1 = fmod_floor(phi, M_PI);
    double u1 = lookup_U(U, ne, nphi, e2, phi1);
    if (phi1 < phi_a && u_oc <= u1 && u1 <= u_ic) {
      o->u_cross[o->n_cross] = u1;
      o->phi_cross[o->n_cross] = alpha + phi - phi1;
      o->branch[o->n_cross] = 1;
      if (Ut) o->t_cross[o->n_cross] = 2.0 * t_a - t_cam -
                                       (lookup_U(Ut, ne, nphi, e2, phi1) * ie +
                                        orc_time_singular(u1));
      o->n_cross++;
    }
  }
  double Dl2 = Dl;
  if (udot > 0.0) {
    if (e2 < ORC_MU) {
      Dl2 = 2.0 * Da - Dl;
    } else {
      o->captured = 1;
      o->delta_prime = INFINITY;
      return 0;
    }
  }
  o->delta_prime = delta + Dl2;
  return 0;
}

int orc_trace_table(const double* D, int32_t n, const double* U, int32_t ne, int32_t nphi,
                    double u, double delta, double alpha, double u_ic, double u_oc,
                    orc_ray* o) {
  return orc_trace_table_t(D, NULL, n, U, NULL, ne, nphi, u, delta, alpha, u_ic, u_oc, o);
}
