/*
 * Animated accretion disc: density of procedural particles on precessing quasi-circular
 * orbits (Appendix B), evaluated at a beam's disc crossing at its retarded time
 * (Section 3.3.3 "Intersections", Algorithm 1).  TEST INFRASTRUCTURE ONLY (see bh_oracle.h).
 *
 * Orbit of a massive particle (Appendix B): with u1 <= u2 <= 1/3 the two largest distances'
 * inverses and u3 = 1 - u1 - u2 (the three roots of the orbit cubic sum to 1),
 *   u(phi) = u1 + (u2 - u1) sn^2(phi sqrt(u3 - u1) / 2, kappa),
 *   kappa = sqrt((u2 - u1) / (u3 - u1)),
 * approximated for quasi-circular orbits by replacing sn(x) with sin(pi x / (2K)):
 *   u(t) = u1 + (u2 - u1) sin^2(pi / (4K) phi(t) sqrt(u3 - u1)),
 *   phi(t) = sqrt(ubar^3 / 2) t + phi0,  ubar = (u1 + u2) / 2,
 * K = K(kappa) the complete elliptic integral of the first kind.
 * A linear particle is the set of points a in [0, 2 pi) with phi_a(t) = a + phi(t).  For a
 * hit point h = (h^t, h^r, h^phi): a = (h^phi - phi(h^t)) mod 2 pi, and the "distance" to
 * the particle centre (a = pi) is d^2 = (a/pi - 1)^2 + (h^r - 1/u_a(h^t))^2.
 * Reading (the paper only asks for a smoothly decreasing function of d): each particle
 * adds f(d) = (1 - d^2)^2 for d < 1, 0 beyond; the disc density is the sum over particles.
 *
 * Particles are given as (r_peri, r_apo, phi0) triples: u2 = 1/r_peri, u1 = 1/r_apo.
 */
#include <math.h>

#include "bh_oracle.h"
#include "oracle_internal.h"

static double k_integrand(double th, void* c) {
  double k = *(const double*)c;
  double s = sin(th);
  return 1.0 / sqrt(1.0 - k * k * s * s);
}

/* K(kappa) = integral_0^1 dx / sqrt((1 - x^2)(1 - kappa^2 x^2)), written with x = sin th
 * as integral_0^{pi/2} dth / sqrt(1 - kappa^2 sin^2 th) */
double orc_ellipk(double kappa) {
  return orc_integrate(k_integrand, &kappa, 0.0, 0.5 * M_PI, 1e-14);
}

typedef struct {
  double u1, du, c, omega, phi0;
} part_t;

static void part_setup(const double* p, part_t* q) {
  double u2 = 1.0 / p[0], u1 = 1.0 / p[1];
  double u3 = 1.0 - u1 - u2;
  double kappa = sqrt((u2 - u1) / (u3 - u1));
  double K = orc_ellipk(kappa);
  double ubar = 0.5 * (u1 + u2);
  q->u1 = u1;
  q->du = u2 - u1;
  q->c = M_PI / (4.0 * K) * sqrt(u3 - u1);
  q->omega = sqrt(ubar * ubar * ubar / 2.0);
  q->phi0 = p[2];
}

/* u of the particle's point a at coordinate time t (Appendix B approximation) */
double orc_particle_u(const double* particle, double a, double t) {
  part_t q;
  part_setup(particle, &q);
  double s = sin(q.c * (a + q.omega * t + q.phi0));
  return q.u1 + q.du * s * s;
}

double orc_disc_density(const double* particles, int32_t n, double ht, double hr,
                        double hphi) {
  double rho = 0.0;
  for (int32_t j = 0; j < n; ++j) {
    part_t q;
    part_setup(particles + 3 * j, &q);
    double ph = q.omega * ht + q.phi0;
    double a = hphi - ph;
    a -= 2.0 * M_PI * floor(a / (2.0 * M_PI));
    double s = sin(q.c * (a + ph));
    double ua = q.u1 + q.du * s * s;
    double da = a / M_PI - 1.0, dr = hr - 1.0 / ua;
    double d2 = da * da + dr * dr;
    if (d2 < 1.0) rho += (1.0 - d2) * (1.0 - d2);
  }
  return rho;
}
