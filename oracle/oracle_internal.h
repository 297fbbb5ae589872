/* Internal helpers of the FP64 oracle.  TEST INFRASTRUCTURE ONLY (see bh_oracle.h). */
#ifndef BH_ORACLE_INTERNAL_H
#define BH_ORACLE_INTERNAL_H

typedef double (*orc_fn)(double x, void* ctx);

/* adaptive Gauss-Legendre integral of f over [a, b] to relative tolerance rel_tol */
double orc_integrate(orc_fn f, void* ctx, double a, double b, double rel_tol);
/* the same 12-point Gauss-Legendre rule on `panels` equal panels (no adaptivity: for
   integrands that may cancel, where a relative tolerance has nothing to hold on to) */
double orc_integrate_panels(orc_fn f, void* ctx, double a, double b, int panels);

/* integrate the orbit equation from (u0, w0 = du/dphi) at phi = 0; shared by the
 * per-pixel trace and the deflection of rays from infinity */
void orc_integrate_ray(double u0, double w0, double alpha, double u_ic, double u_oc,
                       double gr, orc_ray* out);

#endif
