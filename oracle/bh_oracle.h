/*
 * FP64 CPU oracle for the per-pixel black-hole beam tracer of Bruneton,
 * "Real-time High-Quality Rendering of Non-Rotating Black Holes" (arXiv 2010.08735).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the GPU
 * library is checked against.  Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table or
 * constant generator with the GPU library, and the GPU library never calls it.
 *
 * Units: Schwarzschild radius r_s = 1 and c = 1 (Section 3.1), u = 1/r.
 *
 * Two ways to trace a ray:
 *   exact mode  -- the orbit equation u'' = 3/2 u^2 - u (Section 3.3, eq. rayequation) is
 *                  integrated per ray with an adaptive Dormand-Prince 5(4) method and
 *                  event location (escape, capture, disc-plane crossings);
 *   table mode  -- deflection and intersection tables are filled by quadrature of the
 *                  first integral at the texel centres (Section 3.3.2, Appendix A) and the
 *                  paper's TraceRay procedure (Algorithm 1) reads them in FP64.
 * Shading follows Sections 3.3.2 (stars, filtering), 3.3.3 (disc) and 3.4 (lensing,
 * Doppler, beaming).  Parity status of every function is listed in its comment; every
 * function here is pinned by a test that does not reuse this code.
 */
#ifndef BH_ORACLE_H
#define BH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MU (4.0 / 27.0)

/* Camera + disc description, mirrors the GPU library's view record field by field. */
typedef struct {
  double r_s;
  double cam_pos[3];
  double cam_vel[3];
  double cam_rot[9];      /* rows e_w, e_h, e_d; the camera looks along -e_d */
  double fov_y;
  int32_t width, height;
  double disc_r_in, disc_r_out;
  int32_t disc_T_law;     /* 0: T0 (r/3)^T_exp ; 1: T^4 ~ u^3 (1 - sqrt(3u)), peak T0 */
  int32_t pad0;
  double disc_T0, disc_T_exp;
  double disc_opacity, k_disc, k_star;
  /* animated disc (Appendix B): disc_density 0 = uniform, 1 = particles */
  double time;            /* the camera's coordinate time */
  int32_t disc_density;
  int32_t n_particles;
  const double* particles;  /* n_particles triples (r_peri, r_apo, phi0) */
  /* area sources (Section 3.3.2): the map's levels from orc_area_build, or NULL */
  const double* area;
  int32_t area_n0;
  int32_t area_exact;     /* 1: also compute the exact footprint mean (diagnostic) */
  double k_area;
  /* 1: `area` is a band map (orc_area_build_bands), shifted with C(rg, D) (Section 3.4.2):
     through the table `ctable` of ct_n[0] x ct_n[1] x ct_n[2] nodes (orc_cshift_table), or
     exactly (orc_color_shift) if ctable is NULL */
  int32_t area_bands;
  int32_t ct_n[3];
  const double* ctable;
  /* 1: the star map is a band map (orc_cubemap_build_bands), received as S C(r, g, D) */
  int32_t star_bands;
  int32_t pad1;
} orc_view;

/* Result of tracing one ray in its orbital plane. */
typedef struct {
  double delta_prime;     /* escape angle from e_x' (INFINITY if captured)            */
  int32_t captured;
  int32_t n_cross;        /* crossings of the disc annulus, in order along the beam     */
  double u_cross[4];
  double phi_cross[4];    /* rotated azimuth of each crossing                           */
  int32_t branch[4];      /* 0: before the apsis of the backward ray, 1: after it       */
  int32_t steps;          /* accepted integrator steps (exact mode, marching), 0 in
                             table mode                                                  */
  int32_t unfinished;     /* marching: the step budget ran out (drawn as captured)      */
  double t_cross[4];      /* retarded time: coordinate time from the crossing to the
                             camera (exact mode; table mode with time channels)          */
} orc_ray;

/* One rendered pixel with the diagnostics the parity mask needs. */
typedef struct {
  double rgb[3];
  double disc_rgb[3];
  double star_rgb[3];
  double delta_prime;     /* INFINITY if captured */
  double u_cross[2];      /* first and second crossing in beam order (0 if absent) */
  double e2_over_mu;
  double omega_ratio;     /* lensing amplification Omega/Omega' (0 if undefined) */
  double d_cam;           /* frequency ratio received/emitted for static stars */
  double star_A;          /* filtered intensity sum */
  double star_T;          /* intensity-weighted temperature of the footprint */
  double delta, alpha, zeta;
  int32_t x, y;
  int32_t n_cross;
  int32_t branch_bits;    /* bit k set: a crossing on branch k was found */
  int32_t captured;
  int32_t star_zeroed;    /* a member of the 2x2 quad is captured */
  int32_t degenerate;     /* ray radial or ray plane == disc plane */
  int32_t mip_level;      /* -1 if no gather happened */
  int32_t pad0, pad1;
  double t_ret[2];        /* retarded time of each crossing (animated disc only) */
  double hit_az[2];       /* disc azimuth of each crossing (animated disc only) */
  double density[2];      /* particle density at each crossing (animated disc only) */
  double area_rgb[3];     /* received light of the area map (before the disc's
                             transmittance) */
  double area_A, area_T;  /* filtered radiance and colour temperature of the footprint */
  double area_exact_A, area_exact_T;  /* the exact footprint mean (if area_exact) */
  double area_chroma[2];  /* band maps: the footprint's (r, g); area_A is its band sum */
} orc_pixel;

/* ---- geometry of rays (Section 3.3.1) --------------------------------------------- */
double orc_apsis(double e2);                         /* eq. uapsis, e2 < mu */
int orc_trace_exact(double u_c, double delta, double alpha, double u_ic, double u_oc,
                    double gr, orc_ray* out);        /* gr = 1: Schwarzschild, 0: flat */
double orc_deflection(double e);                     /* 2 phi_a - pi for a ray from infinity */
double orc_u_at_phi(double u0, double w0, double phi, double gr); /* u(phi) along a ray */

/* ---- ray marching (the ablation of Section 5, method M3 of Table 1) ----------------- */
/* fixed-step fourth-order Runge-Kutta in phi, h = 2 pi / nsteps, at most nsteps steps;
 * events from the cubic Hermite interpolant of each step (see march.c) */
int orc_march_ray(double u_c, double delta, double alpha, double u_ic, double u_oc,
                  int32_t nsteps, double gr, orc_ray* out);
/* the bare integrator: k steps of size h from (u0, w0) */
void orc_march_state(double u0, double w0, double h, int32_t k, double gr, double* u,
                     double* w);
double orc_hermite(double p0, double m0, double p1, double m1, double h, double s);
double orc_hermite_first_root(double p0, double m0, double p1, double m1, double h);

/* ---- tables by quadrature (table mode) ---------------------------------------------- */
int orc_tables(int32_t d_n, int32_t u_ne, int32_t u_nphi, double* D, double* U, int nthreads);
int orc_table_entry_D(int32_t d_n, int32_t i, int32_t j, double* value, double* e2, double* u);
int orc_table_entry_U(int32_t u_ne, int32_t u_nphi, int32_t i, int32_t j, double* value,
                      double* e2, double* phi);
int orc_trace_table(const double* D, int32_t d_n, const double* U, int32_t u_ne, int32_t u_nphi,
                    double u_c, double delta, double alpha, double u_ic, double u_oc, orc_ray* out);
/* time channels (regularised time tau at the same texel centres) and TraceRay with them */
int orc_tables_time(int32_t d_n, int32_t u_ne, int32_t u_nphi, double* Dt, double* Ut,
                    int nthreads);
int orc_trace_table_t(const double* D, const double* Dt, int32_t d_n, const double* U,
                      const double* Ut, int32_t u_ne, int32_t u_nphi, double u_c, double delta,
                      double alpha, double u_ic, double u_oc, orc_ray* out);
double orc_tau_in(double e2, double u);              /* tau on the incoming branch */
double orc_time_singular(double u);                  /* S(u) = ln(u/(1-u)) - 1/u */

/* ---- emission (Sections 3.3.3, 3.4.2) ----------------------------------------------- */
void orc_band_radiance(double T, double out[3]);     /* R, G, B box bands, W m^-2 sr^-1 */
double orc_planck(double lambda, double T);          /* spectral radiance B_lambda(T) */

/* ---- star cubemap (Section 3.3.2 "Emitted light") ------------------------------------ */
int64_t orc_cubemap_texels(int32_t n0);              /* texel count over all mip levels */
int orc_cubemap_build(const float* dirs, const float* inten, const float* temp, int64_t n,
                      int32_t n0, double* texels);   /* texels: orc_cubemap_texels * 4 */
/* band colours: rgb 3 floats per star; texels: orc_cubemap_texels * 5 (R, G, B, p_u, p_v) */
int orc_cubemap_build_bands(const float* dirs, const float* rgb, int64_t n, int32_t n0,
                            double* texels);

/* ---- area sources (Section 3.3.2 "Emitted light", Section 3.4.1 closing note) -------- */
int64_t orc_area_texels(int32_t n0);                 /* texel count over all mip levels */
/* it: level-0 (I, T) per texel, 6 n0^2 pairs; levels: orc_area_texels * 2 (I, I T) */
int orc_area_build(const float* it, int32_t n0, double* levels);
/* footprint {d + w dw + h dh : |w|, |h| <= 1/2}: A = mean I, B = mean I T */
void orc_area_filter(const double* levels, int32_t n0, const double* d, const double* dw,
                     const double* dh, double* A, double* B);   /* the anisotropic filter */
void orc_area_exact(const double* levels, int32_t n0, const double* d, const double* dw,
                    const double* dh, double* A, double* B);    /* the exact mean, level 0 */
/* band maps: rgbx level-0 (R, G, B, unused) per texel; levels: orc_area_texels * 3 */
int orc_area_build_bands(const float* rgbx, int32_t n0, double* levels);
void orc_area_filter_bands(const double* levels, int32_t n0, const double* d, const double* dw,
                           const double* dh, double out[3]);
void orc_area_exact_bands(const double* levels, int32_t n0, const double* d, const double* dw,
                          const double* dh, double out[3]);

/* ---- light of any colour under the Doppler shift (Section 3.4.2, spectrum.c) --------- */
double orc_absorption(int k, double lambda);         /* A1 (k = 0), A2 (k = 1) */
void orc_chroma_project(double r, double g, double out[2]);
double orc_band_cct(double r, double g);             /* correlated temperature (K) */
void orc_spectrum_of(double r, double g, double out[3]);       /* (T, a1, a2) */
void orc_color_shift(double r, double g, double D, double out[3]);  /* C_b(r, g, D) */
/* table of log2 C_b, ((i ng + j) nd + k) * 3 doubles, and its trilinear lookup */
void orc_cshift_table(int32_t nr, int32_t ng, int32_t nd, double* out, int nthreads);
void orc_cshift_lookup(const double* tab, int32_t nr, int32_t ng, int32_t nd, double r,
                       double g, double D, double out[3]);

/* ---- whole pixels --------------------------------------------------------------------- */
/* quads: (x0, y0) pairs with even coordinates; out: 4 pixels per quad in the order
 * (x0,y0), (x0+1,y0), (x0,y0+1), (x0+1,y0+1).  D == NULL selects exact mode.
 * cubemap == NULL means a black sky. */
int orc_render_quads(const orc_view* v, const double* cubemap, int32_t n0,
                     const double* D, int32_t d_n, const double* U, int32_t u_ne,
                     int32_t u_nphi, const int32_t* quads, int64_t nq, orc_pixel* out,
                     int nthreads);
/* the same with time channels (table mode of an animated disc needs Dt and Ut) */
int orc_render_quads_t(const orc_view* v, const double* cubemap, int32_t n0,
                       const double* D, const double* Dt, int32_t d_n, const double* U,
                       const double* Ut, int32_t u_ne, int32_t u_nphi, const int32_t* quads,
                       int64_t nq, orc_pixel* out, int nthreads);

/* the same with TraceRay replaced by ray marching with at most march_steps steps */
int orc_render_quads_m(const orc_view* v, const double* cubemap, int32_t n0,
                       int32_t march_steps, const int32_t* quads, int64_t nq, orc_pixel* out,
                       int nthreads);

/* ---- bloom (Section 3.4.3): mipmap filters applied to the final image --------------- */
/* in, out: width x height x 4 doubles (row-major); weights[0 .. levels]; levels <= 16 */
int orc_bloom(const double* in, int32_t width, int32_t height, int32_t levels,
              const double* weights, double* out);

/* ---- display encoding after the glare pass (Section 3.4.3): tone curve, sRGB, 8 bits ---- */
/* in: n x 4 doubles (linear RGBA); out: n x 4 bytes R, G, B, 255; scaled (may be NULL):
   n x 3 values 255 v + 1/2 whose floor is each code; exposure finite and > 0 */
int orc_tonemap(const double* in, int64_t n, double exposure, uint8_t* out, double* scaled);

/* ---- animated disc (Appendix B) ------------------------------------------------------- */
double orc_ellipk(double kappa);                     /* complete elliptic integral K */
double orc_particle_u(const double* particle, double a, double t);
double orc_disc_density(const double* particles, int32_t n, double ht, double hr,
                        double hphi);

/* record sizes (layout check of the Python front end) */
int64_t orc_sizeof_pixel(void);
int64_t orc_sizeof_ray(void);
int64_t orc_sizeof_view(void);

/* quadrature helper exposed for its own pin (Gauss-Legendre exactness) */
double orc_quad_poly_check(int degree);

#ifdef __cplusplus
}
#endif
#endif
