/*
 * Whole pixels: beam initialisation, tracing, disc and star shading, per 2x2 quad.
 * TEST INFRASTRUCTURE ONLY (see bh_oracle.h).  Everything in FP64.
 *
 * Beam initialisation (Section 3.2, eqs. staticbasis, camerabasis, d, raybasis, alpha):
 *   pixel (x, y) -> q^w = x + 1/2 - W/2, q^h = H/2 - y - 1/2 (row 0 at the top),
 *   f = (H/2) / tan(fov_y / 2);
 *   camera-frame direction n_C = normalize(q^w e_w + q^h e_h - f e_d);
 *   eq. d projects -e_tau + n_C onto the static observer's space: for a camera moving at
 *   velocity v relative to the static observer this is the aberration
 *   n_S = [n_C + ((gamma-1)(n_C.v^) - gamma |v|) v^] / (gamma (1 - v.n_C));
 *   the static basis vector e_r has pseudo-Cartesian length sqrt(1-u) (eq. staticbasis),
 *   so the coordinate direction is d = sqrt(1-u)(n_S.r^) r^ + (n_S - (n_S.r^) r^);
 *   e_x' = r^, e_z' = normalize(e_x' x d), e_y' = e_z' x e_x', delta = angle(e_x', d);
 *   t = +-normalize(e_z x e_z') with t.e_y' >= 0, alpha = angle(e_x', t).
 * Escape direction d' = cos(delta') e_x' + sin(delta') e_y' (Section 3.3.2).
 *
 * Disc (Sections 3.3.3, 3.4.2): for each crossing u' in order along the beam,
 *   T' = T0 (r'/3)^T_exp (or the paper's T^4 ~ u^3 (1 - sqrt(3u)) law, peak T0),
 *   g(k',l') with the Keplerian 4-velocity k' = [sqrt(2/(2-3u')), 0, 0, sqrt(u'^3/(2-3u'))]
 *   and k'^phi rotated by zeta = e_z.e_z' gives the emitter energy factor
 *   sqrt(2/(2-3u')) (1 + b sqrt(u'^3/2) zeta), b = 1/e, for light reaching the camera;
 *   camera factor D_cam = gamma (1 + v.n_S) / sqrt(1 - u_c) (static observer energy
 *   (1-u)^-1/2 times the special-relativistic Doppler factor, g(k, l) with k = e_tau);
 *   D = D_cam / emitter factor; received band radiance k_disc * L_b(D T').
 *   Front-to-back composite with opacity rho (reading; the paper does not say).
 *   Animated disc (Appendix B): the crossing at beam-plane angle psi (from e_x' towards
 *   e_y') sits in direction cos(psi) e_x' + sin(psi) e_y', whose azimuth about e_z is h^phi;
 *   h^r = 1/u', h^t = camera time - retarded time; the crossing's opacity is
 *   min(1, rho * density(h)) (reading: the density scales the opaque layer).
 *
 * Stars (Section 3.3.2 filtering, Section 3.4.1 lensing): fine 2x2-quad differences give
 *   d_w d' = d'(x0+1, y) - d'(x0, y), d_h d' = d'(x, y0+1) - d'(x, y0); face coordinates of
 *   d' and their derivatives
 *   d U = (d d_a - U sign(d_k) d d_k) / |d_k|;  J = [[d_w U, d_h U], [d_w V, d_h V]];
 *   half extents of J [-1,1]^2: hu = |J00|+|J01|, hv = |J10|+|J11|; level-0 width
 *   E0 = max(hu, hv) n0; mip level L = smallest L with E0 / 2^L <= 8 (at most 9x9 texels);
 *   every texel of level L whose cell meets [U-hu, U+hu] x [V-hv, V+hv] on the centre face
 *   is visited rows then columns; a star at face position s gets (w, h) = J^-1 (s - c) and
 *   weight f(w) f(h), f(x) = max(1 - |x|, 0); A = sum w I, B = sum w I T.
 *   Omega/Omega' = |d_w q x d_h q| / |d_w d' x d_h d'| (Section 3.4.1), q = normalize(q^w,
 *   q^h, -f) the camera-frame direction; both partial derivatives are the same fine 2x2-quad
 *   differences (the pipeline's screen-space derivatives, Section 3.3.2), so the ratio is
 *   exactly 1 wherever d' is a rotation of q (flat space, static camera);
 *   star colour_b = k_star (Omega/Omega') A L_b(D_cam T_pix) / sum_b L_b(T_pix), T_pix = B/A
 *   (static stars: k' = [1, 0, 0, 0]).  If any member of the quad is captured the star
 *   term is zero for the whole quad.  A band-colour star map (emission.c) gathers the
 *   weighted band sums instead; their sum S and chromaticity (r, g) give
 *   colour_b = k_star (Omega/Omega') S C_b(r, g, D_cam) (spectrum.c).
 * Area sources (area.c): the same quad differences give the footprint; the filtered
 *   (A, B) = mean (I, I T) give area colour_b = k_area A L_b(D_cam T_pix) / sum_b L_b(T_pix),
 *   without Omega/Omega'; zero for a quad with a captured member, as for stars.  Band maps
 *   (spectrum.c) filter (R, G, B) instead; the footprint's band sum S and chromaticity
 *   (r, g) = (R, G) / S give colour_b = k_area S C_b(r, g, D_cam), from the C table
 *   (table mode) or computed exactly.  Both sky terms are seen through the disc's
 *   remaining transmittance.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#include "bh_oracle.h"
#include "oracle_internal.h"

typedef struct {
  double rhat[3], ew[3], eh[3], ed[3];
  double f, u_c, sq1mu;
  double gamma, vmag, vhat[3], v[3];
  double u_ic, u_oc;
} vsetup;

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

static void setup(const orc_view* v, vsetup* s) {
  double p[3] = {v->cam_pos[0] / v->r_s, v->cam_pos[1] / v->r_s, v->cam_pos[2] / v->r_s};
  double r = norm3(p);
  for (int i = 0; i < 3; ++i) {
    s->rhat[i] = p[i] / r;
    s->ew[i] = v->cam_rot[i];
    s->eh[i] = v->cam_rot[3 + i];
    s->ed[i] = v->cam_rot[6 + i];
    s->v[i] = v->cam_vel[i];
  }
  s->u_c = 1.0 / r;
  s->sq1mu = sqrt(1.0 - s->u_c);
  s->f = 0.5 * v->height / tan(0.5 * v->fov_y);
  s->vmag = norm3(s->v);
  s->gamma = 1.0 / sqrt(1.0 - s->vmag * s->vmag);
  for (int i = 0; i < 3; ++i) s->vhat[i] = s->vmag > 0 ? s->v[i] / s->vmag : 0.0;
  s->u_ic = v->r_s / v->disc_r_in;
  s->u_oc = v->r_s / v->disc_r_out;
}

typedef struct {
  int captured, degenerate;
  double dprime[3];
  double q[3];      /* camera-frame direction normalize(q^w, q^h, -f) */
  double ey[3];
  double e2, zeta, d_cam, delta, alpha;
  orc_ray ray;
} ray_out;

typedef struct {
  const orc_view* v;
  vsetup s;
  const double* cube;
  int32_t n0, nl;
  const double *D, *U, *Dt, *Ut;
  int32_t d_n, u_ne, u_nphi;
  int32_t march; /* > 0: ray marching with at most this many steps instead of TraceRay */
} ctx_t;

static void trace_pixel(const ctx_t* c, int32_t x, int32_t y, ray_out* o) {
  const vsetup* s = &c->s;
  const orc_view* v = c->v;
  memset(o, 0, sizeof(*o));
  double qw = x + 0.5 - 0.5 * v->width, qh = 0.5 * v->height - y - 0.5;
  double nq = sqrt(qw * qw + qh * qh + s->f * s->f);
  o->q[0] = qw / nq;
  o->q[1] = qh / nq;
  o->q[2] = -s->f / nq;
  double nc[3];
  for (int i = 0; i < 3; ++i) nc[i] = (qw * s->ew[i] + qh * s->eh[i] - s->f * s->ed[i]) / nq;
  /* aberration into the static observer's frame */
  double ns[3];
  if (s->vmag > 0.0) {
    double nv = dot3(nc, s->vhat);
    double k = (s->gamma - 1.0) * nv - s->gamma * s->vmag;
    double den = s->gamma * (1.0 - s->vmag * nv);
    for (int i = 0; i < 3; ++i) ns[i] = (nc[i] + k * s->vhat[i]) / den;
  } else {
    for (int i = 0; i < 3; ++i) ns[i] = nc[i];
  }
  o->d_cam = s->gamma * (1.0 + dot3(s->v, ns)) / s->sq1mu;
  /* coordinate direction */
  double nr = dot3(ns, s->rhat), d[3];
  for (int i = 0; i < 3; ++i) d[i] = ns[i] + (s->sq1mu - 1.0) * nr * s->rhat[i];
  double cz[3];
  cross3(s->rhat, d, cz);
  double ncz = norm3(cz);
  double delta = atan2(ncz, dot3(s->rhat, d));
  o->delta = delta;
  if (ncz < 1e-14 * norm3(d)) {
    o->degenerate = 1;
    if (c->march > 0)
      orc_march_ray(s->u_c, delta, 0.0, -1.0, 2.0, c->march, 1.0, &o->ray);
    else
      orc_trace_exact(s->u_c, delta, 0.0, -1.0, 2.0, 1.0, &o->ray);
    o->captured = o->ray.captured;
    o->e2 = s->u_c * s->u_c * (1.0 - s->u_c);
    for (int i = 0; i < 3; ++i) o->dprime[i] = cos(o->ray.delta_prime) * s->rhat[i];
    return;
  }
  double ez[3] = {cz[0] / ncz, cz[1] / ncz, cz[2] / ncz}, ey[3];
  cross3(ez, s->rhat, ey);
  for (int i = 0; i < 3; ++i) o->ey[i] = ey[i];
  double t[3] = {-ez[1], ez[0], 0.0}; /* e_z x e_z' */
  double nt = norm3(t);
  double alpha = 0.0;
  double u_ic = s->u_ic, u_oc = s->u_oc;
  if (nt < 1e-14) {
    o->degenerate = 1; /* beam plane is the disc plane: no isolated crossings */
    u_ic = -1.0;
    u_oc = 2.0;
  } else {
    for (int i = 0; i < 3; ++i) t[i] /= nt;
    double ty = dot3(t, ey);
    if (ty < 0.0) {
      for (int i = 0; i < 3; ++i) t[i] = -t[i];
      ty = -ty;
    }
    alpha = atan2(ty, dot3(t, s->rhat));
  }
  o->alpha = alpha;
  o->zeta = ez[2];
  double cot = dot3(s->rhat, d) / ncz;
  o->e2 = s->u_c * s->u_c * cot * cot + s->u_c * s->u_c * (1.0 - s->u_c);
  if (c->march > 0)
    orc_march_ray(s->u_c, delta, alpha, u_ic, u_oc, c->march, 1.0, &o->ray);
  else if (c->D)
    orc_trace_table_t(c->D, c->Dt, c->d_n, c->U, c->Ut, c->u_ne, c->u_nphi, s->u_c, delta,
                      alpha, u_ic, u_oc, &o->ray);
  else
    orc_trace_exact(s->u_c, delta, alpha, u_ic, u_oc, 1.0, &o->ray);
  o->captured = o->ray.captured;
  if (!o->captured) {
    double cd = cos(o->ray.delta_prime), sd = sin(o->ray.delta_prime);
    for (int i = 0; i < 3; ++i) o->dprime[i] = cd * s->rhat[i] + sd * ey[i];
  }
}

static double disc_temperature(const orc_view* v, double u) {
  if (v->disc_T_law == 1) {
    double pk = 6.0 / 7.0; /* maximum of s^6 (1 - s), s = sqrt(3u) */
    double fmax = pow(pk, 6) * (1.0 - pk) / 27.0;
    double f = u * u * u * (1.0 - sqrt(3.0 * u));
    if (!(f > 0.0)) return 0.0;
    return v->disc_T0 * pow(f / fmax, 0.25);
  }
  return v->disc_T0 * pow(1.0 / (3.0 * u), v->disc_T_exp);
}

static void face_coords(const double* d, int* face, int* k, double* U, double* V) {
  int kk = 0;
  if (fabs(d[1]) > fabs(d[kk])) kk = 1;
  if (fabs(d[2]) > fabs(d[kk])) kk = 2;
  double m = fabs(d[kk]);
  *k = kk;
  *face = 2 * kk + (d[kk] < 0.0);
  *U = d[(kk + 1) % 3] / m;
  *V = d[(kk + 2) % 3] / m;
}

/* footprint gather; returns the mip level, fills A and B */
/* A, B: the tent-weighted sums of I and I T; for a band map (the view's star_bands) the
   weighted sums of R, G, B go to A[0..2] */
static int gather(const ctx_t* c, const double* dp, const double* dw, const double* dh,
                  double* A, double* B) {
  const int bands = c->v->star_bands, stride = bands ? 5 : 4;
  A[0] = 0.0;
  if (bands) A[1] = A[2] = 0.0;
  *B = 0.0;
  int face, k;
  double U, V;
  face_coords(dp, &face, &k, &U, &V);
  int a = (k + 1) % 3, b = (k + 2) % 3;
  double m = fabs(dp[k]), sg = dp[k] < 0.0 ? -1.0 : 1.0;
  double J00 = (dw[a] - U * sg * dw[k]) / m, J01 = (dh[a] - U * sg * dh[k]) / m;
  double J10 = (dw[b] - V * sg * dw[k]) / m, J11 = (dh[b] - V * sg * dh[k]) / m;
  double hu = fabs(J00) + fabs(J01), hv = fabs(J10) + fabs(J11);
  double E0 = fmax(hu, hv) * c->n0;
  int L = 0;
  while (L < c->nl - 1 && E0 > 8.0 * (double)(1 << L)) ++L;
  double det = J00 * J11 - J01 * J10;
  if (!(fabs(det) >= 1e-20)) return L;
  int32_t nL = c->n0 >> L;
  int64_t off = 0;
  for (int l = 0; l < L; ++l) off += 6LL * (c->n0 >> l) * (c->n0 >> l);
  int32_t x0 = (int32_t)floor(0.5 * (U - hu + 1.0) * nL), x1 = (int32_t)floor(0.5 * (U + hu + 1.0) * nL);
  int32_t y0 = (int32_t)floor(0.5 * (V - hv + 1.0) * nL), y1 = (int32_t)floor(0.5 * (V + hv + 1.0) * nL);
  if (x0 < 0) x0 = 0;
  if (y0 < 0) y0 = 0;
  if (x1 > nL - 1) x1 = nL - 1;
  if (y1 > nL - 1) y1 = nL - 1;
  for (int32_t ty = y0; ty <= y1; ++ty)
    for (int32_t tx = x0; tx <= x1; ++tx) {
      const double* tex = c->cube + (off + ((int64_t)face * nL + ty) * nL + tx) * stride;
      const double* pos = tex + (bands ? 3 : 2);
      if (!((bands ? tex[0] + tex[1] + tex[2] : tex[0]) > 0.0)) continue;
      double su = 2.0 * (tx + pos[0]) / nL - 1.0, sv = 2.0 * (ty + pos[1]) / nL - 1.0;
      double du = su - U, dv = sv - V;
      double w = (J11 * du - J01 * dv) / det;
      double h = (-J10 * du + J00 * dv) / det;
      double wt = fmax(1.0 - fabs(w), 0.0) * fmax(1.0 - fabs(h), 0.0);
      if (bands) {
        for (int b = 0; b < 3; ++b) A[b] += wt * tex[b];
      } else {
        A[0] += wt * tex[0];
        *B += wt * tex[0] * tex[1];
      }
    }
  return L;
}

static void shade_quad(const ctx_t* c, int32_t x0, int32_t y0, orc_pixel* out) {
  const orc_view* v = c->v;
  ray_out r[4];
  for (int m = 0; m < 4; ++m) trace_pixel(c, x0 + (m & 1), y0 + (m >> 1), &r[m]);
  int any_captured = r[0].captured | r[1].captured | r[2].captured | r[3].captured;
  for (int m = 0; m < 4; ++m) {
    orc_pixel* p = &out[m];
    ray_out* o = &r[m];
    memset(p, 0, sizeof(*p));
    p->x = x0 + (m & 1);
    p->y = y0 + (m >> 1);
    p->delta_prime = o->captured ? INFINITY : o->ray.delta_prime;
    p->captured = o->captured;
    p->degenerate = o->degenerate;
    p->e2_over_mu = o->e2 / ORC_MU;
    p->d_cam = o->d_cam;
    p->delta = o->delta;
    p->alpha = o->alpha;
    p->zeta = o->zeta;
    p->mip_level = -1;
    p->n_cross = o->ray.n_cross > 2 ? 2 : o->ray.n_cross;
    for (int k = 0; k < o->ray.n_cross; ++k) {
      if (k < 2) p->u_cross[k] = o->ray.u_cross[k];
      p->branch_bits |= 1 << o->ray.branch[k];
    }
    /* disc, front to back */
    double trans = 1.0;
    double rho = v->disc_opacity;
    double e = sqrt(o->e2);
    for (int k = 0; k < o->ray.n_cross; ++k) {
      double u = o->ray.u_cross[k];
      double Tp = disc_temperature(v, u);
      double kt = sqrt(2.0 / (2.0 - 3.0 * u));
      double om = sqrt(u * u * u / 2.0);
      double D = o->d_cam / (kt * (1.0 + om * o->zeta / e));
      double L[3];
      orc_band_radiance(D * Tp, L);
      double rk = rho;
      if (v->disc_density == 1) {
        double psi = o->ray.phi_cross[k], P[3];
        for (int i = 0; i < 3; ++i) P[i] = cos(psi) * c->s.rhat[i] + sin(psi) * o->ey[i];
        double hphi = atan2(P[1], P[0]);
        double ht = v->time - o->ray.t_cross[k];
        double dens = orc_disc_density(v->particles, v->n_particles, ht, 1.0 / u, hphi);
        rk = fmin(1.0, rho * dens);
        if (k < 2) {
          p->t_ret[k] = o->ray.t_cross[k];
          p->hit_az[k] = hphi;
          p->density[k] = dens;
        }
      }
      for (int b = 0; b < 3; ++b) p->disc_rgb[b] += trans * rk * v->k_disc * L[b];
      trans *= 1.0 - rk;
    }
    /* stars */
    p->star_zeroed = any_captured;
    if (c->cube && !any_captured) {
      int mw0 = (m & 2), mw1 = (m & 2) | 1; /* same row */
      int mh0 = (m & 1), mh1 = (m & 1) | 2; /* same column */
      double dw[3], dh[3], qw[3], qh[3];
      for (int i = 0; i < 3; ++i) {
        dw[i] = r[mw1].dprime[i] - r[mw0].dprime[i];
        dh[i] = r[mh1].dprime[i] - r[mh0].dprime[i];
        qw[i] = r[mw1].q[i] - r[mw0].q[i];
        qh[i] = r[mh1].q[i] - r[mh0].q[i];
      }
      double cd[3], cq[3];
      cross3(dw, dh, cd);
      cross3(qw, qh, cq);
      double om = norm3(cq), omp = norm3(cd);
      p->omega_ratio = omp > 0.0 ? om / omp : 0.0;
      double A, B, Ab[3];
      p->mip_level = gather(c, o->dprime, dw, dh, Ab, &B);
      A = v->star_bands ? Ab[0] + Ab[1] + Ab[2] : Ab[0];
      p->star_A = A;
      if (v->star_bands) {
        /* band colours: S C(r, g, D_cam) (spectrum.c), from the table or exactly */
        if (A > 0.0 && omp > 0.0) {
          double C[3];
          if (v->ctable)
            orc_cshift_lookup(v->ctable, v->ct_n[0], v->ct_n[1], v->ct_n[2], Ab[0] / A,
                              Ab[1] / A, o->d_cam, C);
          else
            orc_color_shift(Ab[0] / A, Ab[1] / A, o->d_cam, C);
          for (int b = 0; b < 3; ++b) p->star_rgb[b] = v->k_star * p->omega_ratio * A * C[b];
        }
      } else if (A > 0.0 && omp > 0.0) {
        double Tpix = B / A;
        p->star_T = Tpix;
        double Lr[3], Ln[3];
        orc_band_radiance(o->d_cam * Tpix, Lr);
        orc_band_radiance(Tpix, Ln);
        double norm = Ln[0] + Ln[1] + Ln[2];
        for (int b = 0; b < 3; ++b)
          p->star_rgb[b] = v->k_star * p->omega_ratio * A * Lr[b] / norm;
      }
    }
    /* area sources: the footprint mean of the map, one Doppler shift per pixel as for
       stars, no lensing amplification (Section 3.4.1) */
    if (v->area && !any_captured) {
      int mw0 = (m & 2), mw1 = (m & 2) | 1, mh0 = (m & 1), mh1 = (m & 1) | 2;
      double dw[3], dh[3], A, B;
      for (int i = 0; i < 3; ++i) {
        dw[i] = r[mw1].dprime[i] - r[mw0].dprime[i];
        dh[i] = r[mh1].dprime[i] - r[mh0].dprime[i];
      }
      if (v->area_bands) {
        double mb[3];
        orc_area_filter_bands(v->area, v->area_n0, o->dprime, dw, dh, mb);
        double S = mb[0] + mb[1] + mb[2], C[3];
        p->area_A = S;
        if (S > 0.0) {
          p->area_chroma[0] = mb[0] / S;
          p->area_chroma[1] = mb[1] / S;
          if (v->ctable)
            orc_cshift_lookup(v->ctable, v->ct_n[0], v->ct_n[1], v->ct_n[2], mb[0] / S,
                              mb[1] / S, o->d_cam, C);
          else
            orc_color_shift(mb[0] / S, mb[1] / S, o->d_cam, C);
          for (int b = 0; b < 3; ++b) p->area_rgb[b] = v->k_area * S * C[b];
        }
        if (v->area_exact) {
          orc_area_exact_bands(v->area, v->area_n0, o->dprime, dw, dh, mb);
          p->area_exact_A = mb[0] + mb[1] + mb[2];
        }
      } else {
        orc_area_filter(v->area, v->area_n0, o->dprime, dw, dh, &A, &B);
        p->area_A = A;
        if (A > 0.0) {
          double Tpix = B / A, Lr[3], Ln[3];
          p->area_T = Tpix;
          orc_band_radiance(o->d_cam * Tpix, Lr);
          orc_band_radiance(Tpix, Ln);
          double norm = Ln[0] + Ln[1] + Ln[2];
          if (norm > 0.0)
            for (int b = 0; b < 3; ++b) p->area_rgb[b] = v->k_area * A * Lr[b] / norm;
        }
        if (v->area_exact) {
          orc_area_exact(v->area, v->area_n0, o->dprime, dw, dh, &A, &B);
          p->area_exact_A = A;
          p->area_exact_T = A > 0.0 ? B / A : 0.0;
        }
      }
    }
    for (int b = 0; b < 3; ++b)
      p->rgb[b] = p->disc_rgb[b] + trans * (p->star_rgb[b] + p->area_rgb[b]);
  }
}

typedef struct {
  const ctx_t* c;
  const int32_t* quads;
  int64_t nq;
  orc_pixel* out;
  int64_t next;
  pthread_mutex_t mu;
} rjob;

static void* rworker(void* p) {
  rjob* j = (rjob*)p;
  for (;;) {
    pthread_mutex_lock(&j->mu);
    int64_t q0 = j->next;
    j->next += 16;
    pthread_mutex_unlock(&j->mu);
    if (q0 >= j->nq) break;
    int64_t q1 = q0 + 16 < j->nq ? q0 + 16 : j->nq;
    for (int64_t q = q0; q < q1; ++q)
      shade_quad(j->c, j->quads[2 * q], j->quads[2 * q + 1], j->out + 4 * q);
  }
  return NULL;
}

int orc_render_quads(const orc_view* v, const double* cube, int32_t n0, const double* D,
                     int32_t d_n, const double* U, int32_t u_ne, int32_t u_nphi,
                     const int32_t* quads, int64_t nq, orc_pixel* out, int nthreads) {
  return orc_render_quads_t(v, cube, n0, D, NULL, d_n, U, NULL, u_ne, u_nphi, quads, nq, out,
                            nthreads);
}

static int render_quads(const orc_view* v, const double* cube, int32_t n0, const double* D,
                        const double* Dt, int32_t d_n, const double* U, const double* Ut,
                        int32_t u_ne, int32_t u_nphi, int32_t march, const int32_t* quads,
                        int64_t nq, orc_pixel* out, int nthreads);

int orc_render_quads_t(const orc_view* v, const double* cube, int32_t n0, const double* D,
                       const double* Dt, int32_t d_n, const double* U, const double* Ut,
                       int32_t u_ne, int32_t u_nphi, const int32_t* quads, int64_t nq,
                       orc_pixel* out, int nthreads) {
  return render_quads(v, cube, n0, D, Dt, d_n, U, Ut, u_ne, u_nphi, 0, quads, nq, out,
                      nthreads);
}

int orc_render_quads_m(const orc_view* v, const double* cube, int32_t n0, int32_t march_steps,
                       const int32_t* quads, int64_t nq, orc_pixel* out, int nthreads) {
  if (march_steps < 1 || v->disc_density != 0) return 1;
  return render_quads(v, cube, n0, NULL, NULL, 0, NULL, NULL, 0, 0, march_steps, quads, nq,
                      out, nthreads);
}

static int render_quads(const orc_view* v, const double* cube, int32_t n0, const double* D,
                        const double* Dt, int32_t d_n, const double* U, const double* Ut,
                        int32_t u_ne, int32_t u_nphi, int32_t march, const int32_t* quads,
                        int64_t nq, orc_pixel* out, int nthreads) {
  if (!(v->r_s > 0) || v->width < 1 || v->height < 1) return 1;
  if (v->disc_density == 1 && (v->n_particles < 0 || (v->n_particles > 0 && !v->particles) ||
                               (D && (!Dt || !Ut))))
    return 1;
  ctx_t c;
  memset(&c, 0, sizeof(c));
  c.v = v;
  setup(v, &c.s);
  if (!(c.s.u_c < 1.0) || !(c.s.vmag < 1.0)) return 1;
  c.cube = cube;
  c.n0 = n0;
  c.nl = 0;
  if (cube)
    while ((n0 >> c.nl) >= 1) ++c.nl;
  c.D = D;
  c.U = U;
  c.Dt = Dt;
  c.Ut = Ut;
  c.d_n = d_n;
  c.u_ne = u_ne;
  c.u_nphi = u_nphi;
  c.march = march;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  rjob j = {&c, quads, nq, out, 0, PTHREAD_MUTEX_INITIALIZER};
  pthread_t th[256];
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, rworker, &j);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  return 0;
}

/* record sizes, so the Python front end can check its layouts */
int64_t orc_sizeof_pixel(void) { return (int64_t)sizeof(orc_pixel); }
int64_t orc_sizeof_ray(void) { return (int64_t)sizeof(orc_ray); }
int64_t orc_sizeof_view(void) { return (int64_t)sizeof(orc_view); }
