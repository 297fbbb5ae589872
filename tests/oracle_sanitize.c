/*
 * Sanitizer run of the FP64 oracle's C code (test infrastructure).  Calls every entry point
 * of oracle/bh_oracle.h on small inputs, the multithreaded ones with several threads, so
 * that tests/test_sanitizers.py can build it under ASan + UBSan and under TSan and check
 * that the runs are clean.  Exits non-zero if a result is not finite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "bh_oracle.h"

static int bad = 0;
#define FINITE(x)                                                \
  do {                                                           \
    if (!isfinite(x)) {                                          \
      fprintf(stderr, "%s:%d: not finite: %s\n", __FILE__, __LINE__, #x); \
      bad = 1;                                                   \
    }                                                            \
  } while (0)

int main(void) {
  /* geometry of single rays */
  orc_ray r;
  orc_trace_exact(1.0 / 15.0, 1.2, 0.4, 1.0 / 3.0, 1.0 / 12.0, 1.0, &r);
  FINITE(r.delta_prime);
  orc_march_ray(1.0 / 15.0, 1.2, 0.4, 1.0 / 3.0, 1.0 / 12.0, 100, 1.0, &r);
  FINITE(r.delta_prime);
  FINITE(orc_apsis(0.1));
  FINITE(orc_deflection(0.2));
  FINITE(orc_u_at_phi(0.05, 0.01, 1.0, 1.0));

  /* tables by quadrature, four threads */
  const int dn = 32, ne = 8, nphi = 8;
  double* D = calloc((size_t)dn * dn, sizeof(double));
  double* U = calloc((size_t)ne * nphi, sizeof(double));
  double* Dt = calloc((size_t)dn * dn, sizeof(double));
  double* Ut = calloc((size_t)ne * nphi, sizeof(double));
  if (orc_tables(dn, ne, nphi, D, U, 4) || orc_tables_time(dn, ne, nphi, Dt, Ut, 4)) bad = 1;
  orc_trace_table_t(D, Dt, dn, U, Ut, ne, nphi, 1.0 / 15.0, 1.2, 0.4, 1.0 / 3.0, 1.0 / 12.0, &r);
  FINITE(r.delta_prime);

  /* emission and a star cube map */
  double L[3];
  orc_band_radiance(6000.0, L);
  FINITE(L[0] + L[1] + L[2]);
  enum { NS = 500, N0 = 16 };
  float dirs[3 * NS], inten[NS], temp[NS];
  unsigned s = 12345u;
  for (int i = 0; i < NS; ++i) {
    for (int k = 0; k < 3; ++k) {
      s = s * 1664525u + 1013904223u;
      dirs[3 * i + k] = (float)((s >> 8) / 16777216.0 * 2.0 - 1.0);
    }
    inten[i] = 0.5f;
    temp[i] = 5000.0f + (float)i;
  }
  double* cube = calloc((size_t)orc_cubemap_texels(N0) * 4, sizeof(double));
  if (orc_cubemap_build(dirs, inten, temp, NS, N0, cube)) bad = 1;

  /* whole pixels: exact mode, table mode and marching, four threads */
  orc_view v;
  memset(&v, 0, sizeof(v));
  v.r_s = 1.0;
  v.cam_pos[0] = 15.0;
  v.cam_pos[2] = 2.0;
  double rot[9] = {0, 1, 0, 0, 0, 1, 1, 0, 0}; /* e_w, e_h, e_d: looking along -x */
  memcpy(v.cam_rot, rot, sizeof(rot));
  v.fov_y = 1.0;
  v.width = v.height = 8;
  v.disc_r_in = 3.0;
  v.disc_r_out = 12.0;
  v.disc_T0 = 1e4;
  v.disc_T_exp = -0.75;
  v.disc_opacity = 1.0;
  v.k_disc = 1e-7;
  v.k_star = 1.0;
  int32_t quads[32];
  int nq = 0;
  for (int y = 0; y < 8; y += 2)
    for (int x = 0; x < 8; x += 2) {
      quads[2 * nq] = x;
      quads[2 * nq + 1] = y;
      ++nq;
    }
  orc_pixel* px = calloc((size_t)4 * nq, sizeof(orc_pixel));
  if (orc_render_quads(&v, cube, N0, NULL, 0, NULL, 0, 0, quads, nq, px, 4)) bad = 1;
  if (orc_render_quads(&v, cube, N0, D, dn, U, ne, nphi, quads, nq, px, 4)) bad = 1;
  if (orc_render_quads_m(&v, cube, N0, 50, quads, nq, px, 4)) bad = 1;
  for (int i = 0; i < 4 * nq; ++i) FINITE(px[i].rgb[0] + px[i].rgb[1] + px[i].rgb[2]);
  double parts[6] = {5.0, 6.0, 0.3, 8.0, 9.0, 2.0};
  v.disc_density = 1;
  v.n_particles = 2;
  v.particles = parts;
  v.time = 100.0;
  if (orc_render_quads_t(&v, cube, N0, D, Dt, dn, U, Ut, ne, nphi, quads, nq, px, 4)) bad = 1;
  FINITE(orc_ellipk(0.5));

  /* area sources: the map's levels, the filter and the exact mean, then whole pixels */
  float it[6 * 8 * 8 * 2];
  for (int i = 0; i < 6 * 8 * 8; ++i) {
    it[2 * i] = 0.1f + (float)(i % 13) * 0.05f;
    it[2 * i + 1] = 4000.0f + (float)(i % 5) * 500.0f;
  }
  double* area = calloc((size_t)orc_area_texels(8) * 2, sizeof(double));
  if (orc_area_build(it, 8, area)) bad = 1;
  double dd[3] = {0.3, 0.9, -0.2}, aw[3] = {0.2, 0.0, 0.1}, ah[3] = {0.0, 0.05, 0.4}, A, B;
  orc_area_filter(area, 8, dd, aw, ah, &A, &B);
  FINITE(A + B);
  orc_area_exact(area, 8, dd, aw, ah, &A, &B);
  FINITE(A + B);
  v.disc_density = 0;
  v.area = area;
  v.area_n0 = 8;
  v.area_exact = 1;
  v.k_area = 1.0;
  if (orc_render_quads(&v, cube, N0, D, dn, U, ne, nphi, quads, nq, px, 4)) bad = 1;
  for (int i = 0; i < 4 * nq; ++i) FINITE(px[i].rgb[0] + px[i].area_exact_A);
  free(area);

  /* band maps and the colour shift (exact and through a small table, several threads) */
  float rgbx[6 * 8 * 8 * 4];
  for (int i = 0; i < 6 * 8 * 8; ++i) {
    rgbx[4 * i] = 0.2f + (float)(i % 7) * 0.03f;
    rgbx[4 * i + 1] = 0.25f + (float)(i % 3) * 0.05f;
    rgbx[4 * i + 2] = 0.15f + (float)(i % 11) * 0.02f;
    rgbx[4 * i + 3] = 0.0f;
  }
  double* bands = calloc((size_t)orc_area_texels(8) * 3, sizeof(double));
  if (orc_area_build_bands(rgbx, 8, bands)) bad = 1;
  double cs[3];
  orc_color_shift(0.3, 0.35, 1.7, cs);
  FINITE(cs[0] + cs[1] + cs[2]);
  double* ctab = calloc(5 * 5 * 5 * 3, sizeof(double));
  orc_cshift_table(5, 5, 5, ctab, 3);
  v.area = bands;
  v.area_bands = 1;
  v.ct_n[0] = v.ct_n[1] = v.ct_n[2] = 5;
  v.ctable = ctab;
  if (orc_render_quads(&v, cube, N0, D, dn, U, ne, nphi, quads, nq, px, 4)) bad = 1;
  for (int i = 0; i < 4 * nq; ++i) FINITE(px[i].rgb[0] + px[i].area_exact_A);
  /* a band-colour star map through the same table */
  float srgb[3 * 40];
  for (int i = 0; i < 3 * 40; ++i) srgb[i] = 0.01f + (float)(i % 9) * 0.02f;
  double* bcube = calloc((size_t)orc_cubemap_texels(N0) * 5, sizeof(double));
  if (orc_cubemap_build_bands(dirs, srgb, 40, N0, bcube)) bad = 1;
  v.star_bands = 1;
  if (orc_render_quads(&v, bcube, N0, D, dn, U, ne, nphi, quads, nq, px, 4)) bad = 1;
  for (int i = 0; i < 4 * nq; ++i) FINITE(px[i].rgb[0] + px[i].star_A);
  v.star_bands = 0;
  free(bcube);
  free(bands);
  free(ctab);

  /* post-process */
  double img[8 * 8 * 4], out[8 * 8 * 4], w[4] = {0.7, 0.2, 0.07, 0.03};
  for (int i = 0; i < 8 * 8 * 4; ++i) img[i] = (i % 7) * 0.1;
  if (orc_bloom(img, 8, 8, 3, w, out)) bad = 1;
  uint8_t codes[8 * 8 * 4];
  double scaled[8 * 8 * 3];
  if (orc_tonemap(out, 64, 2.0, codes, scaled)) bad = 1;

  free(px);
  free(cube);
  free(D);
  free(U);
  free(Dt);
  free(Ut);
  if (!bad) printf("oracle sanitizer run ok\n");
  return bad;
}
