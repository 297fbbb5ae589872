/*
 * libbh -- per-pixel constant-time beam tracer for non-rotating black holes on AMD
 * Instinct MI355X (gfx950), after E. Bruneton, "Real-time High-Quality Rendering of
 * Non-Rotating Black Holes" (arXiv 2010.08735).
 *
 * Units follow Section 3.1: every length is given in the same unit as r_s (the horizon
 * radius) and is divided by r_s inside the library; the speed of light is 1.
 *
 * Conventions shared by every entry point
 *   - Return value: a bh_status.  Arguments are validated before any device work; on error
 *     nothing is launched and bh_last_error() describes the problem (thread-local string,
 *     owned by the library, valid until the next failing call on the same thread).
 *   - Pointers named *_dev are device pointers (HIP global memory); the caller owns them
 *     and must keep them alive until the work that uses them has completed on the stream.
 *   - Pointers named host_* are host pointers.
 *   - hip_stream is a hipStream_t (may be NULL for the null stream).  Work is enqueued on
 *     that stream and the call returns without waiting, unless stated otherwise.
 *   - Handles (bh_ctx, bh_tables, bh_stars) are owned by the library.  Tables and star
 *     maps are reference counted and shared by key: a second request with the same key
 *     returns the resident handle with its count incremented; bh_release_* drops it.
 *     Tables are keyed by their parameters, star maps by their content (a hash of the
 *     three star arrays, the star count, the face size and the texel format).
 *   - Thread safety: every call is safe to make concurrently on one context.
 */
#ifndef BH_H
#define BH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BH_OK = 0,
  BH_EINVAL = 1,     /* invalid argument (geometry, sizes, NaN, null pointer)          */
  BH_ENOMEM = 2,     /* HBM budget exceeded or a device allocation failed              */
  BH_EDEVICE = 3,    /* HIP runtime error                                               */
  BH_EAGAIN = 4,     /* serving queue full; retry later                                 */
  BH_ENOTFOUND = 5,  /* unknown ticket                                                  */
  BH_ECANCELED = 6   /* request cancelled (context destroyed before completion)         */
} bh_status;

typedef struct bh_ctx bh_ctx;
typedef struct bh_tables bh_tables;
typedef struct bh_stars bh_stars;
typedef struct bh_particles bh_particles;

/* ---- context ----------------------------------------------------------------------- */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device memory the
 * library itself allocates (tables, star maps, band table, serving outputs); 0 = no cap.
 * Builds the blackbody band table on the device before returning. */
bh_status bh_create(int device, uint64_t hbm_budget_bytes, bh_ctx** out);
/* Wait for outstanding work, cancel queued requests, free every resource. */
void bh_destroy(bh_ctx* ctx);
/* The calling thread's last failure message (owned by the library, valid until this thread's
 * next failing call).  ctx may be NULL: messages are kept per thread, not per context. */
const char* bh_last_error(const bh_ctx* ctx);
/* Device bytes currently allocated by the library on this context. */
uint64_t bh_bytes_in_use(const bh_ctx* ctx);
/* Release any handle the library returned (tables, star maps, area maps, particles, bloom
 * pyramids): the same as the release call of its type.  Tables and star maps are
 * reference-counted (one release per build call that returned them); the others are
 * freed.  BH_EINVAL for NULL or any address that is not a live handle of this library
 * (the library keeps a registry of live handles and never reads through the address
 * before finding it there). */
bh_status bh_release(void* handle);

/* ---- precomputed tables (Section 3.3.2 "Escape angle", 3.3.3 "Intersections",
 *      Algorithm 1 Precompute, Appendix A) -------------------------------------------- */

#define BH_TAB_FP32 0       /* integrate in FP32 everywhere                              */
#define BH_TAB_FP64_BAND 1  /* FP64 while |u - 2/3| < fp64_band, FP32 elsewhere           */
#define BH_TAB_FP64_ALL 2   /* FP64 everywhere                                           */

typedef struct {
  int32_t d_n;        /* deflection table is d_n x d_n (even, >= 8; paper: 512)          */
  int32_t u_ne;       /* intersection table columns along e (paper: 64)                  */
  int32_t u_nphi;     /* intersection table rows along phi (paper: 32)                   */
  int32_t precision;  /* BH_TAB_*                                                        */
  double fp64_band;   /* half-width of the FP64 band around u = 2/3 (0.05)               */
  double step;        /* integration step in phi (RK4; 0 selects 2e-3)                   */
} bh_table_params;

/* Integrate the orbit equation u'' = 3/2 u^2 - u on the device for every table column
 * and fill the deflection table D(e,u) = phi - atan2(u, du/dphi) (incoming branch) and
 * the intersection table U(e,phi) = u (phi < pi, 1 after the ray falls in), both FP32,
 * at the texel centres k/(N-1) of the Appendix A mappings, and their time channels
 * (Algorithm 1 Precompute stores t beside D and U): e * tau, where the regularised time
 * tau = t - ln(u/(1-u)) + 1/u (+ a constant per ray) is finite along rays from infinity.
 * Shared by parameter key.
 * Synchronises hip_stream before returning (the tables are then ready for any stream). */
bh_status bh_precompute_tables(bh_ctx* ctx, const bh_table_params* p, void* hip_stream,
                               bh_tables** out);
/* Copy the tables to the host: host_D d_n*d_n floats, row j (u coordinate) major, column
 * i (e coordinate) minor; host_U u_nphi*u_ne floats, row (phi) major.  Either may be NULL.
 * Blocking. */
bh_status bh_tables_download(const bh_tables* t, float* host_D, float* host_U);
/* Copy the time channels (e * tau) in the layouts of D and U.  Either may be NULL. */
bh_status bh_tables_download_time(const bh_tables* t, float* host_Dt, float* host_Ut);
bh_status bh_release_tables(bh_tables* t);

/* ---- disc particles (Appendix B) --------------------------------------------------------- */

/* Procedural particles of an animated disc: n triples (r_peri, r_apo, phi0) in host memory
 * (units of r_s; 3 <= r_peri <= r_apo; phi0 the orbital phase at t = 0).  Each particle
 * point a in [0, 2 pi) follows the quasi-circular orbit u = u1 + (u2 - u1)
 * sin^2(pi / (4K) (a + phi(t)) sqrt(u3 - u1)), phi(t) = sqrt(ubar^3 / 2) t + phi0
 * (u1 = 1/r_apo, u2 = 1/r_peri, u3 = 1 - u1 - u2, K = K(sqrt((u2-u1)/(u3-u1)))), and a hit
 * point at distance d from the particle centre gets density (1 - d^2)^2 for d < 1.
 * The library copies the records; n <= 65536.  BH_EINVAL for bad values. */
bh_status bh_create_particles(bh_ctx* ctx, const double* host_triples, int32_t n,
                              bh_particles** out);
bh_status bh_release_particles(bh_particles* p);

/* ---- bloom (Section 3.4.3 "Lens glare effects") ---------------------------------------
 * A point spread function approximated by small-support filters on the mipmaps of the
 * final (linear, not yet tone-mapped) image:
 *   P_0 = I;  P_k = 2x2 box average of P_{k-1} (ceil(n/2) pixels per axis, source indices
 *   clamped to the last row / column), k = 1 .. levels;
 *   U_levels = w_levels P_levels;  U_k = w_k P_k + up(U_{k+1});  O = w_0 I + up(U_1),
 * where up() doubles the resolution bilinearly (fine pixel x samples the coarse grid at
 * x/2 - 1/4, indices clamped to the edge).  Level k's kernel spans about 2^k pixels; the
 * weights w_0 .. w_levels shape the point spread function, and with sum 1 the flux of an
 * interior source is kept.  The paper does not print its filter bank; this is one reading.
 *
 * bh_bloom_create allocates the pyramid for one image size (counted in the HBM budget):
 * width, height in [1, 65536], levels in [0, 16].  bh_bloom_apply reads in_rgba_dev and
 * writes out_rgba_dev (both device, width*height float4, row-major; they may be the same
 * buffer), with weights[0 .. levels] in host memory (finite; copied at the call).  Calls on
 * one handle must not overlap in time (they share the pyramid): issue them on one stream,
 * or use one handle per stream.  bh_bloom_release frees the pyramid after the device has
 * finished with it. */
typedef struct bh_bloom bh_bloom;
bh_status bh_bloom_create(bh_ctx* ctx, int32_t width, int32_t height, int32_t levels,
                          bh_bloom** out);
bh_status bh_bloom_apply(bh_bloom* b, const float* weights, const float* in_rgba_dev,
                         float* out_rgba_dev, void* hip_stream);
bh_status bh_bloom_release(bh_bloom* b);

/* ---- display encoding: the tone mapping after the glare pass (Section 3.4.3) -----------
 *
 * The paper applies its glare pass before tone mapping and prints no operator; this is one
 * reading.  Per colour channel c of a linear pixel: x = exposure * c; y = 1 - exp(-x) (0 for
 * x <= 0 and for NaN); v = the sRGB transfer function of y (IEC 61966-2-1: 12.92 y for
 * y <= 0.0031308, else 1.055 y^(1/2.4) - 0.055); code = floor(255 v + 1/2).  Alpha is
 * encoded as 255.  An encoded pixel is 4 bytes R, G, B, A in memory order (one uint32).
 * The codes are computed in FP32 with hardware exp2 / log2: a code can differ from the
 * exactly rounded one only where 255 v + 1/2 lies within 5e-4 of an integer (the computed
 * value stays within 2e-4 of the exact one).
 *
 * bh_tonemap encodes in_rgba_dev (device, width*height float4, row-major) into
 * out_rgba8_dev (device, width*height uint32); width, height in [1, 65536] with
 * width * height <= 2^31; exposure finite
 * and > 0.  bh_bloom_apply_display runs bh_bloom_apply's glare pass on in_rgba_dev and writes
 * only the encoding of its result to out_rgba8_dev (the linear result is not stored), with
 * the same weights, handle and stream rules.  For both, the output must not overlap the
 * input (BH_EINVAL). */
bh_status bh_tonemap(bh_ctx* ctx, const float* in_rgba_dev, uint32_t* out_rgba8_dev,
                     int32_t width, int32_t height, float exposure, void* hip_stream);
bh_status bh_bloom_apply_display(bh_bloom* b, const float* weights, float exposure,
                                 const float* in_rgba_dev, uint32_t* out_rgba8_dev,
                                 void* hip_stream);

/* ---- star map (Section 3.3.2 "Emitted light") -------------------------------------- */

#define BH_TEXEL_FP16 0     /* RGBA16F texels: I (per-level power-of-two scale), T, p_u, p_v */
#define BH_TEXEL_FP32 1     /* RGBA32F texels                                             */


/* dir_xyz_dev: n x 3 directions (any length > 0), intensity_dev: n emitted intensities
 * summed over the three bands (>= 0), temperature_dev: n blackbody temperatures in K, all
 * device arrays; face_size: level-0 texels per cube face edge, a power of two <= 8192;
 * texel_format: BH_TEXEL_*.
 * Splat the stars into a cube map (one texel holds the intensity sum, the
 * intensity-weighted mean temperature and the intensity-weighted mean position of the
 * stars inside it) and build every mip level with the same rule.  Deterministic.
 * A field whose arrays hash to a resident map of the same star count, face size and
 * format returns that map (its count incremented) without building anything.
 * Synchronises hip_stream before returning. */
bh_status bh_build_stars(bh_ctx* ctx, const float* dir_xyz_dev, const float* intensity_dev,
                         const float* temperature_dev, int64_t n, int32_t face_size,
                         int32_t texel_format, void* hip_stream, bh_stars** out);
/* Stars of any colour (Section 3.4.2: the emitted colour of the star gather received as
 * (X + Y + Z) C(xy, D), here in the band basis of bh_build_area_bands).  rgb_dev: n x 3
 * band intensities (R, G, B) per star, each finite and >= 0 (a star with R + G + B = 0 is
 * left out), device array; dir_xyz_dev, face_size, texel_format as bh_build_stars.  A
 * texel holds the band sums of its stars and their position inside the texel weighted by
 * S = R + G + B; mips combine the four children by the same rule.  FP16 texels store
 * (R, G, B) / scale_L (the per-level power of two of the (I, T) format, from the level's
 * largest band value), p_u, p_v and three zero halves (16 bytes); FP32 texels the same
 * eight values (32 bytes).  A pixel receives k_star x (Omega / Omega') x S x
 * C_b(r, g, D_cam), S the footprint's tent-weighted band sum and (r, g) = (R, G) / S its
 * chromaticity, through the context's colour-shift table (built with the first band map,
 * as for bh_build_area_bands).  Shared by content like bh_build_stars (a band map never
 * shares a key with an (I, T) map); BH_EINVAL for an invalid band value (the check runs on
 * the device); released with bh_release_stars.  Synchronises hip_stream. */
bh_status bh_build_star_bands(bh_ctx* ctx, const float* dir_xyz_dev, const float* rgb_dev,
                              int64_t n, int32_t face_size, int32_t texel_format,
                              void* hip_stream, bh_stars** out);

/* Copy mip level `level` as float (face, y, x, [I, T, p_u, p_v]) to host_texels
 * (6 * (face_size >> level)^2 * 4 floats); for a band map as float (face, y, x,
 * [R, G, B, p_u, p_v, 0, 0, 0]) (8 floats per texel).  Blocking. */
bh_status bh_stars_download(const bh_stars* s, int32_t level, float* host_texels);
bh_status bh_release_stars(bh_stars* s);

/* ---- area sources (Section 3.3.2 "Emitted light"; Section 3.4.1, closing note) -------
 * Extended sources such as nebulae and galaxies, stored in a cube map that is read over
 * each pixel's footprint with anisotropic filtering (unlike point stars, whose light the
 * star map's gather keeps sharp).  A texel holds a radiance I (summed over the three
 * bands, in the units of k_star's star intensities) and a blackbody colour temperature T.
 * A pixel receives k_area x A x L_b(D_cam T_pix) / sum_b L_b(T_pix): A and A T_pix are the
 * footprint means of I and I T, D_cam the camera's Doppler factor for static sources; no
 * lensing amplification Omega / Omega' applies (the beam's subtended area changes in
 * inverse proportion).  The filter: the footprint is the parallelogram of directions
 * d' + w d_w d' + h d_h d', |w|, |h| <= 1/2 (the screen-space differences of the escape
 * direction over the pixel's 2x2 quad); an N x 2 grid of probes (N = ceil(2 l_major /
 * l_minor) in [1, 16], lengths in level-0 texels) reads the box mip pyramid trilinearly at
 * level log2(max(l_major / N, l_minor / 2)) - 1, each probe on the face of its own
 * direction.  Quads with a captured member receive no area light (as for stars). */
typedef struct bh_area bh_area;
/* texels_dev: device array of 6 * face_size^2 (I, T) float pairs, laid out as the star
 * map (face 2k + (d_k < 0), column from U = d_{(k+1)%3} / |d_k|, row from V =
 * d_{(k+2)%3} / |d_k|, row-major per face), I >= 0 and T >= 0 finite; face_size a power
 * of two in [1, 4096].  Builds the map and its mip levels (box means of I and I T) on
 * hip_stream and synchronises it; texels_dev may be freed afterwards.  BH_EINVAL for a bad
 * size, a NULL pointer or an invalid texel (the check runs on the device).  Every call
 * builds a new map; bh_release_area frees it (callers must not release a map that queued
 * work still reads). */
bh_status bh_build_area(bh_ctx* ctx, const float* texels_dev, int32_t face_size,
                        void* hip_stream, bh_area** out);
/* Light of any colour (Section 3.4.2, the colour-shift table C(xy, D)): an area map whose
 * texels hold band radiances (R, G, B) instead of (I, T).  A pixel receives
 * k_area x S x C_b(r, g, D_cam), S the footprint mean of R + G + B and (r, g) its
 * chromaticity (R, G) / S, from a table of the received band radiances per unit emitted
 * band sum.  Each chromaticity stands for one spectrum B_T (1 - a1 A1 - a2 A2): T the
 * blackbody temperature with the same blue-to-red band ratio (1e3 .. 1e6 K), A1, A2
 * Gaussian absorption bands at 450 and 650 nm (width 30 nm), a1, a2 in [-8, 1] fixed by
 * the chromaticity; its received spectrum is D^5 I(D lambda).  Blackbody colours shift
 * exactly as the (I, T) maps do (up to the table's interpolation).  The table has
 * BH_CSHIFT_N^3 nodes, r = i / (N - 1), g = j / (N - 1), log2 D = -3 + 6 k / (N - 1), and
 * holds log2 C_b (each C_b at least 2^-100); it is read trilinearly, linearly in 1 / D
 * along D, coordinates clamped; it is built on the device (FP64 quadrature) with a
 * context's first band map and kept until bh_destroy (32 MiB, counted in the budget).
 * rgbx_dev: device array of 6 * face_size^2 float4 (R, G, B, unused), laid out as in
 * bh_build_area, R, G, B >= 0 finite.  Otherwise as bh_build_area (mips are box means of
 * R, G and B); released with bh_release_area. */
#define BH_CSHIFT_N 128
bh_status bh_build_area_bands(bh_ctx* ctx, const float* rgbx_dev, int32_t face_size,
                              void* hip_stream, bh_area** out);
/* Copy the colour-shift table to host (BH_CSHIFT_N^3 float4 (log2 C_R, log2 C_G, log2 C_B,
 * 0), node ((i N + j) N + k)), building it first if the context has none.  Blocking. */
bh_status bh_color_shift_table_download(bh_ctx* ctx, float* host);
/* Copy mip level `level` to host_texels: (face, y, x, [I, I T]), 6 * (face_size >>
 * level)^2 * 2 floats, or for a band map (face, y, x, [R, G, B, 0]), 4 floats per texel.
 * Blocking. */
bh_status bh_area_download(const bh_area* area, int32_t level, float* host_texels);
bh_status bh_release_area(bh_area* area);

/* ---- rendering (Sections 3.2-3.4) ---------------------------------------------------- */

#define BH_T_POWER 0  /* T' = T0 (r' / 3 r_s)^T_exp                                        */
#define BH_T_PAPER 1  /* T'^4 proportional to u^3 (1 - sqrt(3u)) (Section 3.3.3), peak T0  */

typedef struct {
  double r_s;           /* > 0                                                            */
  double cam_pos[3];    /* Cartesian camera position, |cam_pos| > r_s (Section 5)         */
  double cam_vel[3];    /* camera velocity seen by the static observer at cam_pos, along
                           the Cartesian axes, |v| < 1                                     */
  double cam_rot[9];    /* rows e_w, e_h, e_d (orthonormal) of the camera in its own
                           (boosted) frame; the camera looks along -e_d                    */
  double fov_y;         /* vertical field of view, radians, (0, pi)                       */
  int32_t width, height; /* pixels, each in [1, 65536], width * height <= 2^31           */
  double disc_r_in;     /* >= 3 r_s (innermost stable circular orbit, Section 3.3.3)       */
  double disc_r_out;    /* > disc_r_in                                                     */
  int32_t disc_T_law;   /* BH_T_*                                                          */
  int32_t pad0;
  double disc_T0;       /* K                                                               */
  double disc_T_exp;    /* exponent of the power law (-0.75)                              */
  double disc_opacity;  /* front-to-back opacity of each disc crossing, [0, 1]             */
  double k_disc;        /* exposure applied to disc band radiances (W m^-2 sr^-1)         */
  double k_star;        /* exposure applied to star intensities                           */
  const bh_stars* stars;/* NULL: black sky                                                 */
  /* animated disc (Section 3.3.3 "Emitted light", Appendix B) */
  int32_t disc_density; /* BH_DENSITY_UNIFORM, or BH_DENSITY_PARTICLES: each crossing's
                           opacity is min(1, disc_opacity * particle density) at the
                           crossing's position and retarded time                          */
  int32_t pad1;
  double time;          /* the camera's coordinate time (units of r_s / c)                */
  const bh_particles* particles; /* required with BH_DENSITY_PARTICLES                    */
  const bh_area* area;  /* area-source sky (nebulae, galaxies), or NULL                   */
  double k_area;        /* exposure applied to area radiances, finite                      */
} bh_view;

#define BH_DENSITY_UNIFORM 0
#define BH_DENSITY_PARTICLES 1

/* AOV record written per pixel when aov_dev is not NULL (4 floats):
 *   [0] escape angle delta' (radians, +inf if the beam falls into the hole)
 *   [1] u of the first disc crossing along the beam (0 if none)
 *   [2] u of the second disc crossing (0 if none)
 *   [3] bit pattern (reinterpret as uint32): bit0 captured, bit1 crossing before the
 *       apsis, bit2 crossing after the apsis, bit3 star term zeroed (a member of the 2x2
 *       quad is captured), bit4 degenerate beam plane, bit5 ray marching ran out of steps
 *       (the beam is drawn as captured), bits 8-15 mip level (255: none). */
#define BH_AOV_CAPTURED 1u
#define BH_AOV_CROSS0 2u
#define BH_AOV_CROSS1 4u
#define BH_AOV_STAR_ZEROED 8u
#define BH_AOV_DEGENERATE 16u
#define BH_AOV_UNFINISHED 32u

/* Render one view: out_rgba_dev receives width*height float4 (R, G, B, 1) in row-major
 * order, row 0 at the top; colour = k_disc x disc band radiances composited front to back
 * over k_star x lensed, Doppler-shifted star light plus the view's area-source light.
 * aov_dev may be NULL. */
bh_status bh_render(bh_ctx* ctx, const bh_tables* t, const bh_view* v, float* out_rgba_dev,
                    float* aov_dev, void* hip_stream);

/* The ablation of Section 5 (method M3 of Table 1): render v with TraceRay replaced by a
 * numerical integration of the orbit equation u'' = 3/2 u^2 - u (eq. rayequation), and
 * everything else unchanged.  Classic fourth-order Runge-Kutta in phi with the constant
 * step 2 pi / max_steps and at most max_steps steps (one full turn of the beam plane);
 * inside a step u(phi) is the cubic Hermite interpolant of the end states, which places the
 * escape angle (its first root) and the disc crossings (its value at alpha + m pi).  A beam
 * still travelling after max_steps steps is drawn as captured and flagged
 * BH_AOV_UNFINISHED.  A beam within 1e-6 of the radius moves along r only (escapes at
 * delta' = delta outward, falls in inward).  Needs no tables.  max_steps in [3, 1048576]; the view's disc must be
 * BH_DENSITY_UNIFORM (marching carries no time channels).  Same output layout as
 * bh_render. */
bh_status bh_render_march(bh_ctx* ctx, const bh_view* v, int32_t max_steps, float* out_rgba_dev,
                          float* aov_dev, void* hip_stream);

/* Render n views of any sizes in one persistent launch (work list of tiles, replayed as
 * a HIP graph when the same shapes repeat).  outs_dev[i] has views[i].width*height float4.
 * Per pixel the result is bitwise identical to bh_render.  BH_EINVAL when the views' tiles
 * (each view padded to whole tiles of the selected configuration) hold 2^32 pixels or more. */
bh_status bh_render_batch(bh_ctx* ctx, const bh_tables* t, const bh_view* views, int32_t n,
                          float* const* outs_dev, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): bh_render_batch without any allocation.
 * The launch's view records, tile runs and work counter live in a fixed device array of
 * the library (256 B + 512 x 336 B = 168 KiB, one per GPU, held until the process ends), so n is at
 * most BH_NOALLOC_MAX_VIEWS (BH_EINVAL above); the records are uploaded through pinned host
 * memory that bh_create sets up, and the kernels are launched directly (no graph is
 * built).  Same kernels as bh_render_batch with the same tile configuration and launch
 * form, so the same bits.  Every call on one GPU (any context) uses the same array: calls
 * in order on one stream are safe, calls that overlap on one GPU (other streams or threads)
 * race. */
#define BH_NOALLOC_MAX_VIEWS 512
bh_status bh_render_batch_noalloc(bh_ctx* ctx, const bh_tables* t, const bh_view* views,
                                  int32_t n, float* const* outs_dev, void* hip_stream);

/* Tile configuration of the render kernels (the autotuner chooses among these). */
typedef struct {
  int32_t tile_w, tile_h;  /* pixels per workgroup tile (multiples of 8)                  */
  int32_t waves;           /* wavefronts per workgroup                                    */
  int32_t ppt;             /* pixels per thread                                           */
} bh_tile_config;
int32_t bh_tile_config_count(void);
bh_status bh_tile_config_get(int32_t index, bh_tile_config* out);
/* Select the tile configuration used by bh_render / bh_render_batch and a later
 * bh_serve_start (-1: the built-in default, 8x8 tiles of one pixel per thread, index 3) */
bh_status bh_set_tile_config(bh_ctx* ctx, int32_t index);
/* Select the launch form of the batched calls: 1 = persistent workgroups claiming tiles
 * from an atomic counter, 0 = one workgroup per tile (the default). */
bh_status bh_set_batch_form(bh_ctx* ctx, int32_t persistent);
/* Time every tile configuration with both batched launch forms (persistent workgroups
 * pulling tiles from an atomic counter, or one workgroup per tile) on the given views and
 * keep the fastest.  best_index = 2 * config + persistent; ms_per_config receives
 * 2 * bh_tile_config_count() timings in the same order (or NULL). */
bh_status bh_autotune(bh_ctx* ctx, const bh_tables* t, const bh_view* views, int32_t n,
                      float* const* outs_dev, int32_t reps, int32_t* best_index,
                      float* ms_per_config);

/* ---- serving: continuous batching -------------------------------------------------- */

typedef struct {
  int32_t max_queue;          /* submissions beyond this return BH_EAGAIN                */
  int32_t max_inflight_launches; /* launches kept in flight on the serving stream (6)    */
  int64_t max_tiles_per_launch;  /* tiles per launch; bigger requests are split (262144);
                                    at most 4194303 (BH_EINVAL above: a launch covers fewer
                                    than 2^32 work-items)                                  */
} bh_serve_params;

/* Start the serving scheduler thread on its own stream (call once per context). */
bh_status bh_serve_start(bh_ctx* ctx, const bh_serve_params* p);
/* Queue a frame; returns at once with a ticket.  out_rgba_dev may be NULL, in which case
 * the library allocates the image inside the HBM budget (admission waits for room) and
 * bh_ticket_image returns it; it is freed by bh_ticket_free.  The view record is copied,
 * but the handles it names (tables, star map, particles) and a caller-owned output image
 * must stay alive until bh_poll reports the frame done. */
bh_status bh_submit(bh_ctx* ctx, const bh_tables* t, const bh_view* v, float* out_rgba_dev,
                    uint64_t* ticket);
/* done = 1 when the frame is complete on the device (or has failed); latency_s =
 * completion - submit.  Returns the request's status: BH_OK, BH_ENOMEM (its library image
 * can never fit: nothing else holds or pools budget), BH_EDEVICE (its launch failed) or
 * BH_ECANCELED (the context was destroyed first); BH_ENOTFOUND for an unknown ticket. */
bh_status bh_poll(bh_ctx* ctx, uint64_t ticket, int32_t* done, double* latency_s);
/* Image of a finished ticket that was submitted with out_rgba_dev = NULL. */
bh_status bh_ticket_image(bh_ctx* ctx, uint64_t ticket, float** out_rgba_dev);
/* Forget a finished ticket.  A library-allocated image goes back to the serving pool and
 * is reused by later frames at once, so the caller must first finish every device
 * operation that reads it (for instance synchronize the stream of its copy-out). */
bh_status bh_ticket_free(bh_ctx* ctx, uint64_t ticket);
/* Block until every submitted request is complete. */
bh_status bh_serve_drain(bh_ctx* ctx);

/* ---- unit-level entry points used by the tests ------------------------------------------ */

/* TraceRay (Algorithm 1) alone for n rays given as 5 floats each
 * [u = 1/p^r, delta, alpha, u_ic, u_oc]; writes 4 floats per ray in the AOV layout.
 * n in [0, 2^31] here and in bh_trace_rays_timed, bh_march_rays and bh_band_eval. */
bh_status bh_trace_rays(bh_ctx* ctx, const bh_tables* t, const float* rays_dev, int64_t n,
                        float* out_dev, void* hip_stream);
/* The same, also writing 4 floats per ray to out_time_dev: the retarded times of the two
 * crossings in beam order (coordinate time from the crossing to the camera, Algorithm 1)
 * and, as floats, the integers m_0, m_1 placing each crossing at beam-plane angle
 * alpha + m pi (0 where there is no crossing). */
bh_status bh_trace_rays_timed(bh_ctx* ctx, const bh_tables* t, const float* rays_dev, int64_t n,
                              float* out_dev, float* out_time_dev, void* hip_stream);
/* The ray marching of bh_render_march alone for n rays in the bh_trace_rays layout. */
bh_status bh_march_rays(bh_ctx* ctx, const float* rays_dev, int64_t n, int32_t max_steps,
                        float* out_dev, void* hip_stream);
/* Measurement: render v once (into out_rgba_dev) with a variant of the render kernel that
 * marks every star-map texel the footprints visit, and return how many distinct texels were
 * visited (the star-map bytes one frame must read at least once) and, if req_bytes is not
 * NULL, the bytes all pixels request through the caches (table and band-table fetches,
 * occupancy words, texels, level records, image and AOV stores).  The frame is rendered
 * without the view's area-source map (none of its light, texels or bytes).  The view's star
 * map must be an (I, T) map (BH_EINVAL for a band-colour map).  Blocking. */
bh_status bh_footprint_texels(bh_ctx* ctx, const bh_tables* t, const bh_view* v,
                              float* out_rgba_dev, uint64_t* texels, uint64_t* req_bytes);
/* Measurement: the read bandwidth of data held in the L2 caches.  Every workgroup (8 per
 * CU) streams coalesced 16-byte reads over 256 KiB of a zero-filled device buffer of
 * window_bytes (a power of two in [4 KiB, 4 MiB], so that it fits one XCD's L2), wrapping
 * around; after three untimed passes, bytes_per_s = bytes read / time of `reps` launches.
 * Blocking. */
bh_status bh_probe_l2_read(bh_ctx* ctx, int64_t window_bytes, int32_t reps, double* bytes_per_s);
/* Blackbody band table: n entries of 4 floats [log2 L_R, log2 L_G, log2 L_B,
 * log2 (L_R + L_G + L_B)] at log2 T = x0 + k dx.  Blocking. */
bh_status bh_band_table_info(const bh_ctx* ctx, int32_t* n, float* x0, float* dx);
bh_status bh_band_table_download(const bh_ctx* ctx, float* host_lut);
/* Band radiances (W m^-2 sr^-1) through the band table for n temperatures, 3 floats each. */
bh_status bh_band_eval(bh_ctx* ctx, const float* temps_dev, int64_t n, float* out_dev,
                       void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
