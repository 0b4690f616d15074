/*
 * rt.h -- C ABI of the MI355X (gfx950) backward null-geodesic ray tracer.
 *
 * The library traces one null geodesic per observer-screen pixel backward
 * through a stationary, axisymmetric, Kerr-like rotating spacetime and returns
 * the equatorial-crossing (lensing-band) counts, the transfer maps of the first
 * three crossings and the redshifted thin-disc intensity, following
 * M. Fathi, "Adaptive ray tracing, image diagnostics, and photon ring
 * signatures of rotating dark-matter-dressed black holes":
 *   - spacetimes: Sec. 2, eqs. (9), (13), (23)-(31) (Kerr, Einasto-type and
 *     cored-NFW seeds in Kerr-like Boyer-Lindquist form);
 *   - geodesics: Sec. 3.1, Hamilton's equations (46)-(47), eqs. (57)-(62);
 *   - screen: Sec. 3.2, ZAMO tetrad eqs. (63)-(68), screen map eqs. (70)-(74);
 *   - events: Sec. 3.3, eqs. (75)-(77); lensing bands Sec. 4.2, eqs. (80)-(81);
 *     transfer maps Sec. 4.3, eq. (82);
 *   - emission: Sec. 5.1-5.2, eqs. (85)-(91);
 *   - image reductions: Sec. 6.2, flux and centroid; Sec. 6.4, eq. (108)-(109).
 *
 * Units: M = 1 throughout (eq. (1)).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers on the current HIP device, owned
 *     by the caller; the library never frees them.  Parameter structs are host
 *     memory, read before the call returns.
 *   - Every call is asynchronous on `hip_stream` (a hipStream_t; NULL means the
 *     null stream).  Outputs are valid once that stream has reached the point
 *     of the call.  Scratch memory (work-queue counters and intermediate
 *     buffers) is allocated stream-ordered and released before the work
 *     completes.
 *   - Return value: RT_OK (0) on success, a negative RT_ERR_* code otherwise;
 *     rt_last_error() then describes the failure (thread-local string).  On an
 *     error nothing has been launched.  The library never aborts or prints.
 *   - Equatorial crossings: Boyer-Lindquist theta is continued through the
 *     poles (a ray with l = 0, from a pixel with X = 0, passes over the axis),
 *     so the equator is theta = pi/2 (mod pi); a crossing where theta = -pi/2
 *     (mod 2 pi) reports its azimuth as phi + pi (the same point).
 *   - Screen layout: pixel (ix, iy), 0 <= ix < nx, 0 <= iy < ny, sits at the
 *     centre X = x_min + (ix + 1/2)(x_max - x_min)/nx,
 *                Y = y_min + (iy + 1/2)(y_max - y_min)/ny,
 *     and per-pixel arrays are row-major [ny][nx] (index iy*nx + ix);
 *     per-crossing arrays are [3][ny][nx] (index n*nx*ny + iy*nx + ix).
 */
#ifndef RT_MI355X_RT_H
#define RT_MI355X_RT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_VERSION 2

/* Spacetime (Sec. 2.1, eqs. (4), (9), (13)). */
enum { RT_KERR = 0, RT_EINASTO = 1, RT_CNFW = 2 };

/* Arithmetic of the trace.
 *   RT_FP64   every ray in binary64 at rtol/atol.
 *   RT_MIXED  rays start in binary32 (right-hand side, stages and step
 *             controller in single precision at max(rtol, 1e-6) and
 *             max(atol, 1e-6); the state carried as a compensated float pair).
 *             A ray continues in binary64 at rtol/atol from the first step
 *             that would end within 1.5 R_+ of the horizon, and a ray with two
 *             crossings or more than 1024 accepted binary32 steps is traced
 *             again entirely in binary64 (its outputs are then those of
 *             RT_FP64).  Crossings are located, and all outputs written, in
 *             binary64.  Images of a batch with this precision run after the
 *             binary64 ones, one launch pair each. */
enum { RT_FP64 = 0, RT_MIXED = 1 };

/* Return codes. */
enum {
  RT_OK = 0,
  RT_ERR_ARG = -1,        /* invalid argument (null pointer, bad range, NaN)      */
  RT_ERR_NO_HORIZON = -2, /* Delta(R) has no root in (0.05, 50]: no outer horizon */
  RT_ERR_HIP = -3,        /* HIP runtime or launch failure                        */
  RT_ERR_ALLOC = -4       /* stream-ordered scratch allocation failed             */
};

/* Per-ray termination status (Sec. 3.3). */
enum {
  RT_RAY_CAPTURED = 1,    /* R <= r_stop_fac * R_+ at the end of an accepted step */
  RT_RAY_ESCAPED = 2,     /* R >= r_esc_fac * R_o at the end of an accepted step  */
  RT_RAY_STEP_LIMIT = 3,  /* max_attempts step attempts used                      */
  RT_RAY_NONFINITE = 4    /* 20 consecutive attempts with a non-finite error
                             estimate (each rejected, the step shrunk by 0.2)     */
};

/* Parameters of one image (host memory). */
typedef struct rt_image_params {
  int32_t metric;        /* RT_KERR, RT_EINASTO or RT_CNFW                            */
  int32_t precision;     /* RT_FP64 or RT_MIXED                                       */
  double spin;           /* chi = a/M (eq. (1)); the spacetime must have a horizon    */
  double halo[2];        /* RT_EINASTO: {lambda_E > 0 (eq. (10)), ignored};
                            RT_CNFW: {eta >= 0 (eq. (14)), lambda_c > 0 (eq. (12))};
                            RT_KERR: ignored                                          */
  double incl;           /* theta_o [rad], 0 < theta_o < pi (Sec. 3.2)                */
  double r_obs;          /* R_o, observer radius; > r_out and outside the horizon     */
  int32_t nx, ny;        /* screen pixels, >= 1 each, nx*ny < 2^31                    */
  double x_min, x_max;   /* screen extent in X, x_min < x_max                         */
  double y_min, y_max;   /* screen extent in Y, y_min < y_max                         */
  double rtol, atol;     /* Dormand-Prince 5(4) tolerances, > 0                       */
  double r_stop_fac;     /* capture at R <= r_stop_fac * R_+ (eq. (75)), > 1          */
  double r_esc_fac;      /* escape at R >= r_esc_fac * R_o, > 1                       */
  double r_in;           /* inner disc edge (eq. (77)); <= 0 means R_+                */
  double r_out;          /* outer disc edge, > r_in                                   */
  double emis_pow;       /* thin-disc emissivity R^-emis_pow                          */
  double sigma_in;       /* taper widths of eqs. (85)-(86); both > 0 selects the      */
  double sigma_out;      /*   tanh tapers, otherwise hard edges r_in <= R <= r_out    */
  double h0;             /* first trial affine step, > 0                              */
  int32_t max_attempts;  /* step attempts per ray (accepted + rejected), >= 1         */
  int32_t reserved;      /* must be 0                                                 */
} rt_image_params;

/* Outputs of one image: device pointers, any of which may be NULL (not wanted).
 * Crossing records n >= min(N_cross, 3) are NaN. */
typedef struct rt_image_out {
  uint8_t *ncross;       /* [ny][nx] trusted equatorial crossings, saturating at 255  */
  uint8_t *status;       /* [ny][nx] RT_RAY_*                                         */
  double *r_em;          /* [3][ny][nx] R at crossing n (eq. (82))                    */
  double *phi_em;        /* [3][ny][nx] phi at crossing n (traced ray, phi_0 = 0)     */
  double *t_em;          /* [3][ny][nx] T at crossing n (traced ray, T_0 = 0)         */
  double *g_em;          /* [3][ny][nx] redshift g at crossing n (eq. (89)); 0 where
                            no timelike circular orbit exists                         */
  double *intensity;     /* [ny][nx] I = sum_n I_n                                    */
  double *intensity_n;   /* [3][ny][nx] I_n = w(R_n) g_n^3 R_n^-emis_pow              */
  int32_t *attempts;     /* [ny][nx] step attempts used by the ray                    */
  double *reduce;        /* [3] {F, X_c, Y_c} of `intensity` (Sec. 6.2): the flux by
                            the midpoint rule and the intensity-weighted centroid;
                            requires `intensity` (RT_ERR_ARG otherwise)               */
} rt_image_out;

/* Trace n_images images (params[i] -> out[i]).  Every pixel's ray is
 * integrated with Hamilton's equations and the adaptive Dormand-Prince 5(4)
 * controller; equatorial crossings are located on the continuous extension
 * of each step; the thin-disc intensity uses the Keplerian emitter of
 * eqs. (89)-(91), computed by a per-pixel pass after the trace from the
 * crossing counts and radii (an image whose out has no ncross or r_em gets
 * them in stream-ordered scratch memory).  One image runs the single-image
 * kernel; several images run in one persistent launch per 128 images, rays of
 * all images drawn from one work queue, with results bit-identical to tracing
 * each image alone.
 * Returns RT_ERR_NO_HORIZON if any image has no outer horizon, RT_ERR_ARG for
 * invalid parameters or n_images < 1; in either case nothing is launched. */
int rt_trace_image(const rt_image_params *params, int32_t n_images, const rt_image_out *out,
                   void *hip_stream);

/* The transfer maps only (Sec. 4.2-4.3): like rt_trace_image but the emission
 * outputs (g_em, intensity, intensity_n, reduce) are ignored and not computed. */
int rt_transfer_maps(const rt_image_params *params, int32_t n_images, const rt_image_out *out,
                     void *hip_stream);

/* Outer horizon R_+ (largest root of Delta, eq. (33)) and the image setup the
 * trace uses, on the host: setup[0..3] = {R_+, capture radius, escape radius,
 * inner disc edge}.  `setup` is host memory.  Synchronous. */
int rt_image_setup(const rt_image_params *params, double *setup);

/* Thick-disc image (Sec. 5.1-5.2, eqs. (84)-(90)): every pixel's ray is
 * traced as by rt_trace_image (binary64, params->precision RT_FP64) with the
 * observed intensity I = int g^3 j dlambda integrated along it as a seventh
 * Dormand-Prince component in the same error norm (so the steps also resolve
 * the emitting layer).  j(R, theta) = (rho/R_in)^-p exp(-(rho - R_in)/R_s)
 * exp(-z^2 / (2 H^2)) T(rho) with j_0 = 1, rho = R sin(theta),
 * z = R cos(theta), H = h0 + h_slope rho, p = params->emis_pow, R_in as
 * params->r_in (<= 0: R_+), T the tapers of eqs. (85)-(86) with
 * params->sigma_in/out (hard edges R_in <= rho <= r_out unless both > 0);
 * the emitter moves with the circular equatorial angular velocity of eq. (91)
 * at the same R, u^T from u.u = -1 with the metric at (R, theta); no emission
 * where that has no solution.  Layers much thinner than the steps the
 * geodesic needs can be stepped over (every stage misses them, the error
 * estimate is zero): about 0.05 M at rtol = atol = 1e-8.
 *   out->intensity required; ncross, status, attempts, r_em, phi_em, t_em as
 *   for rt_transfer_maps, or NULL; g_em, intensity_n and reduce must be NULL.
 * RT_ERR_ARG for a null/invalid thick (r_scale, h0 > 0, h_slope >= 0, finite),
 * a missing intensity or a non-null g_em / intensity_n / reduce. */
typedef struct rt_thick_disc {
  double r_scale;        /* R_s of eq. (84), > 0                                       */
  double h0;             /* H_0 of eq. (85), > 0                                       */
  double h_slope;        /* h of eq. (85), >= 0                                        */
} rt_thick_disc;
int rt_trace_thick(const rt_image_params *params, const rt_thick_disc *thick,
                   const rt_image_out *out, void *hip_stream);

/* Parameter scans of the spacetimes (Sec. 2), one point per entry:
 *   points device [n] rt_scan_point (metric and halo as in rt_image_params,
 *          spin chi, theta the polar angle of the ergosurface radius)
 *   out    device [n][4] = {R_+ (eq. (33): the largest root of Delta =
 *          R^2 - F(R) + chi^2 in (0.05, 50]), the ergosurface radius at theta
 *          (the largest root of R^2 - F(R) + chi^2 cos^2 theta, g_TT = 0),
 *          chi_e (the extremal spin: chi_e^2 = max_R (F(R) - R^2)), r_e (the
 *          radius of that maximum)}; NaN where a root or maximum does not
 *          exist (spin beyond extremal) and for an invalid point (unknown
 *          metric, lambda_E or lambda_c <= 0, eta < 0, reserved != 0,
 *          non-finite values)
 * One thread per point: downward scan of spacing 1e-2 for the roots (with
 * the interior-minimum test near extremality), 1e-3 upward for the maximum,
 * each refined by bisection to the last representable bracket; the same code
 * as the image set-up's horizon.  Asynchronous on the stream, no scratch.
 * RT_ERR_ARG for null pointers or n outside [1, 2^24]. */
typedef struct rt_scan_point {
  int32_t metric;        /* RT_KERR, RT_EINASTO or RT_CNFW                            */
  int32_t reserved;      /* must be 0                                                 */
  double spin;           /* chi                                                       */
  double halo[2];        /* as rt_image_params.halo                                   */
  double theta;          /* polar angle of the ergosurface radius [rad]               */
} rt_scan_point;
int rt_parameter_scan(const rt_scan_point *points, int32_t n, double *out, void *hip_stream);

/* Image-level morphology diagnostics of a raw intensity map (Sec. 6.2) and
 * its bright-peak scale (Sec. 6.3), midpoint rule over the pixel centres of
 * the screen of `params` (only nx, ny and the extent are read):
 *   out device [RT_DIAG_COUNT] = {F, X_c, Y_c, C = |(X_c, Y_c)|, rho_bar,
 *       d_img = 2 rho_bar, w_img, w_img / d_img, A_LR, I_max, <I>_img, P,
 *       rho_peak, d_peak}: rho is the distance from the centroid, rho_bar its
 *       intensity-weighted mean, w_img = [sum (rho - rho_bar)^2 I dX dY / F]^(1/2),
 *       A_LR = (F_R - F_L)/(F_R + F_L) with F_R, F_L the flux of the pixels
 *       with X > X_c and X < X_c, <I>_img the mean intensity of the pixels with
 *       I > 0, P = I_max / <I>_img; rho_peak the centre of the first bin of
 *       largest mean of the origin-centred radial profile, d_peak = 2 rho_peak
 *   profile device [n_bins] or NULL: the mean intensity of the pixels with
 *       floor(|(X, Y)| / bin_width) = k (NaN for an empty bin); pixels beyond
 *       the last bin are not binned
 * Deterministic (fixed summation order).  Scratch (~10 KB + 8 n_bins bytes)
 * is stream-ordered.  RT_ERR_ARG for null intensity/params/out, a bad screen,
 * bin_width <= 0 or n_bins outside [1, 2^20]. */
enum { RT_DIAG_COUNT = 14 };
int rt_image_diagnostics(const double *intensity, const rt_image_params *params, double bin_width,
                         int32_t n_bins, double *out, double *profile, void *hip_stream);

/* Relative deviations of image diagnostics from a reference image's (Sec.
 * 6.2: a dark-matter-dressed model against Kerr under the same emission):
 * delta[i] = (q[i] - ref[i]) / ref[i] for i < n, IEEE arithmetic (ref[i] = 0
 * gives +-inf or NaN).  q, ref, delta are device [n] (e.g. two outputs of
 * rt_image_diagnostics); delta may alias q.  Asynchronous, no scratch.
 * RT_ERR_ARG for null pointers or n outside [1, 2^24]. */
int rt_relative_deviation(const double *q, const double *ref, int32_t n, double *delta,
                          void *hip_stream);

/* rt_image_diagnostics without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same results,
 * bit for bit, with their partial sums in a file-scope device array of the
 * library (about 533 KB on each device it runs on, held until the process
 * ends) instead of stream-ordered scratch.  The array is shared by every call
 * on a device and keeps the last call's contents (every value is written
 * before it is read, so nothing is carried over): calls that overlap on one
 * device, on different streams or threads, race and must be serialised by
 * the caller.  Arguments and errors as for rt_image_diagnostics; without a
 * profile buffer (profile NULL) the profile bins live in that array, so
 * n_bins may be at most RT_DIAG_NOALLOC_MAX_BINS (RT_ERR_ARG otherwise).
 * Calls no hipMalloc, hipFree or allocating library routine; the array's
 * device address is looked up once per device on the first call there. */
enum { RT_DIAG_NOALLOC_MAX_BINS = 65536 };
int rt_image_diagnostics_noalloc(const double *intensity, const rt_image_params *params,
                                 double bin_width, int32_t n_bins, double *out, double *profile,
                                 void *hip_stream);

/* Rays from listed screen points (the adaptive screen of Sec. 4: the screen
 * refined where its classification changes, e.g. the subpixels that
 * rt_refine_points lists).  Ray i starts from the point (X, Y) = (xy[2 i],
 * xy[2 i + 1]) (units of M) of the observer of `params` and is traced exactly
 * as a pixel of rt_trace_image (binary64, params->precision RT_FP64); the
 * screen fields of params (nx, ny, extent) are validated but not used.
 *   xy: device [n][2], 1 <= n < 2^31.  out: as rt_image_out with the pixel
 *   index replaced by the point index (ncross, status, attempts, intensity
 *   [n]; r_em, phi_em, t_em, g_em, intensity_n [3][n], NaN past
 *   min(N_cross, 3)); any may be NULL, but an emission output (intensity,
 *   g_em, intensity_n) needs ncross and r_em, and reduce must be NULL.
 * Stream-ordered (a 256-byte work-queue counter allocated and freed on the
 * stream).  RT_ERR_ARG for null params/xy/out, n out of range, precision
 * other than RT_FP64, a non-null reduce, an emission output without ncross
 * or r_em, or host memory. */
int rt_trace_points(const rt_image_params *params, const double *xy, int64_t n,
                    const rt_image_out *out, void *hip_stream);

/* Screen refinement near the lensing-band boundaries (Sec. 4, the adaptive
 * idea; Sec. 4.2, the bands labelled by N_cross): a pixel of the screen of
 * `params` is marked when one of its 4-neighbours has another N_cross or
 * another status in the maps ncross and status (device [ny][nx], as
 * rt_trace_image writes them), i.e. it straddles a band edge, the shadow
 * boundary or the critical curve.  *n_marked (device int64) receives the
 * number of marked pixels; for the marked pixels in pixel order m = 0, 1, ...
 * with m < max_points / sub^2: pix[m] = the pixel index (device int64 array,
 * or NULL) and its sub x sub subpixel centres, row by row:
 *   xy[2 (m sub^2 + b sub + a)]     = x0 + (ix + (a + 1/2) (1/sub)) dX,
 *   xy[2 (m sub^2 + b sub + a) + 1] = y0 + (iy + (b + 1/2) (1/sub)) dY,
 * with (x0, dX, y0, dY) the screen's origin and pixel size (sub = 1 gives the
 * pixel centres of rt_trace_image bit for bit).  1 <= sub <= 16; xy device
 * [max_points][2] (NULL only when max_points = 0, e.g. to count first).
 * Stream-ordered (scratch of 8 bytes per 256 pixels allocated and freed on the
 * stream).  RT_ERR_ARG for null params/ncross/status/n_marked, sub out of
 * range, max_points < 0, a null xy with max_points > 0, or host memory. */
int rt_refine_points(const rt_image_params *params, const uint8_t *ncross, const uint8_t *status,
                     int32_t sub, int64_t max_points, double *xy, int64_t *pix,
                     int64_t *n_marked, void *hip_stream);

/* Shadow boundary (Sec. 4.1, eqs. (78)-(79)): along each screen direction
 * (cos psi, sin psi), the impact parameter b at which the rays from
 * X = b cos psi, Y = b sin psi turn from captured to escaping (a ray escapes
 * when it reaches r_esc_fac R_o; captured rays and rays ending otherwise count
 * as inside).  Multisection: the bracket [lo, hi] starts at [b_lo, b_hi];
 * each pass traces S = samples (64, 32 or 16) rays at b_j = lo + j w,
 * w = (hi - lo)/(S + 1), j = 1..S, and keeps [b_{j-1}, b_j] around the first
 * escaping sample (b_0 = lo), or [b_S, hi] if none escapes, while hi - lo > b_tol (at most 64 passes, and
 * none once a pass leaves the bracket unchanged).  Rays are traced as by
 * rt_trace_image in binary64 (params->precision must be RT_FP64; the screen
 * fields are validated but not used).
 *   dirs    device [n][2] (cos psi, sin psi); any length, the ray starts from
 *           b times it
 *   out     device [n][2] the final bracket (lo, hi); the boundary point of
 *           eq. (79) is (lo + hi)/2 times the direction
 *   status  device [n]: 0, or 1 where the ray at b_lo escapes or the one at
 *           b_hi does not (out is then b_lo, b_hi)
 *   attempts device [n] step attempts of all the direction's rays, or NULL
 * Asynchronous on the stream; no scratch.  RT_ERR_ARG for null pointers,
 * n outside [1, 2^24], samples not 16, 32 or 64, b_lo <= 0, b_lo >= b_hi, b_tol < 1e-13 b_hi or
 * non-finite values. */
int rt_shadow_boundary(const rt_image_params *params, const double *dirs, int32_t n,
                       int32_t samples, double b_lo, double b_hi, double b_tol, double *out,
                       int32_t *status, int64_t *attempts, void *hip_stream);

/* A sample count for rt_shadow_boundary with n directions on the current
 * device: the largest S of 64, 32 and 16 whose n S rays fit in one wavefront
 * per SIMD (4 SIMDs of 64 lanes per compute unit), else 16.  A pass lasts as
 * long as its slowest ray, the one that winds longest near the photon shell:
 * while the device has idle SIMDs, more samples (fewer passes) finish first;
 * once it is full, fewer samples waste less of each pass.  Returns 16, 32 or
 * 64; RT_ERR_ARG for n < 1, RT_ERR_HIP if the device cannot be queried. */
int rt_shadow_boundary_samples(int32_t n);

/* Profiling hook.  When both are non-NULL hipEvent_t handles, every later
 * rt_trace_image / rt_transfer_maps call made on this thread records
 * `start_event` on its stream just before the first trace kernel and
 * `stop_event` just after the last one (the work-queue reset before, the
 * emission pass and the reductions after are outside the bracket).  NULL, NULL switches it off.
 * The events stay owned by the caller.  Returns RT_ERR_ARG if exactly one is
 * NULL. */
int rt_set_kernel_timing(void *start_event, void *stop_event);

/* Normalised visibility amplitudes of a traced image (Sec. 6.4, eqs. (108)-
 * (109)): V(u,v) = sum over pixel centres of I exp(-2 pi i (u X + v Y)) dX dY
 * and amp = |V(u,v)| / |V(0,0)|, at K points (u, v) in cycles per M.
 *   intensity  device [ny][nx] image on the screen of `params` (only nx, ny and
 *              the extent are read)
 *   uv         device [K][2] (u, v) pairs
 *   amp        device [K] normalised amplitudes, or NULL
 *   vis        device [K][2] (Re V, Im V), or NULL (not both NULL)
 * Binary64 on the vector ALU, the phases generated in registers (no phase
 * table in memory); fixed summation order, deterministic.  Scratch (16 K ny/16
 * bytes of partial sums and a few KB) is stream-ordered.  RT_ERR_ARG for a bad
 * screen, K < 1 or K > 2^22. */
int rt_visibility_dft(const double *intensity, const rt_image_params *params, const double *uv,
                      int32_t K, double *amp, double *vis, void *hip_stream);

/* One image of a batched visibility call: as the arguments of
 * rt_visibility_dft (device pointers; the screen given directly). */
typedef struct rt_vis_image {
  const double *intensity;  /* device [ny][nx]                                       */
  const double *uv;         /* device [K][2] (u, v) in cycles per M                  */
  double *amp;              /* device [K] |V| / |V(0,0)|, or NULL                    */
  double *vis;              /* device [K][2] (Re V, Im V), or NULL (not both NULL)   */
  int32_t nx, ny;           /* screen pixels                                         */
  int32_t K;                /* points, 1 <= K <= 2^22                                */
  int32_t reserved;         /* must be 0                                             */
  double x_min, x_max, y_min, y_max;   /* screen extent                              */
} rt_vis_image;

/* rt_visibility_dft for n_images images (host array `images`) in one launch
 * sequence: the work of all images shares the device, so small images do not
 * leave it idle.  Results equal n_images single calls bit for bit.
 * RT_ERR_ARG as for rt_visibility_dft (naming the image), or n_images outside
 * [1, 2^16]. */
int rt_visibility_dft_batch(const rt_vis_image *images, int32_t n_images, void *hip_stream);

/* The compact Fourier-domain summaries of Sec. 6.4: the azimuthally averaged
 * normalised amplitude V(q) and the horizontal cut V(|u|, 0), at n_q radii
 * q (device [n_q], cycles per M, q >= 0).  The average is taken over n_angles
 * equally spaced directions phi_a = 2 pi a / n_angles, a = 0..n_angles-1, of
 * the (u, v) plane (the trapezoid rule of the angular mean, exact for
 * angular harmonics below n_angles): avg[j] = mean_a |V(q_j cos phi_a,
 * q_j sin phi_a)| / |V(0,0)|; the cut is the amplitude at phi = 0:
 * cut[j] = |V(q_j, 0)| / |V(0,0)|.  avg and cut are device [n_q] or NULL (not
 * both).  Scratch (24 n_q n_angles bytes plus that of rt_visibility_dft) is
 * stream-ordered.  RT_ERR_ARG for null pointers, n_q or n_angles < 1 or
 * n_q n_angles > 2^22, or a bad screen. */
int rt_visibility_rings(const double *intensity, const rt_image_params *params, const double *q,
                        int32_t n_q, int32_t n_angles, double *avg, double *cut,
                        void *hip_stream);

/* Bases of the image gradient: the parameters as rt_image_params holds them,
 * q = (spin, incl, halo[0], halo[1]), or for the cored-NFW halo its density
 * and scale, q = (spin, incl, rho_s, r_s) with eta = 4 pi rho_s r_s^2 and
 * lambda_c = r_s (eq. (13) and the halo parametrisation of Sec. 2.1). */
enum { RT_GRAD_NATIVE = 0, RT_GRAD_DENSITY = 1 };

/* Gradient of a scalar loss L(I) of the thin-disc image with respect to the
 * four image parameters q (basis above), by reverse mode through the map the
 * trace computes (Sec. 3.1-3.3 geodesics, Sec. 5.2 eqs. (89)-(91) emission,
 * Sec. 3.2 eqs. (70)-(74) screen map).  It is the exact derivative of the
 * discrete map with its decisions frozen: the accepted step sizes, which
 * attempts were accepted, the step holding each crossing, the termination,
 * and the indicator parts of the disc window (eq. (77)) and of the emitter's
 * existence (A > 0 in eq. (89)); the crossing points move with q by the
 * implicit function theorem on the step's continuous extension, and the inner
 * disc edge, when it is the outer horizon (r_in <= 0), moves with R_+.
 *   params    the image (as for rt_trace_image; precision must be RT_FP64)
 *   dl_dI     device [ny][nx] cotangent dL/dI of the image
 *   basis     RT_GRAD_NATIVE or RT_GRAD_DENSITY (cored NFW only)
 *   grad      device [4]: dL/dq = sum over pixels of dl_dI dI/dq (fixed order,
 *             deterministic)
 *   grad_pix  device [ny][nx][4] per-pixel dl_dI dI/dq, or NULL
 * Pixels with dl_dI = 0 are not traced.  Internally, by checkpointed
 * recomputation: a forward trace stores a checkpoint of every contributing ray
 * before every 32nd accepted step (up to 32 slots per pixel, fewer if the
 * checkpoint budget requires, at least 4; a ray that runs out of slots keeps
 * every other checkpoint and doubles its interval, so rays of any length
 * fit), then a backward pass restores each segment's checkpoint from the last
 * to the first, recomputes its steps -- bit for bit the traced ones -- and
 * reverses them.  Memory: 128 bytes per checkpoint slot and pixel, plus
 * 7.5 KiB per resident lane of the backward pass, all stream-ordered and
 * released by the end of the call; nothing is kept between calls and the
 * stream is not synchronised (the call is fully asynchronous).
 * Errors as for rt_trace_image; RT_ERR_ARG for an unknown basis or the
 * density basis on a metric other than RT_CNFW. */
int rt_image_vjp(const rt_image_params *params, const double *dl_dI, int32_t basis,
                 double *grad, double *grad_pix, void *hip_stream);

/* Counters of the last mixed-precision image traced on this thread and the
 * current device: out[0] = rays finished in binary64 (continued from the
 * horizon zone or traced again), out[1] = of those, rays traced again from the
 * screen, out[2] = step attempts made in binary32, out[3] = step attempts made
 * by the binary64 pass.  `out` holds 4 values.  Synchronous (waits for that
 * call's work).  All 0 before any such call. */
int rt_mixed_stats(int64_t *out);

/* Profiling hook beside rt_set_kernel_timing: when non-NULL (a hipEvent_t),
 * every later rt_trace_image call on this thread records it on its stream
 * between the binary32 pass and the binary64 pass of each mixed-precision
 * image.  NULL switches it off.  The event stays owned by the caller. */
int rt_set_split_timing(void *event);

/* Device memory the gradient's checkpoints may use (thread-local, bytes, at
 * least 1 MiB; default 16 GiB): the slots per pixel are the most of 32 whose
 * 128 bytes each fit n_pix times in the budget, at least 4 (a soft limit for
 * very large screens).  Fewer slots only make long rays double their
 * checkpoint interval sooner and recompute more; results are unchanged. */
int rt_set_checkpoint_budget(int64_t bytes);

/* Statistics of the last rt_image_vjp call on this thread and the current
 * device: out[0..4] = {rays reversed, accepted steps reversed, checkpoint
 * slots per pixel, bytes of scratch memory the call used, recomputations that
 * diverged from the trace (0: a non-zero count means a wrong gradient)}.
 * `out` holds 5 values.  Synchronous (waits for that call's work). */
int rt_vjp_stats(int64_t *out);

/* How the persistent trace kernels hand out work (thread-local setting,
 * applies to later calls on this thread).
 *   order = RT_ORDER_CENTRE (default): a single image's pixels go to
 *     wavefronts in tiles of tile_w x tile_h pixels (0 x 0: 8 x 8), one tile
 *     per claim, tiles ordered by the distance of their centre from the photon
 *     ring's radius around the screen origin (the direction of the hole; the
 *     radius is the critical impact parameter of the metric without spin), so
 *     that the long rays near the ring are traced first and the short ones,
 *     deep in the shadow and far out, fill the end.
 *   order = RT_ORDER_SCREEN: pixels go out in chunks of `chunk` consecutive
 *     ordinals (0: 64) of the screen enumerated in tiles of tile_w x tile_h
 *     pixels (row by row, clipped at the screen edges; 0 x 0: row-major).
 * Batched launches (n_images > 1) always use the screen order within each
 * image, with chunk and tile sizes as set.  `blocks_per_cu` caps the resident
 * workgroups launched per compute unit (0 = as many as fit).  The results of a
 * trace do not depend on these settings (every ray is traced the same way);
 * only its speed does.  The order tables (4 bytes per tile) are built on the
 * host the first time a screen shape and halo are traced and kept per
 * thread. */
enum { RT_ORDER_CENTRE = 0, RT_ORDER_SCREEN = 1 };
typedef struct rt_launch_config {
  int32_t chunk;          /* 0..65536                                            */
  int32_t tile_w, tile_h; /* both 0 or both > 0                                  */
  int32_t blocks_per_cu;  /* 0..64                                               */
  int32_t order;          /* RT_ORDER_CENTRE or RT_ORDER_SCREEN                   */
} rt_launch_config;

/* Set (NULL: restore the defaults) or read the launch configuration.
 * RT_ERR_ARG for out-of-range fields. */
int rt_set_launch_config(const rt_launch_config *cfg);
int rt_get_launch_config(rt_launch_config *cfg);

/* Thread-local description of the last error on this thread ("" if none). */
const char *rt_last_error(void);

/* RT_VERSION of the library. */
int rt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RT_MI355X_RT_H */
