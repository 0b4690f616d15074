// rt_ray.h -- the per-ray computation shared by the trace and adjoint
// kernels: the right-hand side of the geodesic equations, one Dormand-Prince
// 5(4) step attempt with its controller and crossing events, the screen map,
// the emission and the wave-level work hand-out.  Everything a ray computes
// is written here once (host and device; the reverse mode is in rt_vjp.h).
//
// Paper: M. Fathi, "Adaptive ray tracing, image diagnostics, and photon ring
// signatures of rotating dark-matter-dressed black holes".  Units M = 1.
#pragma once

#include "rt_device.h"
#include "rt_dual.h"
#include "rt_kernels.h"
#include "rt_math.h"

namespace rt {
namespace ray {

constexpr double kHalfPi = 1.5707963267948966;
constexpr double kPi = 3.141592653589793;
constexpr double kInvPi = 0.3183098861837907;
// A ray whose error estimate is not finite on this many consecutive attempts
// (its step shrunk by 0.2 each time, to ~1e-14 of where it started) ends with
// RAY_NONFINITE.
constexpr int32_t kNonfiniteRun = 20;

__host__ __device__ __forceinline__ double rcp(double x) { return dm::recip1(x); }
__host__ __device__ __forceinline__ float rcp(float x) { return dm::recip(x); }
template <int N>
__host__ __device__ __forceinline__ Dual<N> rcp(const Dual<N>& x) { return 1.0 / x; }

// The constants of the step loop: a copy of the ImageConst fields the
// right-hand side, the controller and the stop tests read.
struct Hot {
    double chi, chi2, inv_lam, lam_c, inv_lam_c, eta_lc;
    double rtol, atol, r_stop, r_esc;
    int32_t max_attempts;
    // thick-disc source (read by the THICK attempts only)
    int32_t taper;
    double r_in, r_out, emis_pow, thick_h0, thick_h;
    double inv_r_in, inv_rs, tin, tout;   // 1/r_in, 1/R_s, 2/sigma_in, 2/sigma_out
};

__host__ __device__ __forceinline__ Hot hot_of(const ImageConst& c) {
    Hot k;
    k.chi = c.chi;
    k.chi2 = c.chi2;
    k.inv_lam = c.inv_lam;
    k.lam_c = c.lam_c;
    k.inv_lam_c = c.inv_lam_c;
    k.eta_lc = c.eta_lc;
    k.rtol = c.rtol;
    k.atol = c.atol;
    k.r_stop = c.r_stop;
    k.r_esc = c.r_esc;
    k.max_attempts = c.max_attempts;
    k.taper = c.taper;
    k.r_in = c.r_in;
    k.r_out = c.r_out;
    k.emis_pow = c.emis_pow;
    k.thick_h0 = c.thick_h0;
    k.thick_h = c.thick_h;
    k.inv_r_in = c.inv_r_in;
    k.inv_rs = c.inv_thick_rs;
    k.tin = c.tin;
    k.tout = c.tout;
    return k;
}

// ---------------------------------------------------------------- the RHS
// Hamilton's equations for H = g^{ab} p_a p_b / 2 with p_T = -E, p_phi = l.
// The inverse metric of eqs. (49)-(53) is used through the algebraically
// identical separated form of Sec. 3.1 (the Hamilton-Jacobi equation
// multiplied by Sigma):
//   2 Sigma H = N = Delta p_R^2 + p_theta^2 - P^2/Delta + W^2,
//   P = (R^2 + chi^2) E - chi l,   W = l/sin(theta) - chi E sin(theta),
// so that, with Sigma = R^2 + chi^2 cos^2(theta) (eq. (23)),
//   dT/dl   = [P (R^2+chi^2)/Delta + chi (l - chi E sin^2)] / Sigma     (57)
//   dR/dl   = Delta p_R / Sigma                                         (59)
//   dth/dl  = p_theta / Sigma                                           (60)
//   dphi/dl = [chi P/Delta + l/sin^2 - chi E] / Sigma                   (58)
//   dp_R/dl = -dH/dR = (N R/Sigma - dN/dR / 2) / Sigma                  (61)
//   dp_th/dl= -dH/dth = cos/Sigma [W (l/sin^2 + chi E) - chi^2 sin N/Sigma]  (62)
// The N dSigma terms keep the full derivative of H off the constraint shell.
// chiE and chiL are chi E and chi l, constants of the ray.
template <int METRIC, class K, class S>
__host__ __device__ __forceinline__ void rhs_c(const K& k, const S& E, const S& L, const S& chiE,
                                              const S& chiL, const S& R, const S& th,
                                              const S& pR, const S& pth, S d[6]) {
    const S half(0.5), two(2.0), four(4.0);
    S s, co;
    dm::sincos(th, &s, &co);
    S F, dF;
    mass_function<METRIC>(k, R, F, dF);
    const S R2 = R * R;
    const S R2c = R2 + k.chi2;
    const S Sig = R2 + k.chi2 * co * co;
    const S Del = R2c - F;
    const S dDel = two * R - dF;
    // 1/Sigma, 1/Delta and 1/sin(theta) from one reciprocal of their product
    const S SD = Sig * Del;
    const S inv = rcp(SD * s);
    const S sinv = s * inv;
    const S iS = Del * sinv;
    const S iD = Sig * sinv;
    const S is = SD * inv;
    const S P = R2c * E - chiL;
    const S PiD = P * iD;
    const S Lis2 = L * is * is;
    const S W = L * is - chiE * s;
    const S N = Del * pR * pR + pth * pth - P * PiD + W * W;
    const S dN = dDel * (pR * pR + PiD * PiD) - four * R * E * PiD;
    d[0] = (PiD * R2c + k.chi * (L - chiE * s * s)) * iS;
    d[1] = Del * pR * iS;
    d[2] = pth * iS;
    d[3] = (k.chi * PiD + Lis2 - chiE) * iS;
    const S NiS = N * iS;
    d[4] = (R * NiS - half * dN) * iS;
    d[5] = co * iS * (W * (Lis2 + chiE) - k.chi2 * s * NiS);
}

// The same, forming chi E and chi l here (callers that evaluate many steps of
// one ray pass them in, formed once).
template <int METRIC, class K, class S>
__host__ __device__ __forceinline__ void rhs(const K& k, const S& E, const S& L, const S& R, const S& th,
                                    const S& pR, const S& pth, S d[6]) {
    rhs_c<METRIC>(k, E, L, S(k.chi * E), S(k.chi * L), R, th, pR, pth, d);
}

// ------------------------------------------------ Dormand-Prince 5(4) tableau
// Dormand & Prince (1980), first-same-as-last.
constexpr double a21 = 0.2;
constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
constexpr double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
constexpr double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0,
                 a54 = -212.0 / 729.0;
constexpr double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0,
                 a64 = 49.0 / 176.0, a65 = -5103.0 / 18656.0;
constexpr double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0,
                 b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
// Error weights: 5th-order minus embedded 4th-order weights.
constexpr double e1 = 71.0 / 57600.0, e3 = -71.0 / 16695.0, e4 = 71.0 / 1920.0,
                 e5 = -17253.0 / 339200.0, e6 = 22.0 / 525.0, e7 = -1.0 / 40.0;
// Continuous extension in Hairer's form (Solving ODEs I, II.6):
//   y(s) = y0 + s (r2 + (1-s)(r3 + s (r4 + (1-s) r5))),
//   r2 = y1 - y0, r3 = h k1 - r2, r4 = r2 - h k7 - r3, r5 = h sum_i d_i k_i.
constexpr double d1 = -12715105075.0 / 11282082432.0, d3 = 87487479700.0 / 32700410799.0,
                 d4 = -10690763975.0 / 1880347072.0, d5 = 701980252875.0 / 199316789632.0,
                 d6 = -1453857185.0 / 822651844.0, d7 = 69997945.0 / 29380423.0;

struct DenseComp {
    double y0, r2, r3, r4, r5;
    __host__ __device__ double at(double s) const {
        return y0 + s * (r2 + (1.0 - s) * (r3 + s * (r4 + (1.0 - s) * r5)));
    }
};

// ------------------------------------------------------------ emission
// Keplerian equatorial emitter (eqs. (90)-(91)) and redshift (eq. (89)) for a
// photon with constants (E, l) and unit observer-frame energy.  At theta =
// pi/2, Sigma = R^2 and with G = d(F/R^2)/dR the metric derivatives are
// dg_TT = G, dg_Tphi = -chi G, dg_phiphi = 2R + chi^2 G, so eq. (91) reads
// Omega = (chi G + sqrt(-2 R G)) / (2R + chi^2 G).  g = 0 where no timelike
// circular orbit exists.
template <int METRIC, class K, class S>
__host__ __device__ __forceinline__ S redshift(const K& k, const S& R, const S& E, const S& L) {
    S F, dF;
    mass_function<METRIC>(k, R, F, dF);
    const S iR = 1.0 / R;
    const S FoR2 = F * iR * iR;
    const S G = (dF - 2.0 * F * iR) * iR * iR;
    const S disc = -2.0 * R * G;
    if (!(value_of(disc) >= 0.0)) return S(0.0);
    const S Om = (k.chi * G + sqrt(disc)) / (2.0 * R + k.chi2 * G);
    const S gTT = -(1.0 - FoR2);
    const S gTp = -k.chi * FoR2;
    const S gpp = R * R + k.chi2 + k.chi2 * FoR2;
    const S A = -(gTT + Om * (2.0 * gTp + Om * gpp));
    if (!(value_of(A) > 0.0)) return S(0.0);
    const S den = E - Om * L;
    if (!(value_of(den) > 0.0)) return S(0.0);
    return sqrt(A) / den;
}

// Disc window at equatorial radius R (eq. (77), or the tanh tapers of
// eqs. (85)-(86) with rho = R) for an inner edge r_in.
template <class S>
__host__ __device__ __forceinline__ S disc_window(const ImageConst& c, const S& R, const S& r_in) {
    if (c.taper) {
        const S tin = 0.5 * (1.0 + tanh((R - r_in) / c.sigma_in));
        const S tout = 0.5 * (1.0 - tanh((R - c.r_out) / c.sigma_out));
        return tin * tout;
    }
    return S((value_of(R) >= value_of(r_in) && value_of(R) <= c.r_out) ? 1.0 : 0.0);
}

// ------------------------------------------------------------- ray state
struct Ray {
    double y[6];    // T, R, theta, phi, p_R, p_theta
    double k1[6];   // f(y), first-same-as-last
    double I, kI;   // thick disc: intensity so far and g^3 j at y (THICK attempts only)
    double E, L, chiE, chiL;
    double h, lam, last_cross;
    double rc[3];   // radii of the first three trusted crossings
    int32_t attempts, ncross;
    int32_t after_reject;
    int64_t pix;
};

// E and l of a ray, with the products chi E and chi l that its steps use:
// every writer of a ray's constants of motion goes through here.
__host__ __device__ __forceinline__ void set_constants(double chi, double E, double L, Ray& r) {
    r.E = E;
    r.L = L;
    r.chiE = chi * E;
    r.chiL = chi * L;
}

// floor(a / b) for 0 <= a < 2^31 and 1 <= b < 2^31 without an integer
// division (which the GPU emulates in about 25 instructions): (a + 1/2)/b lies
// at least 1/(2b) from an integer, and its binary64 value through the
// one-Newton-step reciprocal (2.3e-15 relative) is within (a + 1/2) 2.3e-15 / b
// of it, below 1/(2b) for every a < 2^31.
__host__ __device__ __forceinline__ int32_t quotient(int32_t a, int32_t b) {
    return static_cast<int32_t>((static_cast<double>(a) + 0.5) * dm::recip1(static_cast<double>(b)));
}

// The two ways of dividing the screen indices: integer division, and
// quotient() (fewer instructions, a few more registers: the batched kernel,
// whose lanes start rays of any image, takes it; in the single-image kernel it
// cost more in spills than it saved).
struct IntQuotient {
    __host__ __device__ int32_t operator()(int32_t a, int32_t b) const { return a / b; }
};
struct FpQuotient {
    __host__ __device__ int32_t operator()(int32_t a, int32_t b) const { return quotient(a, b); }
};

// Pixel index of the p-th pixel of an nx x ny screen in tile order: tiles of
// tw x th pixels, taken row by row; pixels inside a tile row by row; tiles on
// the right and bottom edges are clipped to the screen.  tw = nx, th = 1 is
// plain row-major order.  A bijection of [0, nx ny) for 1 <= tw <= nx and
// 1 <= th <= ny (the launch clamps the tile to the screen).
template <class Q = IntQuotient>
__host__ __device__ __forceinline__ int64_t tile_pixel(int64_t p64, int32_t nx, int32_t ny,
                                                       int32_t tw, int32_t th, Q div = Q{}) {
    // 32-bit index arithmetic: screens hold fewer than 2^31 pixels
    const int32_t p = static_cast<int32_t>(p64);
    const int32_t band = th * nx;                  // pixels per full tile row
    const int32_t r = div(p, band);                // tile row
    const int32_t h = (r + 1) * th <= ny ? th : ny - r * th;
    const int32_t q = p - r * band;                // index inside the tile row
    const int32_t full = div(nx, tw);              // unclipped tiles per row
    const int32_t j = div(q, tw * h);
    int32_t ix, iy;
    if (j < full) {
        const int32_t off = q - j * tw * h;
        const int32_t oy = div(off, tw);
        iy = r * th + oy;
        ix = j * tw + (off - oy * tw);
    } else {
        const int32_t w = nx - full * tw;
        const int32_t off = q - full * tw * h;
        const int32_t oy = div(off, w);
        iy = r * th + oy;
        ix = full * tw + (off - oy * w);
    }
    return static_cast<int64_t>(iy) * nx + ix;
}

// Screen pixel -> initial state (Sec. 3.2, eqs. (70)-(74) with E_loc = 1):
// with n = -(R_o, Y, X)/sqrt(R_o^2 + X^2 + Y^2) in the ZAMO triad, lowering
// p^mu = u_o + n^(a) e_(a) with the observer metric gives
// E = N_o - g_Tphi n^(phi)/sqrt(g_phiphi), l = sqrt(g_phiphi) n^(phi),
// p_R = sqrt(g_RR) n^(R), p_theta = sqrt(g_thth) n^(theta).
struct ScreenDir {
    double nR, nth, nph;
};

// The direction of screen point (X, Y).
__host__ __device__ __forceinline__ ScreenDir screen_dir_xy(const ImageConst& c, double X, double Y) {
    const double inv = dm::rsqrt(c.r_obs * c.r_obs + X * X + Y * Y);
    return ScreenDir{-c.r_obs * inv, -Y * inv, -X * inv};
}

// The direction of the centre of pixel (ix, iy).
__host__ __device__ __forceinline__ ScreenDir screen_dir_ij(const ImageConst& c, int32_t ix,
                                                           int32_t iy) {
    const double X = c.x0 + (static_cast<double>(ix) + 0.5) * c.dx;
    const double Y = c.y0 + (static_cast<double>(iy) + 0.5) * c.dy;
    return screen_dir_xy(c, X, Y);
}

// The direction of pixel pix's centre.
__host__ __device__ __forceinline__ ScreenDir screen_dir(const ImageConst& c, int64_t pix) {
    // 32-bit index arithmetic: screens hold fewer than 2^31 pixels
    const int32_t p = static_cast<int32_t>(pix);
    const int32_t iy = p / c.nx;
    return screen_dir_ij(c, p - iy * c.nx, iy);
}

// The photon's conserved E and l of pixel pix.
__host__ __device__ __forceinline__ void photon_constants(const ImageConst& c, const ScreenDir& n,
                                                          double& E, double& L) {
    E = c.obs_N - c.obs_gTph_over_sq_gphph * n.nph;
    L = c.obs_sq_gphph * n.nph;
}

// A ray from screen direction n, recorded as pixel pix.
template <int METRIC>
__host__ __device__ __forceinline__ void start_ray_dir(const ImageConst& c, const Hot& k,
                                                       const ScreenDir& n, int64_t pix, Ray& r) {
    double E, L;
    photon_constants(c, n, E, L);
    set_constants(k.chi, E, L, r);
    r.y[0] = 0.0;
    r.y[1] = c.r_obs;
    r.y[2] = c.incl;
    r.y[3] = 0.0;
    r.y[4] = c.obs_sq_gRR * n.nR;
    r.y[5] = c.obs_sq_gthth * n.nth;
    rhs<METRIC>(k, r.E, r.L, r.y[1], r.y[2], r.y[4], r.y[5], r.k1);
    r.h = c.h0;
    r.lam = 0.0;
    r.last_cross = -INFINITY;
    r.rc[0] = r.rc[1] = r.rc[2] = 0.0;
    r.attempts = 0;
    r.ncross = 0;
    r.after_reject = 0;
    r.pix = pix;
}

template <int METRIC>
__host__ __device__ __forceinline__ void start_ray(const ImageConst& c, const Hot& k, int64_t pix, Ray& r) {
    start_ray_dir<METRIC>(c, k, screen_dir(c, pix), pix, r);
}

// A pixel as its index and its column and row.
struct Pixel {
    int64_t pix;
    int32_t ix, iy;
};

template <int METRIC>
__host__ __device__ __forceinline__ void start_ray(const ImageConst& c, const Hot& k, const Pixel& px,
                                                   Ray& r) {
    start_ray_dir<METRIC>(c, k, screen_dir_ij(c, px.ix, px.iy), px.pix, r);
}

// Equatorial passage of a step from theta0 to theta1 (Sec. 3.3).
// Boyer-Lindquist theta is continued through the poles (a ray with l = 0
// passes over the axis and leaves (0, pi); (theta, phi) and (-theta, phi + pi)
// are one point), so the equator is theta = pi/2 (mod pi).  The band index
// floor((theta - pi/2)/pi) changes exactly when a step crosses it; for theta
// in (0, pi) that is a change of the boolean theta >= pi/2.  th_eq is the
// crossed equator's theta, up0 whether theta0 lies above it, phi_shift the
// azimuth to add where th_eq = -pi/2 (mod 2 pi) (the far side of the axis).
struct Passage {
    double th_eq, phi_shift;
    bool up0;
};

__host__ __device__ __forceinline__ double equator_band(double th) {
    return floor((th - kHalfPi) * kInvPi);
}

__host__ __device__ __forceinline__ Passage passage_of(double band0, double band1) {
    const double kk = fmax(band0, band1);
    Passage p;
    p.th_eq = kHalfPi + kk * kPi;
    p.phi_shift = (kk - 2.0 * floor(0.5 * kk)) != 0.0 ? kPi : 0.0;
    p.up0 = band0 > band1;
    return p;
}

// Root of theta(s) = th_eq on the step's continuous extension, s in (0, 1),
// given theta(0) and theta(1) on opposite sides.  Writing the extension as
// y0 + s (c1 + s (c2 + s (c3 + s c4))):
//
// crossing_root_safe: Newton's method from the secant root, kept inside the
// shrinking sign bracket (bisection when a Newton step would leave it); it
// stops after a step below 1e-10 (Newton's quadratic convergence leaves the
// new iterate ~1e-20 c2/c1 from the root), when the bracket is exhausted, or at
// once where the extension evaluates to exactly th_eq (the zero Newton step
// from there would not lie strictly inside the bracket).  The quotients use
// the one-Newton-step reciprocal (2e-15): an error of that size in a Newton
// step is corrected by the next.
//
// crossing_root: four plain Newton steps from the secant root, each dividing
// by the derivative through the hardware reciprocal estimate (2^-24 relative;
// the error then contracts as e <- C e^2 + 6e-8 e, from the secant root's
// ~1e-2 to ~1e-20 on a step the controller accepted), then the same
// acceptance as the safeguarded search: an iterate inside (0, 1) whose last
// step is at most 1e-10.  A lane that fails it (an extension that turns near
// the crossing, a poor start, a non-finite derivative) runs the safeguarded
// search.  The plain steps carry no bracket bookkeeping: about a third of the
// instructions per iteration, and a wavefront runs them whenever one of its
// lanes crosses the equator.
__host__ __device__ __forceinline__ double crossing_root_safe(const DenseComp& d, bool up0,
                                                             double th_eq) {
    const double c1 = d.r2 + d.r3;
    const double c2 = d.r4 + d.r5 - d.r3;
    const double c3 = -d.r4 - 2.0 * d.r5;
    const double c4 = d.r5;
    const double f0 = d.y0 - th_eq;   // exact: theta(0) lies within pi/2 of th_eq
    double a = 0.0, b = 1.0;
    double s = -f0 * rcp(d.r2);
    if (!(s > 0.0 && s < 1.0)) s = 0.5;
    for (int it = 0; it < 48; ++it) {
        const double f = f0 + s * (c1 + s * (c2 + s * (c3 + s * c4)));
        if (f == 0.0) break;   // s is a root of the evaluated extension
        if ((f >= 0.0) == up0) a = s; else b = s;
        const double df = c1 + s * (2.0 * c2 + s * (3.0 * c3 + s * 4.0 * c4));
        double sn = s - f * rcp(df);
        if (!(sn > a && sn < b)) sn = 0.5 * (a + b);
        const double step = fabs(sn - s);
        s = sn;
        if (step <= 1e-10 || b - a <= 1e-15) break;
    }
    return s;
}

__host__ __device__ __forceinline__ double crossing_root(const DenseComp& d, bool up0,
                                                        double th_eq) {
    const double c1 = d.r2 + d.r3;
    const double c2 = d.r4 + d.r5 - d.r3;
    const double c3 = -d.r4 - 2.0 * d.r5;
    const double c4 = d.r5;
    const double f0 = d.y0 - th_eq;   // exact: theta(0) lies within pi/2 of th_eq
    const double dc2 = 2.0 * c2, dc3 = 3.0 * c3, dc4 = 4.0 * c4;
    double s = -f0 * dm::recip_estimate(d.r2);
    if (!(s > 0.0 && s < 1.0)) s = 0.5;
    double step = 0.0;
    for (int it = 0; it < 4; ++it) {
        const double f = f0 + s * (c1 + s * (c2 + s * (c3 + s * c4)));
        const double df = c1 + s * (dc2 + s * (dc3 + s * dc4));
        step = f * dm::recip_estimate(df);
        s -= step;
    }
    if (s > 0.0 && s < 1.0 && fabs(step) <= 1e-10) return s;
    return crossing_root_safe(d, up0, th_eq);
}

// dI/dlambda = g^3 j of the thick disc (Sec. 5.1-5.2) at (R, theta) for a
// photon (E, l) of unit observer-frame energy: the emissivity eq. (84) with
// j_0 = 1, rho = R sin(theta), z = R cos(theta), H = H_0 + h rho and the
// window of the image (tapers of eqs. (85)-(86) or hard edges); the emitter
// moves with the circular equatorial angular velocity of eq. (91) at the same
// R, its u^T from u.u = -1 with the metric at (R, theta) (eqs. (89)-(90)); no
// emission where that has no solution.  The quotients go through reciprocals
// of their denominators (g^3 = A^(3/2) (1/den)^3).  The early returns stay:
// a branch-free version kept more values live and spilled.
template <int METRIC>
__host__ __device__ inline double thick_source(const Hot& k, double R, double th, double E, double L) {
    double s, co;
    dm::sincos(th, &s, &co);
    const double rho = R * s, z = R * co;
    if (!(rho > 0.0)) return 0.0;
    double w;
    if (k.taper) {
        // (1 + tanh u)/2 = 1/(1 + e^{-2u}), (1 - tanh u)/2 = 1/(1 + e^{2u}): one
        // reciprocal of the product, 0 where it is infinite (far outside the edges)
        const double p = (1.0 + dm::exp(-(rho - k.r_in) * k.tin)) *
                         (1.0 + dm::exp((rho - k.r_out) * k.tout));
        w = p < INFINITY ? rcp(p) : 0.0;
    } else {
        w = (rho >= k.r_in && rho <= k.r_out) ? 1.0 : 0.0;
    }
    if (w == 0.0) return 0.0;
    const double H = k.thick_h0 + k.thick_h * rho;
    const double zH = z * rcp(H);
    // the three factors of eq. (84) as one exponential
    const double j = dm::exp(-k.emis_pow * dm::log1p(rho * k.inv_r_in - 1.0) -
                             (rho - k.r_in) * k.inv_rs - 0.5 * zH * zH) *
                     w;
    double F, dF;
    mass_function<METRIC>(k, R, F, dF);
    const double iR = rcp(R);
    const double G = (dF - 2.0 * F * iR) * (iR * iR);   // d(F/R^2)/dR
    const double disc = -2.0 * R * G;
    if (!(disc >= 0.0)) return 0.0;
    const double Om = (k.chi * G + sqrt(disc)) * rcp(2.0 * R + k.chi2 * G);
    const double FiS = F * rcp(R * R + k.chi2 * co * co);   // F/Sigma
    const double s2 = s * s;
    const double gTT = -(1.0 - FiS);
    const double gTph = -FiS * k.chi * s2;
    const double gphph = (R * R + k.chi2 + FiS * k.chi2 * s2) * s2;
    const double A = -(gTT + 2.0 * Om * gTph + Om * Om * gphph);
    if (!(A > 0.0)) return 0.0;
    const double den = E - Om * L;
    if (!(den > 0.0)) return 0.0;
    const double id = rcp(den);
    return A * sqrt(A) * (id * id * id) * j;
}

// A thick-disc ray: as start_ray, with I = 0 and its source at the start.
template <int METRIC>
__host__ __device__ __forceinline__ void start_ray_thick(const ImageConst& c, const Hot& k, int64_t pix,
                                                         Ray& r) {
    start_ray<METRIC>(c, k, pix, r);
    r.I = 0.0;
    r.kI = thick_source<METRIC>(k, r.y[1], r.y[2], r.E, r.L);
}

// One step attempt.  Returns 0 while the ray runs, else its final status.
// The 5th-order update, the error estimate and the continuous-extension
// coefficient r5 are accumulated as the stages are produced, so a stage
// derivative stays live only while later stage inputs still need it.
// `sink(j, k_j)` sees each stage derivative k_{j+1} (j = 0..5, six
// components) as it is produced; the trace kernels pass StageNone, the
// gradient's tape kernels record them.
struct StageNone {
    __host__ __device__ __forceinline__ void operator()(int, const double*) const {}
};

// THICK: the thick disc's intensity as a seventh component (dI/dlambda =
// thick_source, no feedback), in the error norm with the other six.
template <int METRIC, class Sink = StageNone, bool THICK = false>
__host__ __device__ __forceinline__ int32_t attempt(const Hot& k, const OutPtrs& o, int64_t n_pix,
                                                    Ray& r, Sink sink = Sink{}) {
    if (r.attempts >= k.max_attempts) return RAY_STEP_LIMIT;
    ++r.attempts;
    const double h = r.h;
    double ab[6], ae[6], ad[6];     // sums of b_i k_i, e_i k_i, d_i k_i
    double k2[6], k3[6], k4[6], k5[6], kk[6], t[6];
    sink(0, r.k1);
    for (int i = 0; i < 6; ++i) {
        ab[i] = b1 * r.k1[i];
        ae[i] = e1 * r.k1[i];
        ad[i] = d1 * r.k1[i];
    }
    double abI = 0.0, aeI = 0.0;   // THICK: sums of b_i kI_i, e_i kI_i
    if constexpr (THICK) {
        abI = b1 * r.kI;
        aeI = e1 * r.kI;
    }
// THICK: the source at the current stage input t (b_2 = e_2 = 0: stage 2
// needs none)
#define RT_ACC_I(bb, ee)                                                         \
    if constexpr (THICK) {                                                       \
        const double kI_ = thick_source<METRIC>(k, t[1], t[2], r.E, r.L);        \
        abI += bb * kI_;                                                         \
        aeI += ee * kI_;                                                         \
    }
#define RT_STAGE(expr, out)                                                      \
    for (int i = 0; i < 6; ++i) t[i] = r.y[i] + h * (expr);                       \
    rhs_c<METRIC>(k, r.E, r.L, r.chiE, r.chiL, t[1], t[2], t[4], t[5], out);
#define RT_ACC(bb, ee, dd, kv)                                                   \
    for (int i = 0; i < 6; ++i) {                                                \
        ab[i] += bb * kv[i];                                                     \
        ae[i] += ee * kv[i];                                                     \
        ad[i] += dd * kv[i];                                                     \
    }
    RT_STAGE(a21 * r.k1[i], k2)
    sink(1, k2);
    RT_STAGE(a31 * r.k1[i] + a32 * k2[i], k3)
    sink(2, k3);
    RT_ACC(b3, e3, d3, k3)
    RT_ACC_I(b3, e3)
    RT_STAGE(a41 * r.k1[i] + a42 * k2[i] + a43 * k3[i], k4)
    sink(3, k4);
    RT_ACC(b4, e4, d4, k4)
    RT_ACC_I(b4, e4)
    RT_STAGE(a51 * r.k1[i] + a52 * k2[i] + a53 * k3[i] + a54 * k4[i], k5)
    sink(4, k5);
    RT_ACC(b5, e5, d5, k5)
    RT_ACC_I(b5, e5)
    RT_STAGE(a61 * r.k1[i] + a62 * k2[i] + a63 * k3[i] + a64 * k4[i] + a65 * k5[i], kk)
    sink(5, kk);
    RT_ACC(b6, e6, d6, kk)
    RT_ACC_I(b6, e6)
#undef RT_STAGE
#undef RT_ACC
#undef RT_ACC_I
    double yn[6];
    for (int i = 0; i < 6; ++i) yn[i] = r.y[i] + h * ab[i];
    rhs_c<METRIC>(k, r.E, r.L, r.chiE, r.chiL, yn[1], yn[2], yn[4], yn[5], kk);   // k7 (first-same-as-last)
    double acc = 0.0;
    for (int i = 0; i < 6; ++i) {
        ae[i] += e7 * kk[i];
        ad[i] += d7 * kk[i];
        const double sc = k.atol + k.rtol * fmax(fabs(r.y[i]), fabs(yn[i]));
        const double q = ae[i] * rcp(sc);
        acc += q * q;
    }
    double ynI = 0.0, kI7 = 0.0;
    if constexpr (THICK) {
        kI7 = thick_source<METRIC>(k, yn[1], yn[2], r.E, r.L);
        aeI += e7 * kI7;
        ynI = r.I + h * abI;
        const double sc = k.atol + k.rtol * fmax(fabs(r.I), fabs(ynI));
        const double q = aeI * rcp(sc);
        acc += q * q;
    }
    // err^2 = mean of the squared scaled errors (h e_i/sc_i)^2, with h^2 taken
    // out of the sum; the step is accepted when
    // err < 1 and the size factor is 0.9 err^(-1/5) = 0.9 (err^2)^(-1/10),
    // clipped to [0.2, 10] (err = 0 gives the maximum, a non-finite err the
    // minimum).  Outside err^2 in [1e-12, 1e12] the clip decides the factor.
    const double err2 = (h * h) * acc * (THICK ? 1.0 / 7.0 : 1.0 / 6.0);
    const double grow = 0.9 * dm::rpow_tenth(fmin(fmax(err2, 1e-12), 1e12));
    if (!(err2 < 1.0)) {  // reject; NaN lands here too
        const bool finite = __builtin_isfinite(err2);
        r.h = h * (finite ? fmax(0.2, grow) : 0.2);
        // 1 after a rejection, plus 2 per consecutive non-finite estimate
        r.after_reject = finite ? 1 : (r.after_reject | 1) + 2;
        return r.after_reject >= 2 * kNonfiniteRun + 1 ? RAY_NONFINITE : 0;
    }
    double factor = err2 == 0.0 ? 10.0 : fmin(10.0, grow);
    if (r.after_reject) factor = fmin(1.0, factor);
    r.after_reject = 0;

    // Equatorial crossing (Sec. 3.3): theta's band index changes.
    const double band0 = equator_band(r.y[2]);
    const double band1 = equator_band(yn[2]);
    if (band0 != band1) {
        const Passage ps = passage_of(band0, band1);
        auto dense = [&](int i) {
            DenseComp d;
            d.y0 = r.y[i];
            d.r2 = yn[i] - r.y[i];
            d.r3 = h * r.k1[i] - d.r2;
            d.r4 = d.r2 - h * kk[i] - d.r3;
            d.r5 = h * ad[i];
            return d;
        };
        const double s = crossing_root(dense(2), ps.up0, ps.th_eq);
        const double Rc = dense(1).at(s);
        const double pthc = dense(5).at(s);
        const double lc = r.lam + s * h;
        // trusted crossing (Sec. 4.2): |dtheta/dlambda| = |p_theta|/R^2 bounded away
        // from zero and not a repeat within a tiny affine interval
        if (fabs(pthc) >= 1e-12 * Rc * Rc && (lc - r.last_cross) >= 1e-10) {
            const int n = r.ncross;
            if (n < 3) {
                const int64_t off = static_cast<int64_t>(n) * n_pix + r.pix;
                // (selects, not r.rc[n]: a runtime index would put the ray in scratch)
                r.rc[0] = n == 0 ? Rc : r.rc[0];
                r.rc[1] = n == 1 ? Rc : r.rc[1];
                r.rc[2] = n == 2 ? Rc : r.rc[2];
                if (o.r_em) o.r_em[off] = Rc;
                if (o.phi_em) o.phi_em[off] = dense(3).at(s) + ps.phi_shift;
                if (o.t_em) o.t_em[off] = dense(0).at(s);
            }
            if (r.ncross < 255) ++r.ncross;
            r.last_cross = lc;
        }
    }

    for (int i = 0; i < 6; ++i) {
        r.y[i] = yn[i];
        r.k1[i] = kk[i];
    }
    if constexpr (THICK) {
        r.I = ynI;
        r.kI = kI7;
    }
    r.lam += h;
    r.h = h * factor;
    if (r.y[1] <= k.r_stop) return RAY_CAPTURED;   // eq. (75)
    if (r.y[1] >= k.r_esc) return RAY_ESCAPED;
    return 0;
}

// Ray epilogue: the per-pixel transfer-map outputs.  Records n >=
// min(N_cross, 3) are NaN: written here when FILL_NAN, else by the per-pixel
// pass after the trace (emit_pixel), which the trace kernels of one image and
// of a batch leave it to: a wavefront runs this epilogue whenever one of its
// rays ends, about a third of its step attempts.  The emission is that pass
// too.
template <bool FILL_NAN = true>
__device__ __forceinline__ void finish_ray(const ImageConst& c, const OutPtrs& o, const Ray& r,
                                           int32_t status) {
    const int64_t p = r.pix;
    if (o.ncross) o.ncross[p] = static_cast<uint8_t>(r.ncross);
    if (o.status) o.status[p] = static_cast<uint8_t>(status);
    if (o.attempts) o.attempts[p] = r.attempts;
    if constexpr (FILL_NAN) {
        const int64_t n_pix = c.n_pix;
        const int nrec = r.ncross < 3 ? r.ncross : 3;
        const double nan = __builtin_nan("");
        for (int n = nrec; n < 3; ++n) {
            const int64_t off = static_cast<int64_t>(n) * n_pix + p;
            if (o.r_em) o.r_em[off] = nan;
            if (o.phi_em) o.phi_em[off] = nan;
            if (o.t_em) o.t_em[off] = nan;
        }
    }
}

// The pass after the trace, pixel p: NaN in the transfer-map records n >=
// min(N_cross, 3) (finish_ray<false> leaves them), then, for an image with
// emission, the emission (Sec. 5.2) of its recorded crossings: the redshift
// (eq. (89)) and disc intensity of each of the first min(N_cross, 3) crossing
// radii, their sum, NaN for the records beyond.  Reads o.ncross and o.r_em as
// the trace wrote them and recomputes the photon's E and l from the screen
// map, so it gives what the ray's own epilogue would.  One thread per pixel
// after the trace: the trace's wavefronts then do not carry this code through
// their divergent epilogue, where it cost most of the lanes' time.
template <int METRIC>
__device__ __forceinline__ void emit_pixel(const ImageConst& c, const Hot& k, const OutPtrs& o,
                                           int64_t p) {
    const int64_t n_pix = c.n_pix;
    const int ncr = o.ncross[p];
    const int nrec = ncr < 3 ? ncr : 3;
    const double nan = __builtin_nan("");
    for (int n = nrec; n < 3; ++n) {
        const int64_t off = static_cast<int64_t>(n) * n_pix + p;
        if (o.r_em) o.r_em[off] = nan;
        if (o.phi_em) o.phi_em[off] = nan;
        if (o.t_em) o.t_em[off] = nan;
    }
    if (!c.emission) return;
    double E, L;
    photon_constants(c, screen_dir(c, p), E, L);
    double intensity = 0.0;
    for (int n = 0; n < 3; ++n) {
        const int64_t off = static_cast<int64_t>(n) * n_pix + p;
        double g = nan, In = nan;
        if (n < nrec) {
            const double R = o.r_em[off];
            g = redshift<METRIC>(k, R, E, L);
            In = disc_window(c, R, c.r_in) * g * g * g * pow(R, -c.emis_pow);
            intensity += In;
        }
        if (o.g_em) o.g_em[off] = g;
        if (o.intensity_n) o.intensity_n[off] = In;
    }
    if (o.intensity) o.intensity[p] = intensity;
}

// Wave-level hand-out of pixels: lanes without a ray take consecutive
// ordinals from the wave's current chunk; the wave claims a new chunk (one
// atomic, lane 0) when it runs dry.  Called with all lanes converged.
// `claim()` returns false when the queue is exhausted and otherwise sets the
// chunk's ordinal range [next, end) (and whatever image state it tracks);
// `take(ordinal)` starts a ray on the calling lane.
template <class Claim, class Take>
__device__ __forceinline__ void refill(bool& active, bool& exhausted, int64_t& next,
                                       int64_t& end, Claim claim, Take take) {
    const int lane = __lane_id();
    unsigned long long need = __ballot(!active);
    while (need != 0ull) {
        if (next >= end) {
            if (!claim()) {
                exhausted = true;
                return;
            }
        }
        const int64_t avail = end - next;
        const int nneed = __popcll(need);
        const int tk = avail < nneed ? static_cast<int>(avail) : nneed;
        const int rank = __popcll(need & ((1ull << lane) - 1ull));
        if (!active && rank < tk) {
            take(next + rank);
            active = true;
        }
        next += tk;
        need = __ballot(!active);
    }
}

// Claim of the next chunk of ordinals [next, end) below `total` by the whole
// wave (one atomic, lane 0).  Called with all lanes converged.
__device__ __forceinline__ bool claim_chunk(unsigned long long* queue, int32_t chunk,
                                            int64_t total, int64_t& next, int64_t& end) {
    unsigned long long base = 0;
    if (__lane_id() == 0) base = atomicAdd(queue, static_cast<unsigned long long>(chunk));
    base = __shfl(base, 0);
    if (static_cast<int64_t>(base) >= total) return false;
    next = static_cast<int64_t>(base);
    end = next + chunk < total ? next + chunk : total;
    return true;
}


// A wave's current claim in tile-order hand-out (wave-uniform).
struct TileClaim {
    int32_t x0, y0, w;
    float inv_w;   // 1/w, for the row of an ordinal inside the tile
};

// Next claim of a screen's pixels by the whole wave: a chunk of ordinals of
// the tile enumeration, or the next tile of shape.order (one atomic either
// way).  Sets the claimed range [next, end) of ordinals within the claim.
__device__ __forceinline__ bool claim_screen(const LaunchShape& shape, int32_t nx, int32_t ny,
                                             unsigned long long* queue, int64_t& next,
                                             int64_t& end, TileClaim& t) {
    if (!shape.order)
        return claim_chunk(queue, shape.chunk, static_cast<int64_t>(nx) * ny, next, end);
    const int32_t tiles_x = (nx + shape.tile_w - 1) / shape.tile_w;
    const int32_t n_tiles = tiles_x * ((ny + shape.tile_h - 1) / shape.tile_h);
    unsigned long long q = 0;
    if (__lane_id() == 0) q = atomicAdd(queue, 1ull);
    q = __shfl(q, 0);
    if (static_cast<int64_t>(q) >= n_tiles) return false;
    const int32_t id = shape.order[q];
    const int32_t ty = id / tiles_x;
    t.x0 = (id - ty * tiles_x) * shape.tile_w;
    t.y0 = ty * shape.tile_h;
    t.w = nx - t.x0 < shape.tile_w ? nx - t.x0 : shape.tile_w;
    t.inv_w = 1.0f / static_cast<float>(t.w);
    const int32_t h = ny - t.y0 < shape.tile_h ? ny - t.y0 : shape.tile_h;
    next = 0;
    end = static_cast<int64_t>(t.w) * h;
    return true;
}

// Pixel of ordinal p of the current claim.  Inside a tile the row is
// floor((p + 1/2)/w) in binary32: exact, since the quotient's fraction stays
// 1/(2w) away from an integer and its rounding error is ~1e-7 (p/w)
// (tiles are far smaller than 2^15 pixels), which saves an integer division.
__device__ __forceinline__ Pixel claimed(const LaunchShape& shape, int32_t nx, int32_t ny,
                                         const TileClaim& t, int64_t p) {
    Pixel px;
    if (!shape.order) {
        px.pix = tile_pixel(p, nx, ny, shape.tile_w, shape.tile_h);
        px.iy = static_cast<int32_t>(px.pix) / nx;
        px.ix = static_cast<int32_t>(px.pix) - px.iy * nx;
        return px;
    }
    const int32_t o = static_cast<int32_t>(p);
    const int32_t row = static_cast<int32_t>((static_cast<float>(o) + 0.5f) * t.inv_w);
    px.ix = t.x0 + (o - row * t.w);
    px.iy = t.y0 + row;
    px.pix = static_cast<int64_t>(px.iy) * nx + px.ix;
    return px;
}

// Pixel index of ordinal p of the current claim.
__device__ __forceinline__ int64_t claimed_pixel(const LaunchShape& shape, int32_t nx, int32_t ny,
                                                 const TileClaim& t, int64_t p) {
    return claimed(shape, nx, ny, t, p).pix;
}

}  // namespace ray
}  // namespace rt
