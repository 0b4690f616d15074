// rt_device.h -- spacetime functions and per-image constants of the MI355X
// ray tracer, usable from host setup code and from the gfx950 kernels.
//
// Paper: M. Fathi, "Adaptive ray tracing, image diagnostics, and photon ring
// signatures of rotating dark-matter-dressed black holes".  Units M = 1.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "rt_dual.h"
#include "rt_math.h"

namespace rt {

enum : int32_t { KERR = 0, EINASTO = 1, CNFW = 2 };
// Kernel variant of CNFW (a template argument only, never an image's metric)
// for images whose halo has 0 <= eta <= dm::kExpm1Near (ImageConst::ex_near).
constexpr int32_t CNFW_NEAR = 3;
__host__ __device__ constexpr bool is_cnfw(int32_t m) { return m == CNFW || m == CNFW_NEAR; }
enum : int32_t { RAY_CAPTURED = 1, RAY_ESCAPED = 2, RAY_STEP_LIMIT = 3, RAY_NONFINITE = 4 };

// Everything a kernel needs to know about one image.  Passed by value as a
// kernel argument (it lands in the kernarg segment and is read through the
// scalar cache), or gathered from a device table in a batched launch.
struct ImageConst {
    int32_t metric;
    int32_t max_attempts;
    int32_t nx, ny;
    int64_t n_pix;
    // spacetime
    double chi, chi2;
    double inv_lam;      // Einasto: 1/lambda_E
    double lam_c;        // cored NFW: lambda_c
    double inv_lam_c;    // cored NFW: 1/lambda_c
    double eta_lc;       // cored NFW: eta * lambda_c
    // observer (Sec. 3.2): ZAMO normalisation and tetrad scale factors at (R_o, theta_o)
    double r_obs, incl;
    double obs_N;        // N_o, eq. (65)
    double obs_gTph_over_sq_gphph;   // g_Tphi / sqrt(g_phiphi)
    double obs_sq_gRR, obs_sq_gthth, obs_sq_gphph;
    // screen: X = x0 + (ix + 1/2) dx, Y = y0 + (iy + 1/2) dy
    double x0, dx, y0, dy;
    // integrator and events
    double rtol, atol, h0;
    double r_stop, r_esc;
    // mixed precision: binary32 bulk tolerances and the radius (1.5 R_+) below
    // which a ray continues in binary64
    double rtol32, atol32, r_zone;
    // emission
    double r_in, r_out, emis_pow, sigma_in, sigma_out;
    int32_t taper;       // 1: tanh tapers of eqs. (85)-(86); 0: hard window, eq. (77)
    int32_t emission;    // 0: transfer maps only
    // cored NFW with 0 <= eta <= kExpm1Near: the exponent of eq. (13), which
    // lies in [-eta, 0), never needs expm1's argument reduction, and the
    // kernels run their CNFW_NEAR variant
    int32_t ex_near;
    // thick disc (Sec. 5.1): radial scale R_s and height H = H_0 + h rho of eqs. (84)-(85)
    double thick_rs, thick_h0, thick_h;
    // the thick-disc source's divisors inverted on the host: 1/r_in, 1/R_s,
    // 2/sigma_in and 2/sigma_out (the last two 0 without tapers)
    double inv_r_in, inv_thick_rs, tin, tout;
};

// e^x - 1 of the cored-NFW exponent: in binary64 by the kernel of the near
// range x in [-kExpm1Near, 0] when `near` (binary32: without the argument
// reduction, exact there); dual numbers use the general function.
__host__ __device__ inline double expm1_ex(double x, bool near) { return dm::expm1(x, near); }
__host__ __device__ inline float expm1_ex(float x, bool near) { return dm::expm1(x, near); }
template <class S>
__host__ __device__ inline S expm1_ex(const S& x, bool) {
    return dm::expm1(x);
}

// The cored-NFW halo terms 1/R, 1/(R + lambda_c) and log(1 + R/lambda_c) in
// binary64 from one reciprocal: with 1 + R/lambda_c = m 2^e (dm::log_split;
// the sum is one fused operation), 1/(R (R + lambda_c) (m + 1)) gives both
// reciprocals and the logarithm kernel's quotient 2 (m - 1)/(m + 1) by
// multiplications.  Errors as dm::log1p_fast's: half an ulp of 1 + R/lambda_c
// absolute in the logarithm, plus the one-step reciprocal's 2.2e-15 relative
// in all three.
struct CnfwTerms {
    double iR, iRl, lg;
};
__host__ __device__ inline CnfwTerms cnfw_terms(double R, double lam_c, double inv_lam_c) {
    const double Rl = R + lam_c;
    const dm::LogSplit s = dm::log_split(fma(R, inv_lam_c, 1.0));
    const double d = R * Rl;
    const double inv = dm::recip1(fma(d, s.m, d));
    const double a = fma(s.m, inv, inv);   // 1/(R (R + lambda_c))
    CnfwTerms t;
    t.iR = Rl * a;
    t.iRl = R * a;
    const double w = fma(s.m, 2.0, -2.0) * (d * inv);   // 2 (m - 1)/(m + 1)
    t.lg = fma(s.e, dm::kLn2Hi, fma(s.e, dm::kLn2Lo, dm::log_kernel(w)));
    return t;
}

// F(R) = 2 R mu(R) (eq. (24)) and dF/dR for the chosen seed.  The mass
// functions mu_E (from eq. (9)) and mu_cNFW (from eq. (13)) are written in
// cancellation-free forms: mu_E = 1 - e^{-x}(1 + x + x^2/2) with x = R/lambda_E,
// mu_cNFW = 1 - (R/2) expm1(Ex) with Ex the exponent of eq. (13).  K is any
// struct with the fields inv_lam, lam_c, inv_lam_c, eta_lc; S is double,
// float or a dual number (then K's fields may be dual too).
template <int METRIC, class K, class S>
__host__ __device__ inline void mass_function(const K& c, const S& R, S& F, S& dF) {
    const S one(1.0), two(2.0), half(0.5);
    if constexpr (METRIC == KERR) {
        F = two * R;
        dF = two;
    } else if constexpr (METRIC == EINASTO) {
        const S x = R * c.inv_lam;
        const S e = dm::exp(-x);
        const S mu = one - e * (one + x * (one + half * x));
        const S dmu = half * e * x * x * c.inv_lam;
        F = two * R * mu;
        dF = two * (mu + R * dmu);
    } else {
        S iR, iRl, lg;
        if constexpr (std::is_same<S, double>::value) {
            const CnfwTerms t = cnfw_terms(R, c.lam_c, c.inv_lam_c);
            iR = t.iR;
            iRl = t.iRl;
            lg = t.lg;
        } else {
            // 1/R and 1/(R + lambda_c) from one reciprocal of their product
            const S Rl = R + c.lam_c;
            const S inv = dm::recip1(R * Rl);
            iR = Rl * inv;
            iRl = R * inv;
            lg = dm::log1p_fast(R * c.inv_lam_c);
        }
        const S ex = c.eta_lc * (iRl - two * iR * lg);
        const S dex = c.eta_lc * (two * iR * (iR * lg - iRl) - iRl * iRl);
        const S em1 = expm1_ex(ex, METRIC == CNFW_NEAR);
        F = R * (two - R * em1);
        dF = two - R * (two * em1 + R * (em1 + one) * dex);
    }
}

// The metric constants with a scalar type of choice (dual numbers when
// differentiating with respect to them); a K for mass_function.
template <class S>
struct Coeffs {
    S chi, chi2, inv_lam, lam_c, inv_lam_c, eta_lc;
};

// Runtime dispatch of mass_function (host setup and the batched kernel).
__host__ __device__ inline void mass_function_any(const ImageConst& c, double R, double& F,
                                                  double& dF) {
    if (c.metric == EINASTO)
        mass_function<EINASTO>(c, R, F, dF);
    else if (c.metric == CNFW)
        mass_function<CNFW>(c, R, F, dF);
    else
        mass_function<KERR>(c, R, F, dF);
}

}  // namespace rt
