// rt_math.h -- compact binary64 elementary functions for the trace kernels.
//
// The right-hand side of the geodesic equations needs sin and cos of theta
// and, for the dark-matter seeds, exp, expm1 and log1p of well-scaled
// arguments; the step controller needs x^(-1/10).  The general-purpose
// library versions carry large-argument and special-case paths these
// arguments never take, and they dominate the instruction count of a step.
// The versions below are written from textbook methods:
//   * argument reduction by a constant split in several parts, evaluated with
//     fused multiply-adds (Cody & Waite, "Software Manual for the Elementary
//     Functions", 1980), valid for |x| < 2^20 * pi/2 (sincos) and |x| < 700
//     (exp), the ranges used here;
//   * Taylor series of sin, cos, exp and expm1 on the reduced interval,
//     truncated where the first omitted term is below 2^-60 relative;
//   * log(m) = 2 atanh((m-1)/(m+1)) for m in [sqrt(1/2), sqrt(2)), whose odd
//     series converges like 0.1716^(2n+1);
//   * x^(-1/10) by a Newton step on x y^10 = 1 from a binary32 estimate.
// Each is accurate to a few units in the last place on its stated domain
// (x^(-1/10): 1e-12 relative; tests/test_devmath.py measures the host
// versions against mpmath).  All are
// __host__ __device__ so the same source is tested on the CPU.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace rt {
namespace dm {

// pi/2 and ln 2 as sums of three doubles (each the nearest double to the
// remainder of the previous ones).
constexpr double kPio2Hi = 1.5707963267948966;
constexpr double kPio2Mid = 6.123233995736766e-17;
constexpr double kPio2Lo = -1.4973849048591698e-33;
constexpr double kTwoOverPi = 0.6366197723675814;
constexpr double kLn2Hi = 0.6931471805599453;
constexpr double kLn2Lo = 2.3190468138462996e-17;
constexpr double kInvLn2 = 1.4426950408889634;

// 1/x for finite, non-zero, normal x: a first estimate refined by two
// Newton-Raphson steps r <- r (2 - x r), each of which squares the relative
// error; within about one ulp.  On the device the estimate is the hardware
// reciprocal; on the host (tests) it is the division itself.
__host__ __device__ inline double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
#else
    double r = 1.0 / x;
#endif
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// 1/x to ~1e-14 relative for finite, non-zero, normal x: the hardware
// reciprocal (within 2^-24.4, measured on gfx950) refined by one Newton step,
// which squares its relative error (2.1e-15 measured).  For the right-hand
// side and the error norm of the integrator, whose results carry the
// tolerance-level truncation error of the step anyway.
__host__ __device__ inline double recip1(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double r = __builtin_amdgcn_rcp(x);
#else
    const double r = 1.0 / x;
#endif
    return fma(r, fma(-x, r, 1.0), r);
}

// sin and cos of x, |x| < 1.6e6.
__host__ __device__ inline void sincos(double x, double* s_out, double* c_out) {
    const double k = rint(x * kTwoOverPi);
    double r = fma(-k, kPio2Hi, x);
    r = fma(-k, kPio2Mid, r);
    r = fma(-k, kPio2Lo, r);
    const double z = r * r;
    // sin r = r + r z (-1/3! + z (1/5! - ... + z^7/17!))
    double ps = 1.0 / 355687428096000.0;
    ps = fma(ps, z, -1.0 / 1307674368000.0);
    ps = fma(ps, z, 1.0 / 6227020800.0);
    ps = fma(ps, z, -1.0 / 39916800.0);
    ps = fma(ps, z, 1.0 / 362880.0);
    ps = fma(ps, z, -1.0 / 5040.0);
    ps = fma(ps, z, 1.0 / 120.0);
    ps = fma(ps, z, -1.0 / 6.0);
    const double sr = fma(r * z, ps, r);
    // cos r = 1 + z (-1/2! + z (1/4! - ... + z^7/16!))
    double pc = 1.0 / 20922789888000.0;
    pc = fma(pc, z, -1.0 / 87178291200.0);
    pc = fma(pc, z, 1.0 / 479001600.0);
    pc = fma(pc, z, -1.0 / 3628800.0);
    pc = fma(pc, z, 1.0 / 40320.0);
    pc = fma(pc, z, -1.0 / 720.0);
    pc = fma(pc, z, 1.0 / 24.0);
    pc = fma(pc, z, -0.5);
    const double cr = fma(z, pc, 1.0);
    // quadrant: x = k pi/2 + r
    const int q = static_cast<int>(k) & 3;
    double s = (q & 1) ? cr : sr;
    double c = (q & 1) ? sr : cr;
    if (q & 2) s = -s;
    if ((q + 1) & 2) c = -c;
    *s_out = s;
    *c_out = c;
}

// e^r - 1 for |r| <= ln(2)/2 + 1e-9, Taylor series to r^14.
__host__ __device__ inline double expm1_reduced(double r) {
    double p = 1.0 / 87178291200.0;
    p = fma(p, r, 1.0 / 6227020800.0);
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    return fma(r * r, p, r);
}

// e^x; 0 below -745, +inf above 709.8.
__host__ __device__ inline double exp(double x) {
    const double xc = fmin(fmax(x, -760.0), 720.0);
    const double k = rint(xc * kInvLn2);
    double r = fma(-k, kLn2Hi, xc);
    r = fma(-k, kLn2Lo, r);
    return ldexp(1.0 + expm1_reduced(r), static_cast<int>(k));
}

// e^x - 1 without cancellation for small |x|, branch-free: with x = k ln 2 + r,
// e^x - 1 = 2^k (e^r - 1) + (2^k - 1), one fused multiply-add of exact
// operands (2^k - 1 is exact for the k that matter; k = 0 for |x| <= ln(2)/2,
// where the result is the reduced series itself).  -1 below -745; x is
// clamped at 709, below the overflow of e^x.
__host__ __device__ inline double expm1(double x) {
    const double xc = fmin(fmax(x, -745.0), 709.0);
    const double k = rint(xc * kInvLn2);
    double r = fma(-k, kLn2Hi, xc);
    r = fma(-k, kLn2Lo, r);
    const double tk = ldexp(1.0, static_cast<int>(k));
    return fma(tk, expm1_reduced(r), tk - 1.0);
}

// log(1 + u) for u > -1 (finite).
__host__ __device__ inline double log1p(double u) {
    const double v = 1.0 + u;
    // rounding error of 1 + u, carried as a first-order correction
    const double corr = (u - (v - 1.0)) * recip(v);
    int e;
    double m = frexp(v, &e);          // v = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double t = (m - 1.0) * recip(m + 1.0);
    const double z = t * t;
    // log m = 2 (t + t^3/3 + ... + t^23/23)
    double p = 1.0 / 23.0;
    p = fma(p, z, 1.0 / 21.0);
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double logm = 2.0 * fma(t * z, p, t);
    const double de = static_cast<double>(e);
    return fma(de, kLn2Hi, logm + fma(de, kLn2Lo, corr));
}

// Binary32 estimate of x^(-1/10), x in [1e-12, 1e12]: on the device
// 2^(-log2(x)/10) from the hardware base-2 logarithm and exponential (within
// 4.2e-7, measured over that range on gfx950), on the host powf.
__host__ __device__ inline float rpow_tenth_estimate(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_exp2f(-0.1f * __builtin_amdgcn_logf(x));
#else
    return powf(x, -0.1f);
#endif
}

// x^(-1/10) for x in [1e-12, 1e12]: the binary32 estimate refined by one
// Newton step y <- y (1 + (1 - x y^10)/10), which squares its relative error
// (below 1e-12 on the device, 9.4e-13 measured; the step-size factor needs
// far less).
__host__ __device__ inline double rpow_tenth(double x) {
    double y = static_cast<double>(rpow_tenth_estimate(static_cast<float>(x)));
    for (int it = 0; it < 1; ++it) {
        const double y2 = y * y;
        const double y4 = y2 * y2;
        const double y10 = y4 * y4 * y2;
        const double d = fma(-x, y10, 1.0);
        y = fma(0.1 * y, d, y);
    }
    return y;
}

// Binary32 versions for the single-precision bulk trace: the device math
// library's functions and the hardware reciprocal (about one binary32 ulp),
// and the binary32 estimate of x^(-1/10) (4.2e-7).
__host__ __device__ inline float recip(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
__host__ __device__ inline float recip1(float x) { return recip(x); }
__host__ __device__ inline void sincos(float x, float* s_out, float* c_out) {
    ::sincosf(x, s_out, c_out);
}
__host__ __device__ inline float exp(float x) { return ::expf(x); }
__host__ __device__ inline float expm1(float x) { return ::expm1f(x); }
__host__ __device__ inline float log1p(float u) { return ::log1pf(u); }
__host__ __device__ inline float rpow_tenth(float x) { return rpow_tenth_estimate(x); }

}  // namespace dm
}  // namespace rt
