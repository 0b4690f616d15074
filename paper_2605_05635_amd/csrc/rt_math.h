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
//     Functions", 1980), valid for |x| < 2^20 * pi (sincos) and |x| < 700
//     (exp), the ranges used here;
//   * polynomial kernels for sin, cos and e^r - 1 on the reduced interval and
//     for log(m) = 2 atanh((m-1)/(m+1)), m in [sqrt(1/2), sqrt(2)): Chebyshev
//     interpolants of the smooth remainder functions, degrees chosen so that
//     the approximation error stays below 1e-17 relative (poly_coeffs.py
//     generates the coefficients and states each bound);
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

// pi and ln 2 as sums of two doubles (each the nearest double to the
// remainder of the previous one).
constexpr double kPiHi = 3.141592653589793;
constexpr double kPiMid = 1.2246467991473532e-16;
constexpr double kInvPi = 0.3183098861837907;
constexpr double kLn2Hi = 0.6931471805599453;
constexpr double kLn2Lo = 2.3190468138462996e-17;
constexpr double kInvLn2 = 1.4426950408889634;

// The integer nearest to a x (ties to even, as rint) by the shift trick: the
// sum in fma(a, x, 1.5 2^52) has a unit in the last place of 1, so its one
// rounding is the rounding of the exact a x to an integer, and the low word of
// its encoding holds that integer in two's complement.  For |a x| < 2^51.  An
// FMA, an add and no conversion instruction, where rint and the conversion
// to int each issue at a fraction of the FMA rate.
constexpr double kRoundShift = 6755399441055744.0;   // 1.5 * 2^52
struct NearestInt {
    double k;    // the integer as a double
    int32_t i;   // the same integer
};
__host__ __device__ inline NearestInt nearest_int(double a, double x) {
    const double kk = fma(a, x, kRoundShift);
    NearestInt n;
    n.k = kk - kRoundShift;
    n.i = static_cast<int32_t>(static_cast<uint32_t>(__builtin_bit_cast(uint64_t, kk)));
    return n;
}

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
#elif defined(RT_HOST_RECIP1_ESTIMATE_ERROR)
    // host test builds: a starting estimate with the hardware estimate's error
    const double r = (1.0 / x) * (1.0 + RT_HOST_RECIP1_ESTIMATE_ERROR);
#else
    const double r = 1.0 / x;
#endif
    return fma(r, fma(-x, r, 1.0), r);
}

// An estimate of 1/x: on the device the hardware reciprocal (within 2^-24.4
// relative, measured on gfx950), on the host the division.  For iterations
// that correct their own errors.
__host__ __device__ inline double recip_estimate(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcp(x);
#elif defined(RT_HOST_RECIP_ESTIMATE_ERROR)
    // host test builds: a relative error of the hardware estimate's size
    return (1.0 / x) * (1.0 + RT_HOST_RECIP_ESTIMATE_ERROR);
#else
    return 1.0 / x;
#endif
}

// 1/sqrt(x) for positive normal x: on the device the hardware estimate
// refined by two Newton steps y <- y + y (1 - x y^2)/2, each of which squares
// its relative error (to a few ulp from the estimate's ~2^-23); on the host
// 1/sqrt(x).  Eleven instructions where the division of a correctly rounded
// square root takes about thirty.
__host__ __device__ inline double rsqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(x);
    for (int it = 0; it < 2; ++it) {
        const double r = fma(-x * y, y, 1.0);
        y = fma(y, 0.5 * r, y);
    }
    return y;
#else
    return 1.0 / std::sqrt(x);
#endif
}

// sin and cos of x, |x| < 3.2e6: x = k pi + r with |r| <= pi/2, so that
// sin x = (-1)^k sin r and cos x = (-1)^k cos r.  Reducing by pi rather than
// pi/2 leaves a sign flip of both results in place of the quadrant's swap and
// negations (one shift and two exclusive-ors where the swap took about 16
// instructions), at one more polynomial degree each.  The two-double pi
// leaves an absolute error of |k| 3e-33 in r: near the multiples of pi with
// |k| <= 16 (so throughout the polar angle's range) sin keeps its relative
// accuracy (the extra error is below 0.12 ulp); cos is accurate to 2e-17
// absolute (relative only away from its zeros).
__host__ __device__ inline void sincos(double x, double* s_out, double* c_out) {
    const NearestInt n = nearest_int(x, kInvPi);
    const double k = n.k;
    double r = fma(-k, kPiHi, x);
    r = fma(-k, kPiMid, r);
    const double z = r * r;
    // sin r = r + r z S(z), cos r = 1 + z C(z) on |r| <= pi/2: polynomial
    // kernels of degree 7 in z (generated by poly_coeffs.py; 3.6e-17 relative
    // and 1.7e-17 absolute)
    double ps = 2.7314447669863206e-15;
    ps = fma(ps, z, -7.643970296798566e-13);
    ps = fma(ps, z, 1.6058977312464087e-10);
    ps = fma(ps, z, -2.5052107616996182e-08);
    ps = fma(ps, z, 2.7557319219163234e-06);
    ps = fma(ps, z, -0.00019841269841254974);
    ps = fma(ps, z, 0.008333333333333316);
    ps = fma(ps, z, -0.16666666666666666);
    const double sr = fma(r * z, ps, r);
    double pc = 4.627675985018022e-14;
    pc = fma(pc, z, -1.1464689885720016e-11);
    pc = fma(pc, z, 2.0876630867422994e-09);
    pc = fma(pc, z, -2.755731776732053e-07);
    pc = fma(pc, z, 2.4801587292446213e-05);
    pc = fma(pc, z, -0.0013888888888860709);
    pc = fma(pc, z, 0.04166666666666634);
    pc = fma(pc, z, -0.5);
    const double cr = fma(z, pc, 1.0);
    // (-1)^k as the sign bit of the high word
    const uint64_t flip = static_cast<uint64_t>(static_cast<uint32_t>(n.i) << 31) << 32;
    *s_out = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, sr) ^ flip);
    *c_out = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, cr) ^ flip);
}

// e^r - 1 = r + r^2 E(r) for |r| <= ln(2)/2 + 1e-9: a polynomial kernel of
// degree 10 (generated by poly_coeffs.py; 8.5e-19 relative).
__host__ __device__ inline double expm1_reduced(double r) {
    double p = 2.091467937680297e-09;
    p = fma(p, r, 2.5105206374263736e-08);
    p = fma(p, r, 2.755727366134811e-07);
    p = fma(p, r, 2.75572554257457e-06);
    p = fma(p, r, 2.4801587325533363e-05);
    p = fma(p, r, 0.00019841269874800493);
    p = fma(p, r, 0.0013888888888883752);
    p = fma(p, r, 0.008333333333326141);
    p = fma(p, r, 0.04166666666666667);
    p = fma(p, r, 0.1666666666666667);
    p = fma(p, r, 0.5);
    return fma(r * r, p, r);
}

// e^x; 0 below -745, +inf above 709.8.
__host__ __device__ inline double exp(double x) {
    const double xc = fmin(fmax(x, -760.0), 720.0);
    const NearestInt n = nearest_int(xc, kInvLn2);
    const double k = n.k;
    double r = fma(-k, kLn2Hi, xc);
    r = fma(-k, kLn2Lo, r);
    return ldexp(1.0 + expm1_reduced(r), n.i);
}

// e^x - 1 without cancellation for small |x|, branch-free: with x = k ln 2 + r,
// e^x - 1 = 2^k (e^r - 1) + (2^k - 1), one fused multiply-add of exact
// operands (2^k - 1 is exact for the k that matter; k = 0 for |x| <= ln(2)/2,
// where the result is the reduced kernel itself).  -1 below -745; x is
// clamped at 709, below the overflow of e^x.
__host__ __device__ inline double expm1(double x) {
    const double xc = fmin(fmax(x, -745.0), 709.0);
    const NearestInt n = nearest_int(xc, kInvLn2);
    const double k = n.k;
    double r = fma(-k, kLn2Hi, xc);
    r = fma(-k, kLn2Lo, r);
    const double tk = ldexp(1.0, n.i);
    return fma(tk, expm1_reduced(r), tk - 1.0);
}

// e^x - 1 = x + x^2 EN(x) for x in [-kExpm1Near, 0] (+-1e-9), the range of
// the cored-NFW exponent when 0 <= eta <= kExpm1Near: no argument reduction,
// and on the half interval a polynomial kernel of degree 8 (generated by
// poly_coeffs.py; 7.4e-18 relative).
constexpr double kExpm1Near = 0.34;
__host__ __device__ inline double expm1_near(double x) {
    double p = 2.399505199127987e-07;
    p = fma(p, x, 2.7335759431393298e-06);
    p = fma(p, x, 2.4794062080910826e-05);
    p = fma(p, x, 0.00019841120114754993);
    p = fma(p, x, 0.001388888713436031);
    p = fma(p, x, 0.00833333332176611);
    p = fma(p, x, 0.041666666666284255);
    p = fma(p, x, 0.1666666666666618);
    p = fma(p, x, 0.5);
    return fma(x * x, p, x);
}

// e^x - 1 when the caller can guarantee x in [-kExpm1Near, 0] (`near`, a
// wave-uniform flag): expm1_near; otherwise the reduced form.
__host__ __device__ inline double expm1(double x, bool near) {
    return near ? expm1_near(x) : expm1(x);
}

// log m = 2 atanh(w/2) = w (1 + v LW(v)), v = w^2, for w = 2 (m - 1)/(m + 1)
// with m in [sqrt(1/2), sqrt(2)), i.e. |w| <= 0.3431458: a polynomial kernel
// of degree 6 in v (generated by poly_coeffs.py; 4.5e-18 relative).  Taking
// the quotient with the factor 2 (2m - 2 is exact) saves the doubling of the
// result.
__host__ __device__ inline double log_kernel(double w) {
    const double v = w * w;
    double p = 4.460586451734852e-06;
    p = fma(p, v, 1.8715480469428627e-05);
    p = fma(p, v, 8.878363830694202e-05);
    p = fma(p, v, 0.0004340275612264664);
    p = fma(p, v, 0.002232142861404335);
    p = fma(p, v, 0.012499999999968595);
    p = fma(p, v, 0.08333333333333337);
    return fma(w * v, p, w);
}

// v = m 2^e for a positive normal v, with m in [0.70710677, 1.41421354): the
// exponent field of v's encoding is re-based so that the split falls at the
// high word 0x3fe6a09e, just below sqrt(1/2) (the argument reduction of the
// classic fdlibm logarithm).  Integer operations on the high word and one
// conversion, where frexp, the comparison with sqrt(1/2) and the selects of m
// and e take nine instructions.  (The kernel's w then reaches 1e-7 relative
// beyond its interval's end, where the interpolant's error is still its bound.)
struct LogSplit {
    double m, e;
};
__host__ __device__ inline LogSplit log_split(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    uint32_t hi = static_cast<uint32_t>(b >> 32) + (0x3ff00000u - 0x3fe6a09eu);
    LogSplit s;
    s.e = static_cast<double>(static_cast<int32_t>(hi >> 20) - 0x3ff);
    hi = (hi & 0x000fffffu) + 0x3fe6a09eu;
    s.m = __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | (b & 0xffffffffull));
    return s;
}

// log(1 + u) for u > -1 (finite).  CORRECT = true: within a few ulp (the
// rounding error of 1 + u is carried as a first-order correction, and the
// quotient t uses the two-step reciprocal).  CORRECT = false (log1p_fast):
// neither; the error is then below 1.2e-16 absolute (half an ulp of 1 + u,
// relative to 1 + u) plus 2.2e-15 relative (the one-step reciprocal).
template <bool CORRECT>
__host__ __device__ inline double log1p_impl(double u) {
    const double v = 1.0 + u;
    double corr = 0.0;
    if (CORRECT) {
        // rounding error of 1 + u (a term below one ulp of the result: the
        // unrefined reciprocal suffices)
#if defined(__HIP_DEVICE_COMPILE__)
        corr = (u - (v - 1.0)) * __builtin_amdgcn_rcp(v);
#else
        corr = (u - (v - 1.0)) / v;
#endif
    }
    int e;
    double m = frexp(v, &e);          // v = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double w = fma(m, 2.0, -2.0) * (CORRECT ? recip(m + 1.0) : recip1(m + 1.0));
    const double logm = log_kernel(w);
    const double de = static_cast<double>(e);
    return fma(de, kLn2Hi, logm + fma(de, kLn2Lo, corr));
}

__host__ __device__ inline double log1p(double u) { return log1p_impl<true>(u); }

// For the cored-NFW mass function (R/lambda_c >= R_+/lambda_c): there the
// logarithm enters F only through the halo term, so its error reaches F as a
// relative error below about 1e-15, far below the integrator's tolerance, and
// the correction and the second reciprocal step would cost about 5 % of the
// trace.
__host__ __device__ inline double log1p_fast(double u) { return log1p_impl<false>(u); }

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

// Binary32 versions for the single-precision bulk trace: the same methods with
// binary32 reduction constants and lower-degree kernels (poly_coeffs.py; each
// approximation below 3.4e-9 relative, a twentieth of a binary32 ulp), the
// hardware reciprocal (about one binary32 ulp) and the binary32 estimate of
// x^(-1/10) (4.2e-7).
constexpr float kPio2HiF = 1.5707963705062866f;
constexpr float kPio2MidF = -4.371138828673793e-08f;
constexpr float kPio2LoF = -1.7151245100058819e-15f;
constexpr float kTwoOverPiF = 0.6366197466850281f;
constexpr float kLn2HiF = 0.6931471824645996f;
constexpr float kLn2LoF = -1.9046542121259336e-09f;
constexpr float kInvLn2F = 1.4426950216293335f;

// nearest_int in binary32 (shift 1.5 2^23): for |a x| < 2^22.
constexpr float kRoundShiftF = 12582912.0f;
struct NearestIntF {
    float k;
    int32_t i;
};
__host__ __device__ inline NearestIntF nearest_int(float a, float x) {
    const float kk = fmaf(a, x, kRoundShiftF);
    NearestIntF n;
    n.k = kk - kRoundShiftF;
    n.i = static_cast<int32_t>(__builtin_bit_cast(uint32_t, kk) - 0x4B400000u);
    return n;
}

__host__ __device__ inline float recip(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
__host__ __device__ inline float recip1(float x) { return recip(x); }

// sin and cos of x, |x| < 1e4.
__host__ __device__ inline void sincos(float x, float* s_out, float* c_out) {
    const NearestIntF n = nearest_int(x, kTwoOverPiF);
    const float k = n.k;
    float r = fmaf(-k, kPio2HiF, x);
    r = fmaf(-k, kPio2MidF, r);
    r = fmaf(-k, kPio2LoF, r);
    const float z = r * r;
    float ps = 2.7249925551586784e-06f;
    ps = fmaf(ps, z, -0.00019840087043121457f);
    ps = fmaf(ps, z, 0.008333331905305386f);
    ps = fmaf(ps, z, -0.1666666716337204f);
    const float sr = fmaf(r * z, ps, r);
    float pc = 2.4463788577122614e-05f;
    pc = fmaf(pc, z, -0.0013887588866055012f);
    pc = fmaf(pc, z, 0.04166664928197861f);
    pc = fmaf(pc, z, -0.5f);
    const float cr = fmaf(z, pc, 1.0f);
    const int q = n.i & 3;
    float s = (q & 1) ? cr : sr;
    float c = (q & 1) ? sr : cr;
    if (q & 2) s = -s;
    if ((q + 1) & 2) c = -c;
    *s_out = s;
    *c_out = c;
}

// e^r - 1 for |r| <= ln(2)/2 + 1e-9.
__host__ __device__ inline float expm1_reduced(float r) {
    float p = 0.00019890980911441147f;
    p = fmaf(p, r, 0.0013933641603216529f);
    p = fmaf(p, r, 0.00833331048488617f);
    p = fmaf(p, r, 0.04166646674275398f);
    p = fmaf(p, r, 0.1666666716337204f);
    p = fmaf(p, r, 0.5f);
    return fmaf(r * r, p, r);
}

// e^x, x clamped to [-104, 88.7].
__host__ __device__ inline float exp(float x) {
    const float xc = fminf(fmaxf(x, -104.0f), 88.7f);
    const NearestIntF n = nearest_int(xc, kInvLn2F);
    const float k = n.k;
    float r = fmaf(-k, kLn2HiF, xc);
    r = fmaf(-k, kLn2LoF, r);
    return ldexpf(1.0f + expm1_reduced(r), n.i);
}

// e^x - 1 (the binary64 method: 2^k (e^r - 1) + (2^k - 1)); -1 below -104.
__host__ __device__ inline float expm1(float x) {
    const float xc = fminf(fmaxf(x, -104.0f), 88.0f);
    const NearestIntF n = nearest_int(xc, kInvLn2F);
    const float k = n.k;
    float r = fmaf(-k, kLn2HiF, xc);
    r = fmaf(-k, kLn2LoF, r);
    const float tk = ldexpf(1.0f, n.i);
    return fmaf(tk, expm1_reduced(r), tk - 1.0f);
}
__host__ __device__ inline float expm1(float x, bool near) {
    return near ? expm1_reduced(x) : expm1(x);
}

// log(1 + u) for u > -1 (finite).
template <bool CORRECT>
__host__ __device__ inline float log1p_impl(float u) {
    const float v = 1.0f + u;
    const float corr = CORRECT ? (u - (v - 1.0f)) * recip(v) : 0.0f;
    int e;
    float m = frexpf(v, &e);
    if (m < 0.70710678f) {
        m *= 2.0f;
        e -= 1;
    }
    const float t = (m - 1.0f) * recip(m + 1.0f);
    const float z = t * t;
    float p = 0.14789974689483643f;
    p = fmaf(p, z, 0.1999439001083374f);
    p = fmaf(p, z, 0.33333343267440796f);
    const float logm = 2.0f * fmaf(t * z, p, t);
    const float de = static_cast<float>(e);
    return fmaf(de, kLn2HiF, logm + fmaf(de, kLn2LoF, corr));
}
__host__ __device__ inline float log1p(float u) { return log1p_impl<true>(u); }
// Without the correction for the rounding of 1 + u: 6e-8 absolute more.
__host__ __device__ inline float log1p_fast(float u) { return log1p_impl<false>(u); }

__host__ __device__ inline float rpow_tenth(float x) { return rpow_tenth_estimate(x); }

}  // namespace dm
}  // namespace rt
