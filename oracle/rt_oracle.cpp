// rt_oracle.cpp -- CPU reference ("oracle") for the backward null-geodesic ray
// tracer of M. Fathi, "Adaptive ray tracing, image diagnostics, and photon ring
// signatures of rotating dark-matter-dressed black holes".
//
// TEST INFRASTRUCTURE ONLY.  This file is not part of the product path: only
// the test suite, the smoke check and the benchmark's CPU-baseline leg may
// load it.  It shares no source, header, table or helper with the HIP library
// and includes none of it.
//
// Everything is scalar IEEE binary64, written for readability, not speed.
// Build flags (oracle/build_oracle.py): -O2 -ffp-contract=off, no fast-math.
// The physics is written once, as templates over the scalar type: T = double
// for the trace, T = Dual<4> (value plus derivatives along chi, theta_o and
// the two halo parameters) for the image gradient.  A Dual's value part is
// computed with exactly the double expressions, so a dual run takes the same
// decisions as the double run.
//
// Conventions (paper Sec. 2, eq. (1)): M = 1, R = r/M, T = t/M, chi = a/M.
// State of a ray: y = (T, R, theta, phi, p_R, p_theta); E = -p_T and
// l = p_phi are constants of motion (Sec. 3.1, eq. (48)).
//
// Readings where the paper is silent:
//  * integrator: Dormand-Prince 5(4) with its 4th-order continuous extension
//    (Dormand & Prince 1980; Hairer, Norsett & Wanner, Solving ODEs I, II.5-6),
//    standard step controller (safety 0.9, factor in [0.2, 10], exponent -1/5,
//    no growth right after a rejection), RMS error norm over all six
//    components with scale atol + rtol*max(|y|,|y_new|), first step h0.
//  * capture R <= r_stop_fac * R_+ and escape R >= r_esc_fac * R_o, both tested
//    at the end of each accepted step (Sec. 3.3, eq. (75)).
//  * the equatorial plane is theta = pi/2 (mod pi): Boyer-Lindquist theta is
//    continued through the poles (a ray with l = 0 passes over the axis and
//    theta leaves (0, pi); (theta, phi) and (-theta, phi + pi) are the same
//    point).  The band index k = floor((theta - pi/2)/pi) labels the regions
//    between equatorial passages; an equatorial crossing is a change of k
//    across an accepted step (for theta in (0, pi) that is a change of the
//    boolean theta >= pi/2).  Its position is the root of the continuous
//    extension's theta(s) - theta_eq on s in [0,1], theta_eq = pi/2 + k pi for
//    the larger of the two band indices, found by 60 bisections (Sec. 3.3,
//    eq. (76)); where theta_eq = -pi/2 (mod 2 pi) the point's azimuth is
//    phi + pi.  A crossing is trusted when |dtheta/dlambda| >= 1e-12 at the
//    root and the affine gap to the previous trusted crossing is >= 1e-10
//    (Sec. 4.2).  Crossings of the final step count before the stop test.
//  * a ray whose error estimate is not finite on kNonfiniteRun consecutive
//    attempts (its step shrunk by 0.2 each time, to ~1e-14 of where it
//    started) ends with status NONFINITE.
//  * thin-disc intensity: I = sum_{n<3} w(R_n) g_n^3 R_n^(-emis_pow), the
//    equatorial limit of eq. (88) with the emitter of eqs. (89)-(91); g = 0
//    where no timelike circular orbit exists.
//  * gradient: the derivative of the computed discrete map.  Step sizes,
//    accept/reject decisions, the crossing steps and the termination step are
//    held fixed; the crossing position follows the implicit-function theorem
//    on theta(s) = pi/2 and the outer horizon on Delta(R_+) = 0.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace {

// ---------------------------------------------------------------- parameters
enum : int32_t { KERR = 0, EINASTO = 1, CNFW = 2 };

// Status codes of a traced ray.
enum : int32_t { RUNNING = 0, CAPTURED = 1, ESCAPED = 2, STEP_LIMIT = 3, NONFINITE = 4 };

}  // namespace

extern "C" {

// Parameters of one image.  Field order mirrors the ctypes Structure in
// oracle/oracle.py; keep the two in step.
struct OrcParams {
    int32_t metric;        // KERR, EINASTO or CNFW
    int32_t max_attempts;  // step-attempt budget per ray
    double spin;           // chi
    double halo0;          // Einasto: lambda_E;  cNFW: eta
    double halo1;          // cNFW: lambda_c
    double incl;           // theta_o [rad]
    double r_obs;          // R_o
    int32_t nx, ny;        // screen pixels
    double x_min, x_max, y_min, y_max;  // screen extent; pixel centres inside
    double rtol, atol;     // Dormand-Prince tolerances
    double r_stop_fac;     // capture at R <= r_stop_fac * R_+
    double r_esc_fac;      // escape at R >= r_esc_fac * R_o
    double r_in;           // inner disc edge; <= 0 means R_+
    double r_out;          // outer disc edge
    double emis_pow;       // emissivity exponent p in R^-p
    double sigma_in;       // taper widths; both > 0 selects eqs. (85)-(86)
    double sigma_out;
    double h0;             // first trial step
};

// Everything the oracle knows about one ray.
struct OrcRay {
    int32_t status;
    int32_t ncross;        // trusted crossings, saturating at 255
    int32_t attempts;      // step attempts (accepted + rejected)
    int32_t accepted;
    int32_t filtered;      // crossings rejected by the trust filter
    int32_t pad;
    double E, L;           // constants of motion
    double r_em[3], phi_em[3], t_em[3], g_em[3], i_n[3];
    double intensity;
    double lambda_end;     // affine parameter at termination
    double max_constraint; // max over accepted states of |2 Sigma H| / (sum of |terms|)
    double carter_drift;   // max over accepted states of |K/K0 - 1|
    double y_end[6];
};

}  // extern "C"

namespace {

constexpr double kNaN = std::numeric_limits<double>::quiet_NaN();
constexpr double kHalfPi = 1.57079632679489661923;
constexpr double kPi = 3.14159265358979323846;
constexpr int kNonfiniteRun = 20;

// Band index of theta between equatorial passages: theta = pi/2 + k pi is the
// equator, band k holds [pi/2 + k pi, pi/2 + (k + 1) pi).
double equator_band(double theta) { return std::floor((theta - kHalfPi) / kPi); }

// Fault injection for the failure-handling tests: attempts numbered
// [g_fault_from, g_fault_to] (1-based, per ray) get a non-finite error
// estimate, as a stage that produced NaN would give.  Off by default.
int g_fault_from = 0, g_fault_to = -1;

// ----------------------------------------------------------- dual numbers
// Forward-mode dual number: value v and N directional derivatives d.
template <int N>
struct Dual {
    double v = 0.0;
    double d[N] = {};
    Dual() = default;
    Dual(double x) : v(x) {}  // NOLINT: constants promote implicitly
};

template <int N>
Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v + b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N>
Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v - b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N>
Dual<N> operator-(const Dual<N>& a) {
    Dual<N> r(-a.v);
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N>
Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v * b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N>
Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v / b.v);
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
    return r;
}
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }

// Elementary functions: chain rule with the libm value.
template <int N>
Dual<N> chain(const Dual<N>& a, double value, double deriv) {
    Dual<N> r(value);
    for (int i = 0; i < N; ++i) r.d[i] = deriv * a.d[i];
    return r;
}
template <int N> Dual<N> exp(const Dual<N>& a) { const double e = std::exp(a.v); return chain(a, e, e); }
template <int N> Dual<N> expm1(const Dual<N>& a) { return chain(a, std::expm1(a.v), std::exp(a.v)); }
template <int N> Dual<N> log1p(const Dual<N>& a) { return chain(a, std::log1p(a.v), 1.0 / (1.0 + a.v)); }
template <int N> Dual<N> sin(const Dual<N>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int N> Dual<N> cos(const Dual<N>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int N> Dual<N> sqrt(const Dual<N>& a) { const double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int N> Dual<N> tanh(const Dual<N>& a) { const double t = std::tanh(a.v); return chain(a, t, 1.0 - t * t); }
template <int N>
Dual<N> pow(const Dual<N>& a, double b) {
    return chain(a, std::pow(a.v, b), b * std::pow(a.v, b - 1.0));
}
template <int N> Dual<N> fabs(const Dual<N>& a) { return a.v < 0.0 ? -a : a; }
template <int N> Dual<N> fmax(const Dual<N>& a, const Dual<N>& b) { return (a.v >= b.v || std::isnan(b.v)) ? a : b; }
template <int N> Dual<N> fmin(const Dual<N>& a, const Dual<N>& b) { return (a.v <= b.v || std::isnan(b.v)) ? a : b; }

inline double val(double x) { return x; }
template <int N> double val(const Dual<N>& x) { return x.v; }

using std::cos;
using std::exp;
using std::expm1;
using std::fabs;
using std::fmax;
using std::fmin;
using std::log1p;
using std::pow;
using std::sin;
using std::sqrt;
using std::tanh;

// The differentiable parameters of an image: spin, inclination, halo.
template <class T>
struct Phys {
    T chi, incl, h0, h1;
};

Phys<double> phys_of(const OrcParams& p) { return {p.spin, p.incl, p.halo0, p.halo1}; }

// Parameters seeded as the four derivative directions (chi, theta_o, halo0, halo1).
Phys<Dual<4>> phys_seeded(const OrcParams& p) {
    Phys<Dual<4>> q{Dual<4>(p.spin), Dual<4>(p.incl), Dual<4>(p.halo0), Dual<4>(p.halo1)};
    q.chi.d[0] = 1.0;
    q.incl.d[1] = 1.0;
    q.h0.d[2] = 1.0;
    q.h1.d[3] = 1.0;
    return q;
}

// ------------------------------------------------------- Sec. 2.1: the seeds
// Radial functions of one metric at radius R: the lapse H_i (eqs. (9), (13)),
// the mass function mu_i (eq. (15)), F_i = 2 R mu_i (eq. (24)) and
// derivatives.  mu_i is evaluated in a form that is algebraically identical
// to R(1 - H_i)/2 but free of cancellation, so that Kerr is reproduced
// exactly when the halo term vanishes (e^{-R/lambda_E} underflows, or
// eta = 0).
template <class T>
struct Radial {
    T H, dH, mu, dmu, F, dF;
};

template <class T>
Radial<T> radial(const OrcParams& p, const Phys<T>& q, const T& R) {
    Radial<T> o{};
    if (p.metric == EINASTO) {
        // eq. (9): H_E = 1 - 2/R + (2/R + 2/lam + R/lam^2) exp(-R/lam)
        // => mu_E = 1 - exp(-x)(1 + x + x^2/2), x = R/lam  (eq. (15))
        const T lam = q.h0;
        const T x = R / lam;
        const T ex = exp(-x);
        o.mu = 1.0 - ex * (1.0 + x + 0.5 * x * x);
        o.dmu = ex * 0.5 * x * x / lam;
    } else if (p.metric == CNFW) {
        // eq. (13): H_cNFW = exp(Ex) - 2/R with
        // Ex = eta lam_c [1/(R+lam_c) - (2/R) ln(1 + R/lam_c)]
        // => mu = 1 - (R/2)(exp(Ex) - 1)  (eq. (15))
        const T eta = q.h0, lc = q.h1;
        const T lg = log1p(R / lc);
        const T ex = eta * lc * (1.0 / (R + lc) - 2.0 / R * lg);
        const T dex = eta * lc * (-1.0 / ((R + lc) * (R + lc)) + 2.0 / (R * R) * lg
                                  - 2.0 / (R * (R + lc)));
        const T em1 = expm1(ex);
        o.mu = 1.0 - 0.5 * R * em1;
        o.dmu = -0.5 * em1 - 0.5 * R * exp(ex) * dex;
    } else {
        o.mu = T(1.0);  // Schwarzschild seed H = 1 - 2/R
        o.dmu = T(0.0);
    }
    o.H = 1.0 - 2.0 * o.mu / R;                       // eq. (8)
    o.dH = -2.0 * o.dmu / R + 2.0 * o.mu / (R * R);
    o.F = 2.0 * R * o.mu;                             // eq. (24)
    o.dF = 2.0 * o.mu + 2.0 * R * o.dmu;
    return o;
}

// --------------------------------------------- Sec. 2.2 / 3.1: the metric
template <class T>
struct Metric {
    T F, dF, Delta, dDelta, Sigma;
    T g_TT, g_Tph, g_RR, g_thth, g_phph;             // eqs. (27)-(31)
    T u_TT, u_Tph, u_RR, u_thth, u_phph;             // eqs. (49)-(53)
    T dR_TT, dR_Tph, dR_RR, dR_thth, dR_phph;        // d/dR of (49)-(53)
    T dt_TT, dt_Tph, dt_RR, dt_thth, dt_phph;        // d/dtheta of (49)-(53)
};

template <class T>
Metric<T> metric(const OrcParams& p, const Phys<T>& q, const T& R, const T& th) {
    Metric<T> m{};
    const Radial<T> r = radial(p, q, R);
    const T chi = q.chi, chi2 = chi * chi;
    const T s = sin(th), c = cos(th);
    const T s2 = s * s;
    m.F = r.F;
    m.dF = r.dF;
    m.Sigma = R * R + chi2 * c * c;               // eq. (23)
    m.Delta = R * R - r.F + chi2;                 // eq. (25)
    m.dDelta = 2.0 * R - r.dF;
    const T Sg = m.Sigma, D = m.Delta, F = r.F;

    // covariant components, eqs. (27)-(31)
    m.g_TT = -(1.0 - F / Sg);
    m.g_Tph = -chi * F * s2 / Sg;
    m.g_RR = Sg / D;
    m.g_thth = Sg;
    m.g_phph = s2 * (R * R + chi2 + chi2 * F * s2 / Sg);

    // contravariant components, eqs. (49)-(53)
    const T A = (R * R + chi2) * (R * R + chi2) - chi2 * D * s2;
    const T SD = Sg * D;
    const T B = D - chi2 * s2;
    m.u_TT = -A / SD;
    m.u_Tph = -chi * F / SD;
    m.u_RR = D / Sg;
    m.u_thth = 1.0 / Sg;
    m.u_phph = B / (SD * s2);

    // radial derivatives (Sigma_R = 2R, Delta_R = dDelta; sin(theta) fixed)
    const T Sg_R = 2.0 * R, D_R = m.dDelta;
    const T A_R = 4.0 * R * (R * R + chi2) - chi2 * s2 * D_R;
    const T SD_R = Sg_R * D + Sg * D_R;
    const T B_R = D_R;
    m.dR_TT = -(A_R * SD - A * SD_R) / (SD * SD);
    m.dR_Tph = -chi * (r.dF * SD - F * SD_R) / (SD * SD);
    m.dR_RR = (D_R * Sg - D * Sg_R) / (Sg * Sg);
    m.dR_thth = -Sg_R / (Sg * Sg);
    m.dR_phph = (B_R * SD - B * SD_R) / (SD * SD * s2);

    // polar derivatives (Sigma_th = -2 chi^2 s c, (s^2)_th = 2 s c; Delta fixed)
    const T Sg_t = -2.0 * chi2 * s * c, s2_t = 2.0 * s * c;
    const T A_t = -chi2 * D * s2_t;
    const T SD_t = Sg_t * D;
    const T B_t = -chi2 * s2_t;
    const T Q = SD * s2, Q_t = SD_t * s2 + SD * s2_t;
    m.dt_TT = -(A_t * SD - A * SD_t) / (SD * SD);
    m.dt_Tph = chi * F * SD_t / (SD * SD);
    m.dt_RR = -D * Sg_t / (Sg * Sg);
    m.dt_thth = -Sg_t / (Sg * Sg);
    m.dt_phph = (B_t * Q - B * Q_t) / (Q * Q);
    return m;
}

// eq. (54): 2 H = g^{ab} p_a p_b with p_T = -E, p_phi = l.
template <class T>
T two_hamiltonian(const Metric<T>& m, const T& E, const T& L, const T& pR, const T& pth) {
    const T pT = -E, pph = L;
    return m.u_TT * pT * pT + 2.0 * m.u_Tph * pT * pph + m.u_phph * pph * pph
         + m.u_RR * pR * pR + m.u_thth * pth * pth;
}

// Hamilton's equations (46)-(47), written out as eqs. (57)-(62).
template <class T>
void rhs(const OrcParams& p, const Phys<T>& q, const T& E, const T& L, const T y[6], T dy[6]) {
    const T R = y[1], th = y[2], pR = y[4], pth = y[5];
    const Metric<T> m = metric(p, q, R, th);
    const T pT = -E, pph = L;
    dy[0] = m.u_TT * pT + m.u_Tph * pph;              // eq. (57)
    dy[1] = m.u_RR * pR;                               // eq. (59)
    dy[2] = m.u_thth * pth;                            // eq. (60)
    dy[3] = m.u_Tph * pT + m.u_phph * pph;             // eq. (58)
    dy[4] = -0.5 * (m.dR_TT * pT * pT + 2.0 * m.dR_Tph * pT * pph + m.dR_phph * pph * pph
                    + m.dR_RR * pR * pR + m.dR_thth * pth * pth);   // eq. (61)
    dy[5] = -0.5 * (m.dt_TT * pT * pT + 2.0 * m.dt_Tph * pT * pph + m.dt_phph * pph * pph
                    + m.dt_RR * pR * pR + m.dt_thth * pth * pth);   // eq. (62)
}

// -------------------------------------------------- Sec. 2.3: horizons
// Outer horizon: the largest root of Delta_i(R) = 0 (eq. (33)).  Delta is
// sampled downward from R = 50 in steps of 1e-3; the first sign change
// (Delta > 0 above, <= 0 below) is refined by bisection to a bracket of
// relative width 4 eps.  Returns false when there is no root.
bool outer_horizon(const OrcParams& p, double* r_plus) {
    const Phys<double> q = phys_of(p);
    auto Delta = [&](double R) {
        const Radial<double> r = radial(p, q, R);
        return R * R - r.F + p.spin * p.spin;
    };
    const double step = 1e-3;
    double hi = 50.0;
    if (!(Delta(hi) > 0.0)) return false;
    for (long k = 1;; ++k) {
        const double lo = 50.0 - static_cast<double>(k) * step;
        if (lo < 0.05) return false;
        if (Delta(lo) <= 0.0) {
            double a = lo, b = hi;  // Delta(a) <= 0 < Delta(b)
            for (int it = 0; it < 200 && (b - a) > 4.0 * 2.220446049250313e-16 * b; ++it) {
                const double mid = 0.5 * (a + b);
                if (Delta(mid) > 0.0) b = mid; else a = mid;
            }
            *r_plus = 0.5 * (a + b);
            return true;
        }
        hi = lo;
    }
}

// The horizon as a function of the parameters: the root's value from
// outer_horizon, its derivatives from Delta(R_+(q), q) = 0.
template <class T>
T horizon_of(const OrcParams& p, const Phys<T>& q, double r_plus);

template <>
double horizon_of(const OrcParams&, const Phys<double>&, double r_plus) { return r_plus; }

template <>
Dual<4> horizon_of(const OrcParams& p, const Phys<Dual<4>>& q, double r_plus) {
    const Dual<4> R(r_plus);
    const Radial<Dual<4>> r = radial(p, q, R);
    const Dual<4> D = R * R - r.F + q.chi * q.chi;
    Dual<4> out(r_plus);
    const double dD_dR = 2.0 * r_plus - r.dF.v;
    for (int i = 0; i < 4; ++i) out.d[i] = -D.d[i] / dD_dR;
    return out;
}

// Extremal spin (eqs. (34)-(37)): chi_e^2 = -R_e^2 H(R_e) at the deepest
// minimum of R^2 H(R), where 2H + R H' = 0.  Returns false when R^2 H has no
// negative minimum (no horizon for any spin).
bool extremal_spin(const OrcParams& p0, double* chi_e, double* r_e) {
    OrcParams p = p0;
    p.spin = 0.0;
    const Phys<double> q = phys_of(p);
    auto D = [&](double R) { const Radial<double> r = radial(p, q, R); return 2.0 * r.H + R * r.dH; };
    auto V = [&](double R) { const Radial<double> r = radial(p, q, R); return R * R * r.H; };
    double best = 0.0, best_r = kNaN;
    const double step = 1e-3;
    double a = 0.01, Da = D(a);
    for (long k = 1; a < 50.0; ++k) {
        const double b = 0.01 + static_cast<double>(k) * step;
        const double Db = D(b);
        if (Da < 0.0 && Db >= 0.0) {  // d(R^2 H)/dR = R (2H + R H') goes - to +: a minimum
            double lo = a, hi = b;
            for (int it = 0; it < 200 && (hi - lo) > 4.0 * 2.220446049250313e-16 * hi; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (D(mid) < 0.0) lo = mid; else hi = mid;
            }
            const double rm = 0.5 * (lo + hi);
            const double v = V(rm);
            if (v < best) { best = v; best_r = rm; }
        }
        a = b;
        Da = Db;
    }
    if (!(best < 0.0)) return false;
    *chi_e = std::sqrt(-best);
    *r_e = best_r;
    return true;
}

// ------------------------------------------- Sec. 3.2: observer and screen
template <class T>
struct Observer {
    Metric<T> m;
    T omega, N;
    T u[4];                    // u_o^mu, eqs. (64)-(65)
    T eR[4], eth[4], eph[4];   // eqs. (66)-(68)
};

template <class T>
Observer<T> observer(const OrcParams& p, const Phys<T>& q) {
    Observer<T> o{};
    o.m = metric(p, q, T(p.r_obs), q.incl);
    const Metric<T>& m = o.m;
    o.omega = -m.g_Tph / m.g_phph;                                               // eq. (63)
    o.N = sqrt(-(m.g_TT + 2.0 * o.omega * m.g_Tph + o.omega * o.omega * m.g_phph));  // eq. (65)
    const T zero(0.0);
    const T u[4] = {1.0 / o.N, zero, zero, o.omega / o.N};                       // eq. (64)
    const T eR[4] = {zero, 1.0 / sqrt(m.g_RR), zero, zero};
    const T et[4] = {zero, zero, 1.0 / sqrt(m.g_thth), zero};
    const T ep[4] = {zero, zero, zero, 1.0 / sqrt(m.g_phph)};
    for (int i = 0; i < 4; ++i) {
        o.u[i] = u[i];
        o.eR[i] = eR[i];
        o.eth[i] = et[i];
        o.eph[i] = ep[i];
    }
    return o;
}

// Lower an index with the metric at the observer: p_mu = g_{mu nu} p^nu (eq. (74)).
template <class T>
void lower(const Metric<T>& m, const T up[4], T dn[4]) {
    dn[0] = m.g_TT * up[0] + m.g_Tph * up[3];
    dn[1] = m.g_RR * up[1];
    dn[2] = m.g_thth * up[2];
    dn[3] = m.g_Tph * up[0] + m.g_phph * up[3];
}

// Screen point (X, Y) -> initial momentum, eqs. (70)-(74) with E_loc = 1.
template <class T>
void initial_momentum(const Observer<T>& o, double r_obs, double X, double Y, T p_up[4],
                      T p_dn[4]) {
    const double d = std::sqrt(r_obs * r_obs + X * X + Y * Y);
    const double nR = -r_obs / d, nth = -Y / d, nph = -X / d;  // eqs. (70)-(72)
    for (int mu = 0; mu < 4; ++mu)                               // eq. (73)
        p_up[mu] = o.u[mu] + nR * o.eR[mu] + nth * o.eth[mu] + nph * o.eph[mu];
    lower(o.m, p_up, p_dn);                                      // eq. (74)
}

// ------------------------------------- Dormand-Prince 5(4) (reading, above)
// Butcher tableau of Dormand & Prince (1980).
const double A21 = 1.0 / 5.0;
const double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
const double A41 = 44.0 / 45.0, A42 = -56.0 / 15.0, A43 = 32.0 / 9.0;
const double A51 = 19372.0 / 6561.0, A52 = -25360.0 / 2187.0, A53 = 64448.0 / 6561.0,
             A54 = -212.0 / 729.0;
const double A61 = 9017.0 / 3168.0, A62 = -355.0 / 33.0, A63 = 46732.0 / 5247.0,
             A64 = 49.0 / 176.0, A65 = -5103.0 / 18656.0;
// 5th-order weights (also row 7 of the tableau: first-same-as-last).
const double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0,
             B5 = -2187.0 / 6784.0, B6 = 11.0 / 84.0;
// 4th-order embedded weights.
const double BH1 = 5179.0 / 57600.0, BH3 = 7571.0 / 16695.0, BH4 = 393.0 / 640.0,
             BH5 = -92097.0 / 339200.0, BH6 = 187.0 / 2100.0, BH7 = 1.0 / 40.0;
// Continuous extension: y(lambda + s h) = y + h sum_i k_i b_i(s), where
// b_i(s) = sum_{j=1..4} DENSE[i][j-1] s^j  (Hairer-Norsett-Wanner, II.6).
const double DENSE[7][4] = {
    {1.0, -8048581381.0 / 2820520608.0, 8663915743.0 / 2820520608.0,
     -12715105075.0 / 11282082432.0},
    {0.0, 0.0, 0.0, 0.0},
    {0.0, 131558114200.0 / 32700410799.0, -68118460800.0 / 10900136933.0,
     87487479700.0 / 32700410799.0},
    {0.0, -1754552775.0 / 470086768.0, 14199869525.0 / 1410260304.0,
     -10690763975.0 / 1880347072.0},
    {0.0, 127303824393.0 / 49829197408.0, -318862633887.0 / 49829197408.0,
     701980252875.0 / 199316789632.0},
    {0.0, -282668133.0 / 205662961.0, 2019193451.0 / 616988883.0,
     -1453857185.0 / 822651844.0},
    {0.0, 40617522.0 / 29380423.0, -110615467.0 / 29380423.0, 69997945.0 / 29380423.0}};

template <class T>
struct Step {
    T k[7][6];
    T y_new[6];
    T err;  // RMS scaled error norm
};

// One attempted step from y (with k1 = f(y) already known) of size h.
template <class T>
void dp5_attempt(const OrcParams& p, const Phys<T>& q, const T& E, const T& L, const T y[6],
                 const T k1[6], double h, Step<T>* st) {
    T tmp[6];
    for (int i = 0; i < 6; ++i) st->k[0][i] = k1[i];
    for (int i = 0; i < 6; ++i) tmp[i] = y[i] + h * (A21 * st->k[0][i]);
    rhs(p, q, E, L, tmp, st->k[1]);
    for (int i = 0; i < 6; ++i) tmp[i] = y[i] + h * (A31 * st->k[0][i] + A32 * st->k[1][i]);
    rhs(p, q, E, L, tmp, st->k[2]);
    for (int i = 0; i < 6; ++i)
        tmp[i] = y[i] + h * (A41 * st->k[0][i] + A42 * st->k[1][i] + A43 * st->k[2][i]);
    rhs(p, q, E, L, tmp, st->k[3]);
    for (int i = 0; i < 6; ++i)
        tmp[i] = y[i] + h * (A51 * st->k[0][i] + A52 * st->k[1][i] + A53 * st->k[2][i]
                             + A54 * st->k[3][i]);
    rhs(p, q, E, L, tmp, st->k[4]);
    for (int i = 0; i < 6; ++i)
        tmp[i] = y[i] + h * (A61 * st->k[0][i] + A62 * st->k[1][i] + A63 * st->k[2][i]
                             + A64 * st->k[3][i] + A65 * st->k[4][i]);
    rhs(p, q, E, L, tmp, st->k[5]);
    for (int i = 0; i < 6; ++i)
        st->y_new[i] = y[i] + h * (B1 * st->k[0][i] + B3 * st->k[2][i] + B4 * st->k[3][i]
                                   + B5 * st->k[4][i] + B6 * st->k[5][i]);
    rhs(p, q, E, L, st->y_new, st->k[6]);
    T acc(0.0);
    for (int i = 0; i < 6; ++i) {
        const T e5m4 = h * ((B1 - BH1) * st->k[0][i] + (B3 - BH3) * st->k[2][i]
                            + (B4 - BH4) * st->k[3][i] + (B5 - BH5) * st->k[4][i]
                            + (B6 - BH6) * st->k[5][i] + (0.0 - BH7) * st->k[6][i]);
        const T sc = p.atol + p.rtol * fmax(fabs(y[i]), fabs(st->y_new[i]));
        const T qq = e5m4 / sc;
        acc = acc + qq * qq;
    }
    st->err = sqrt(acc / 6.0);
}

// Component i of the continuous extension at fraction s of an accepted step.
template <class T, class S>
T dense(const T y[6], const Step<T>& st, double h, int i, const S& s) {
    T acc(0.0);
    for (int j = 0; j < 7; ++j) {
        const S bj = s * (DENSE[j][0] + s * (DENSE[j][1] + s * (DENSE[j][2] + s * DENSE[j][3])));
        acc = acc + bj * st.k[j][i];
    }
    return y[i] + h * acc;
}

// d/ds of component i of the continuous extension.
template <class T>
T dense_ds(const Step<T>& st, double h, int i, double s) {
    T acc(0.0);
    for (int j = 0; j < 7; ++j) {
        const double dbj = DENSE[j][0] + s * (2.0 * DENSE[j][1] + s * (3.0 * DENSE[j][2]
                                                                       + s * 4.0 * DENSE[j][3]));
        acc = acc + dbj * st.k[j][i];
    }
    return h * acc;
}

// The crossing root as a function of the parameters: its value is the
// bisection's s; for dual numbers its derivatives follow from
// theta(s*(q), q) = pi/2, i.e. ds* = -(d theta at fixed s) / (d theta / d s).
inline double root_of(double s, double, const Step<double>&, double) { return s; }

Dual<4> root_of(double s, const Dual<4>& th_minus_half_pi, const Step<Dual<4>>& st, double h) {
    const double slope = dense_ds(st, h, 2, s).v;
    Dual<4> out(s);
    for (int i = 0; i < 4; ++i) out.d[i] = -th_minus_half_pi.d[i] / slope;
    return out;
}

// ----------------------------------------- Sec. 5.2: redshift and emission
// Keplerian emitter on the equator at radius R (eqs. (89)-(91)); returns g for
// a photon with constants (E, l) and observer-frame energy obs_energy
// (= -p.u_obs, eq. (89) numerator).  Returns 0 when no timelike circular orbit
// exists at R.
template <class T>
T redshift(const OrcParams& p, const Phys<T>& q, const T& R, const T& E, const T& L,
           const T& obs_energy) {
    // d/dR of g_TT, g_Tphi, g_phiphi at theta = pi/2 (eqs. (27), (28), (31)),
    // by the same chain rule as the metric: with Sigma = R^2 there,
    // g_TT = -(1 - F/R^2), g_Tphi = -chi F/R^2, g_phiphi = R^2 + chi^2 + chi^2 F/R^2.
    const Radial<T> r = radial(p, q, R);
    const T chi = q.chi, chi2 = chi * chi;
    const T dFoR2 = r.dF / (R * R) - 2.0 * r.F / (R * R * R);
    const T dgTT = dFoR2;
    const T dgTph = -chi * dFoR2;
    const T dgphph = 2.0 * R + chi2 * dFoR2;
    const T disc = dgTph * dgTph - dgTT * dgphph;
    if (!(val(disc) >= 0.0)) return T(0.0);
    const T Om = (-dgTph + sqrt(disc)) / dgphph;                      // eq. (91)
    const Metric<T> m = metric(p, q, R, T(kHalfPi));
    const T A = -(m.g_TT + 2.0 * Om * m.g_Tph + Om * Om * m.g_phph);
    if (!(val(A) > 0.0)) return T(0.0);
    const T uT = 1.0 / sqrt(A);                                       // u.u = -1
    const T em_energy = uT * (E - Om * L);                            // -p_mu u_em^mu, eq. (90)
    if (!(val(em_energy) > 0.0)) return T(0.0);
    return obs_energy / em_energy;                                    // eq. (89)
}

// Disc window at equatorial radius R: hard edges (eq. (77)) or the tanh
// tapers of eqs. (85)-(86) with rho = R on the equator.
template <class T>
T window(const OrcParams& p, const T& R, const T& r_in) {
    if (p.sigma_in > 0.0 && p.sigma_out > 0.0) {
        const T tin = 0.5 * (1.0 + tanh((R - r_in) / p.sigma_in));
        const T tout = 0.5 * (1.0 - tanh((R - p.r_out) / p.sigma_out));
        return tin * tout;
    }
    return T((val(R) >= val(r_in) && val(R) <= p.r_out) ? 1.0 : 0.0);
}

// Normalised null-constraint residual and Carter-like constant K (Sec. 3.1,
// eq. (56): K = p_theta^2 + (l/sin(theta) - chi E sin(theta))^2).
void invariants(const OrcParams& p, double E, double L, const double y[6], double* resid,
                double* K) {
    const Phys<double> q = phys_of(p);
    const Metric<double> m = metric(p, q, y[1], y[2]);
    const double pT = -E, pph = L, pR = y[4], pth = y[5];
    const double terms[5] = {m.u_TT * pT * pT, 2.0 * m.u_Tph * pT * pph, m.u_phph * pph * pph,
                             m.u_RR * pR * pR, m.u_thth * pth * pth};
    double sum = 0.0, mag = 0.0;
    for (double t : terms) { sum += t; mag += std::fabs(t); }
    *resid = std::fabs(sum) / mag;
    const double s = std::sin(y[2]);
    const double W = L / s - p.spin * E * s;
    *K = pth * pth + W * W;
}

struct ImageSetup {
    double r_plus, r_stop, r_esc, r_in;
};

bool image_setup(const OrcParams& p, ImageSetup* s) {
    if (!outer_horizon(p, &s->r_plus)) return false;
    s->r_stop = p.r_stop_fac * s->r_plus;
    s->r_esc = p.r_esc_fac * p.r_obs;
    s->r_in = p.r_in > 0.0 ? p.r_in : s->r_plus;
    return true;
}

// Log of the attempts of one ray: step size and whether it was accepted.
struct AttemptLog {
    std::vector<double> h;
    std::vector<uint8_t> accepted;
};

// What a traced ray returns in scalar type T.
template <class T>
struct RayT {
    T E, L;
    T r_em[3], phi_em[3], t_em[3], g_em[3], i_n[3];
    T intensity;
};

// ----------------------------------------------------- one backward ray
// Traces the ray of screen point (X, Y).  With record != null every attempt's
// step size and decision are appended to it; with replay != null the attempts
// are replayed from it instead of being chosen by the controller (the frozen
// discrete map).  If `log` is non-null, every accepted step appends
// (lambda, h, y[6]) -- 8 doubles -- up to log_cap rows.  For T = Dual the
// decisions come from the value parts, so they are those of the double run.
template <class T>
void trace_ray(const OrcParams& p, const Phys<T>& q, const ImageSetup& S, double X, double Y,
               OrcRay* out, RayT<T>* tout, double* log, int log_cap, int* n_log,
               AttemptLog* record, const AttemptLog* replay) {
    OrcRay r{};
    RayT<T> rt{};
    r.status = RUNNING;
    for (int n = 0; n < 3; ++n) {
        r.r_em[n] = r.phi_em[n] = r.t_em[n] = r.g_em[n] = r.i_n[n] = kNaN;
        rt.r_em[n] = rt.phi_em[n] = rt.t_em[n] = rt.g_em[n] = rt.i_n[n] = T(kNaN);
    }
    const Observer<T> obs = observer(p, q);
    const T r_in = p.r_in > 0.0 ? T(p.r_in) : horizon_of(p, q, S.r_plus);
    T p_up[4], p_dn[4];
    initial_momentum(obs, p.r_obs, X, Y, p_up, p_dn);
    const T E = -p_dn[0], L = p_dn[3];                    // eq. (48)
    const T obs_energy = -(p_dn[0] * obs.u[0] + p_dn[3] * obs.u[3]);  // = E_loc
    rt.E = E;
    rt.L = L;
    r.E = val(E);
    r.L = val(L);
    T y[6] = {T(0.0), T(p.r_obs), q.incl, T(0.0), p_dn[1], p_dn[2]};
    T k1[6];
    rhs(p, q, E, L, y, k1);
    double yv[6];
    for (int i = 0; i < 6; ++i) yv[i] = val(y[i]);
    double resid0, K0;
    invariants(p, r.E, r.L, yv, &resid0, &K0);
    r.max_constraint = resid0;
    r.carter_drift = 0.0;
    double h = p.h0, lambda = 0.0, last_cross = -std::numeric_limits<double>::infinity();
    bool after_reject = false;
    int nonfinite_run = 0;   // consecutive attempts with a non-finite error estimate
    int nl = 0;
    size_t ri = 0;
    Step<T> st;
    T intensity(0.0);
    for (;;) {
        if (replay) {
            if (ri >= replay->h.size()) { r.status = STEP_LIMIT; break; }
            h = replay->h[ri];
        } else if (r.attempts >= p.max_attempts) {
            r.status = STEP_LIMIT;
            break;
        }
        ++r.attempts;
        dp5_attempt(p, q, E, L, y, k1, h, &st);
        if (r.attempts >= g_fault_from && r.attempts <= g_fault_to) st.err = T(kNaN);
        const double err = val(st.err);
        bool accept = err < 1.0;
        if (replay) accept = replay->accepted[ri] != 0;
        if (record) {
            record->h.push_back(h);
            record->accepted.push_back(accept ? 1 : 0);
        }
        ++ri;
        if (!accept) {  // rejected (also when err is NaN)
            const bool finite = std::isfinite(err);
            const double f = finite ? std::fmax(0.2, 0.9 * std::pow(err, -0.2)) : 0.2;
            h *= f;
            after_reject = true;
            nonfinite_run = finite ? 0 : nonfinite_run + 1;
            if (nonfinite_run >= kNonfiniteRun && !replay) { r.status = NONFINITE; break; }
            continue;
        }
        nonfinite_run = 0;
        double factor = err == 0.0 ? 10.0 : std::fmin(10.0, 0.9 * std::pow(err, -0.2));
        if (after_reject) factor = std::fmin(1.0, factor);
        after_reject = false;
        ++r.accepted;

        // Equatorial crossing on this accepted step (Sec. 3.3, eq. (76)): the
        // band index of theta changes; the crossed equator is theta_eq.
        const double band0 = equator_band(val(y[2]));
        const double band1 = equator_band(val(st.y_new[2]));
        if (band0 != band1) {
            const double kk = std::fmax(band0, band1);
            const double th_eq = kHalfPi + kk * kPi;
            const bool above0 = band0 > band1;   // theta(0) >= theta_eq
            double a = 0.0, b = 1.0;  // theta(a) on the side of theta(0)
            for (int it = 0; it < 60; ++it) {
                const double mid = 0.5 * (a + b);
                const bool am = (val(dense(y, st, h, 2, mid)) - th_eq) >= 0.0;
                if (am == above0) a = mid; else b = mid;
            }
            const double s = 0.5 * (a + b);
            // root as a function of the parameters: theta(s*) = theta_eq fixes
            // ds* = -dtheta/theta_s (implicit-function theorem); its value is s
            const T sT = root_of(s, dense(y, st, h, 2, s) - th_eq, st, h);
            // theta_eq = -pi/2 (mod 2 pi) is the equator on the far side of the axis
            const double phi_shift = std::fmod(std::fabs(kk), 2.0) == 1.0 ? kPi : 0.0;
            const T Rc = dense(y, st, h, 1, sT);
            const double pth = val(dense(y, st, h, 5, s));
            const double thdot = pth / (val(Rc) * val(Rc));  // eq. (60), Sigma = R^2 on the equator
            const double lam_c = lambda + s * h;
            if (std::fabs(thdot) >= 1e-12 && (lam_c - last_cross) >= 1e-10) {
                const int n = r.ncross;
                if (n < 3) {
                    rt.r_em[n] = Rc;
                    rt.phi_em[n] = dense(y, st, h, 3, sT) + phi_shift;
                    rt.t_em[n] = dense(y, st, h, 0, sT);
                    const T g = redshift(p, q, Rc, E, L, obs_energy);
                    rt.g_em[n] = g;
                    rt.i_n[n] = window(p, Rc, r_in) * g * g * g * pow(Rc, -p.emis_pow);
                    intensity = intensity + rt.i_n[n];
                    r.r_em[n] = val(rt.r_em[n]);
                    r.phi_em[n] = val(rt.phi_em[n]);
                    r.t_em[n] = val(rt.t_em[n]);
                    r.g_em[n] = val(g);
                    r.i_n[n] = val(rt.i_n[n]);
                }
                if (r.ncross < 255) ++r.ncross;
                last_cross = lam_c;
            } else {
                ++r.filtered;
            }
        }

        for (int i = 0; i < 6; ++i) {
            y[i] = st.y_new[i];
            k1[i] = st.k[6][i];
            yv[i] = val(y[i]);
        }
        lambda += h;
        if (log && nl < log_cap) {
            double* row = log + 8 * nl;
            row[0] = lambda;
            row[1] = h;
            std::memcpy(row + 2, yv, sizeof yv);
            ++nl;
        }
        double resid, K;
        invariants(p, r.E, r.L, yv, &resid, &K);
        r.max_constraint = std::fmax(r.max_constraint, resid);
        r.carter_drift = std::fmax(r.carter_drift, std::fabs(K / K0 - 1.0));
        h *= factor;

        if (replay) continue;                                   // stops are part of the log
        if (yv[1] <= S.r_stop) { r.status = CAPTURED; break; }  // eq. (75)
        if (yv[1] >= S.r_esc) { r.status = ESCAPED; break; }
    }
    rt.intensity = intensity;
    r.intensity = val(intensity);
    r.lambda_end = lambda;
    std::memcpy(r.y_end, yv, sizeof yv);
    if (n_log) *n_log = nl;
    if (out) *out = r;
    if (tout) *tout = rt;
}

// ------------------------------------- Sec. 5.1-5.2: thick-disc emission
// Parameters of the volumetric emissivity eq. (84) beyond those of the image:
// the radial scale R_s and the height H(rho) = H_0 + h rho (eq. (85)).
struct ThickParams {
    double r_scale, h0, h_slope;
};

// j(R, theta) of eq. (84) with j_0 = 1: rho = R sin(theta), z = R cos(theta),
// the tanh tapers of eqs. (85)-(86) (hard edges R_in <= rho <= R_out when a
// width is not positive).
double thick_emissivity(const OrcParams& p, const ThickParams& t, double r_in, double R, double th) {
    const double rho = R * std::sin(th), z = R * std::cos(th);
    if (!(rho > 0.0)) return 0.0;
    double w;
    if (p.sigma_in > 0.0 && p.sigma_out > 0.0)
        w = 0.5 * (1.0 + std::tanh((rho - r_in) / p.sigma_in)) *
            (0.5 * (1.0 - std::tanh((rho - p.r_out) / p.sigma_out)));
    else
        w = (rho >= r_in && rho <= p.r_out) ? 1.0 : 0.0;
    if (w == 0.0) return 0.0;
    const double H = t.h0 + t.h_slope * rho;
    return std::pow(rho / r_in, -p.emis_pow) * std::exp(-(rho - r_in) / t.r_scale) *
           std::exp(-z * z / (2.0 * H * H)) * w;
}

// Redshift of eq. (89) for an emitter at (R, theta) moving with the circular
// equatorial angular velocity of eq. (91) at the same R, u^T from u.u = -1
// with the metric at (R, theta); 0 where that has no solution.
double thick_redshift(const OrcParams& p, const Phys<double>& q, double R, double th, double E,
                      double L, double obs_energy) {
    const Radial<double> r = radial(p, q, R);
    const double chi = q.chi, chi2 = chi * chi;
    const double dFoR2 = r.dF / (R * R) - 2.0 * r.F / (R * R * R);
    const double dgTT = dFoR2, dgTph = -chi * dFoR2, dgphph = 2.0 * R + chi2 * dFoR2;
    const double disc = dgTph * dgTph - dgTT * dgphph;
    if (!(disc >= 0.0)) return 0.0;
    const double Om = (-dgTph + std::sqrt(disc)) / dgphph;
    const Metric<double> m = metric(p, q, R, th);
    const double A = -(m.g_TT + 2.0 * Om * m.g_Tph + Om * Om * m.g_phph);
    if (!(A > 0.0)) return 0.0;
    const double em_energy = (E - Om * L) / std::sqrt(A);
    if (!(em_energy > 0.0)) return 0.0;
    return obs_energy / em_energy;
}

// dI/dlambda = g^3 j at state y (eq. (88)).
double thick_source(const OrcParams& p, const Phys<double>& q, const ThickParams& t, double r_in,
                    double E, double L, double obs_energy, const double y[6]) {
    const double j = thick_emissivity(p, t, r_in, y[1], y[2]);
    if (j == 0.0) return 0.0;
    const double g = thick_redshift(p, q, y[1], y[2], E, L, obs_energy);
    return g * g * g * j;
}

// One ray of the thick disc: the Dormand-Prince 5(4) integration of the
// geodesic with the intensity I as a seventh component (dI/dlambda = g^3 j,
// which does not feed back), the RMS error norm taken over all seven
// components; otherwise the controller and stops of trace_ray.
void trace_ray_thick(const OrcParams& p, const ThickParams& t, const ImageSetup& S, double X,
                     double Y, int32_t* status, int32_t* attempts, double* intensity) {
    const Phys<double> q = phys_of(p);
    const Observer<double> obs = observer(p, q);
    double p_up[4], p_dn[4];
    initial_momentum(obs, p.r_obs, X, Y, p_up, p_dn);
    const double E = -p_dn[0], L = p_dn[3];
    const double obs_energy = -(p_dn[0] * obs.u[0] + p_dn[3] * obs.u[3]);
    const double r_in = S.r_in;
    double y[7] = {0.0, p.r_obs, q.incl, 0.0, p_dn[1], p_dn[2], 0.0};
    auto f = [&](const double* yy, double* d) {
        rhs(p, q, E, L, yy, d);
        d[6] = thick_source(p, q, t, r_in, E, L, obs_energy, yy);
    };
    double k[7][7];
    f(y, k[0]);
    double h = p.h0;
    bool after_reject = false;
    int nonfinite_run = 0;
    int32_t att = 0, st = RUNNING;
    const double A[6][5] = {{0, 0, 0, 0, 0}, {A21, 0, 0, 0, 0}, {A31, A32, 0, 0, 0},
                            {A41, A42, A43, 0, 0}, {A51, A52, A53, A54, 0},
                            {A61, A62, A63, A64, A65}};
    const double Bw[7] = {B1, 0.0, B3, B4, B5, B6, 0.0};
    const double Ew[7] = {B1 - BH1, 0.0, B3 - BH3, B4 - BH4, B5 - BH5, B6 - BH6, 0.0 - BH7};
    for (;;) {
        if (att >= p.max_attempts) { st = STEP_LIMIT; break; }
        ++att;
        double tmp[7], yn[7];
        for (int j = 1; j < 6; ++j) {
            for (int i = 0; i < 7; ++i) {
                double sum = 0.0;
                for (int l = 0; l < j; ++l) sum += A[j][l] * k[l][i];
                tmp[i] = y[i] + h * sum;
            }
            f(tmp, k[j]);
        }
        for (int i = 0; i < 7; ++i) {
            double sum = 0.0;
            for (int l = 0; l < 7; ++l) sum += Bw[l] * k[l][i];
            yn[i] = y[i] + h * sum;
        }
        f(yn, k[6]);
        double acc = 0.0;
        for (int i = 0; i < 7; ++i) {
            double e = 0.0;
            for (int l = 0; l < 7; ++l) e += Ew[l] * k[l][i];
            const double sc = p.atol + p.rtol * std::fmax(std::fabs(y[i]), std::fabs(yn[i]));
            const double qq = h * e / sc;
            acc += qq * qq;
        }
        double err = std::sqrt(acc / 7.0);
        if (att >= g_fault_from && att <= g_fault_to) err = kNaN;
        if (!(err < 1.0)) {
            const bool finite = std::isfinite(err);
            h *= finite ? std::fmax(0.2, 0.9 * std::pow(err, -0.2)) : 0.2;
            after_reject = true;
            nonfinite_run = finite ? 0 : nonfinite_run + 1;
            if (nonfinite_run >= kNonfiniteRun) { st = NONFINITE; break; }
            continue;
        }
        nonfinite_run = 0;
        double factor = err == 0.0 ? 10.0 : std::fmin(10.0, 0.9 * std::pow(err, -0.2));
        if (after_reject) factor = std::fmin(1.0, factor);
        after_reject = false;
        for (int i = 0; i < 7; ++i) {
            y[i] = yn[i];
            k[0][i] = k[6][i];
        }
        h *= factor;
        if (y[1] <= S.r_stop) { st = CAPTURED; break; }
        if (y[1] >= S.r_esc) { st = ESCAPED; break; }
    }
    *status = st;
    *attempts = att;
    *intensity = y[6];
}

void pixel_centre(const OrcParams& p, int64_t idx, double* X, double* Y) {
    const int64_t ix = idx % p.nx, iy = idx / p.nx;
    *X = p.x_min + (static_cast<double>(ix) + 0.5) * ((p.x_max - p.x_min) / p.nx);
    *Y = p.y_min + (static_cast<double>(iy) + 0.5) * ((p.y_max - p.y_min) / p.ny);
}

}  // namespace

// =================================================================== C ABI
extern "C" {

// Radial functions: out = {H, dH/dR, mu, dmu/dR, F, dF/dR}.
void orc_radial(const OrcParams* p, double R, double* out) {
    const Radial<double> r = radial(*p, phys_of(*p), R);
    out[0] = r.H; out[1] = r.dH; out[2] = r.mu; out[3] = r.dmu; out[4] = r.F; out[5] = r.dF;
}

// Metric at (R, theta): out = {F, dF, Delta, dDelta, Sigma,
//  g_TT, g_Tphi, g_RR, g_thth, g_phph, g^TT, g^Tphi, g^RR, g^thth, g^phph,
//  d_R g^.. (5), d_theta g^.. (5)}  -- 25 doubles.
void orc_metric(const OrcParams* p, double R, double th, double* out) {
    const Metric<double> m = metric(*p, phys_of(*p), R, th);
    const double v[25] = {m.F, m.dF, m.Delta, m.dDelta, m.Sigma,
                          m.g_TT, m.g_Tph, m.g_RR, m.g_thth, m.g_phph,
                          m.u_TT, m.u_Tph, m.u_RR, m.u_thth, m.u_phph,
                          m.dR_TT, m.dR_Tph, m.dR_RR, m.dR_thth, m.dR_phph,
                          m.dt_TT, m.dt_Tph, m.dt_RR, m.dt_thth, m.dt_phph};
    std::memcpy(out, v, sizeof v);
}

double orc_two_hamiltonian(const OrcParams* p, double E, double L, const double* y) {
    return two_hamiltonian(metric(*p, phys_of(*p), y[1], y[2]), E, L, y[4], y[5]);
}

void orc_rhs(const OrcParams* p, double E, double L, const double* y, double* dy) {
    rhs(*p, phys_of(*p), E, L, y, dy);
}

int orc_horizon(const OrcParams* p, double* r_plus) { return outer_horizon(*p, r_plus) ? 0 : -2; }

int orc_extremal_spin(const OrcParams* p, double* chi_e, double* r_e) {
    return extremal_spin(*p, chi_e, r_e) ? 0 : -2;
}

// Observer: out = {omega, N, u^mu (4), e_R^mu (4), e_th^mu (4), e_ph^mu (4),
//                  g_TT, g_Tphi, g_RR, g_thth, g_phph}  -- 23 doubles.
void orc_observer(const OrcParams* p, double* out) {
    const Observer<double> o = observer(*p, phys_of(*p));
    double* q = out;
    *q++ = o.omega; *q++ = o.N;
    for (int i = 0; i < 4; ++i) *q++ = o.u[i];
    for (int i = 0; i < 4; ++i) *q++ = o.eR[i];
    for (int i = 0; i < 4; ++i) *q++ = o.eth[i];
    for (int i = 0; i < 4; ++i) *q++ = o.eph[i];
    *q++ = o.m.g_TT; *q++ = o.m.g_Tph; *q++ = o.m.g_RR; *q++ = o.m.g_thth; *q++ = o.m.g_phph;
}

void orc_initial_momentum(const OrcParams* p, double X, double Y, double* p_up, double* p_dn) {
    const Observer<double> o = observer(*p, phys_of(*p));
    initial_momentum(o, p->r_obs, X, Y, p_up, p_dn);
}

double orc_redshift(const OrcParams* p, double R, double E, double L) {
    return redshift(*p, phys_of(*p), R, E, L, 1.0);
}

// One ray at screen point (X, Y).  Returns 0, or -2 when there is no horizon.
int orc_trace_ray(const OrcParams* p, double X, double Y, OrcRay* out, double* log, int log_cap,
                  int* n_log) {
    ImageSetup S;
    if (!image_setup(*p, &S)) return -2;
    trace_ray<double>(*p, phys_of(*p), S, X, Y, out, nullptr, log, log_cap, n_log, nullptr,
                      nullptr);
    return 0;
}

// Rays of the pixels idx[0..n) (row-major, iy = idx / nx).  Each output array
// is indexed by k in [0, n) (compact), and any pointer may be null:
//   ncross, status, attempts: int32[n];  r_em, phi_em, t_em, g_em, i_n:
//   double[3*n] as [3][n];  intensity: double[n].
int orc_trace_pixels(const OrcParams* p, const int64_t* idx, int64_t n, int32_t* ncross,
                     int32_t* status, int32_t* attempts, double* r_em, double* phi_em,
                     double* t_em, double* g_em, double* i_n, double* intensity) {
    ImageSetup S;
    if (!image_setup(*p, &S)) return -2;
    const Phys<double> q = phys_of(*p);
    for (int64_t k = 0; k < n; ++k) {
        double X, Y;
        pixel_centre(*p, idx[k], &X, &Y);
        OrcRay r;
        trace_ray<double>(*p, q, S, X, Y, &r, nullptr, nullptr, 0, nullptr, nullptr, nullptr);
        if (ncross) ncross[k] = r.ncross;
        if (status) status[k] = r.status;
        if (attempts) attempts[k] = r.attempts;
        for (int j = 0; j < 3; ++j) {
            if (r_em) r_em[j * n + k] = r.r_em[j];
            if (phi_em) phi_em[j * n + k] = r.phi_em[j];
            if (t_em) t_em[j * n + k] = r.t_em[j];
            if (g_em) g_em[j * n + k] = r.g_em[j];
            if (i_n) i_n[j * n + k] = r.i_n[j];
        }
        if (intensity) intensity[k] = r.intensity;
    }
    return 0;
}

// Intensity and its gradient along (chi, theta_o, halo0, halo1) for the
// pixels idx[0..n): intensity[k] and grad[4 k + j] = dI/dq_j of the frozen
// discrete map (forward-mode dual numbers).
int orc_trace_grad_pixels(const OrcParams* p, const int64_t* idx, int64_t n, double* intensity,
                          double* grad) {
    ImageSetup S;
    if (!image_setup(*p, &S)) return -2;
    const Phys<Dual<4>> q = phys_seeded(*p);
    for (int64_t k = 0; k < n; ++k) {
        double X, Y;
        pixel_centre(*p, idx[k], &X, &Y);
        RayT<Dual<4>> r;
        trace_ray<Dual<4>>(*p, q, S, X, Y, nullptr, &r, nullptr, 0, nullptr, nullptr, nullptr);
        if (intensity) intensity[k] = r.intensity.v;
        for (int j = 0; j < 4; ++j) grad[4 * k + j] = r.intensity.d[j];
    }
    return 0;
}

// The frozen discrete map at perturbed parameters: the attempt sequence
// (step sizes and decisions) of each pixel's ray is recorded at the
// parameters `base`, then replayed at `pert` (same screen); intensity[k] is
// the replayed intensity.  Used for frozen-step finite differences.
int orc_replay_pixels(const OrcParams* base, const OrcParams* pert, const int64_t* idx, int64_t n,
                      double* intensity) {
    ImageSetup S0, S1;
    if (!image_setup(*base, &S0) || !image_setup(*pert, &S1)) return -2;
    for (int64_t k = 0; k < n; ++k) {
        double X, Y;
        pixel_centre(*base, idx[k], &X, &Y);
        AttemptLog log;
        trace_ray<double>(*base, phys_of(*base), S0, X, Y, nullptr, nullptr, nullptr, 0, nullptr,
                          &log, nullptr);
        RayT<double> r;
        trace_ray<double>(*pert, phys_of(*pert), S1, X, Y, nullptr, &r, nullptr, 0, nullptr,
                          nullptr, &log);
        intensity[k] = r.intensity;
    }
    return 0;
}

// Image setup summary: out = {R_+, r_stop, r_esc, r_in}.
// Thick-disc intensity of the pixels idx[0..n) (Sec. 5.1-5.2); thick =
// {R_s, H_0, h}.  Any output pointer may be null.
int orc_trace_thick_pixels(const OrcParams* p, const double* thick, const int64_t* idx, int64_t n,
                           int32_t* status, int32_t* attempts, double* intensity) {
    ImageSetup S;
    if (!image_setup(*p, &S)) return -2;
    const ThickParams t{thick[0], thick[1], thick[2]};
    for (int64_t k = 0; k < n; ++k) {
        double X, Y;
        pixel_centre(*p, idx[k], &X, &Y);
        int32_t st, att;
        double I;
        trace_ray_thick(*p, t, S, X, Y, &st, &att, &I);
        if (status) status[k] = st;
        if (attempts) attempts[k] = att;
        if (intensity) intensity[k] = I;
    }
    return 0;
}

int orc_image_setup(const OrcParams* p, double* out) {
    ImageSetup S;
    if (!image_setup(*p, &S)) return -2;
    out[0] = S.r_plus; out[1] = S.r_stop; out[2] = S.r_esc; out[3] = S.r_in;
    return 0;
}

// Fault injection (tests of the failure handling): attempts from..to of
// every later ray get a non-finite error estimate; from > to switches it off.
void orc_set_fault(int from, int to) {
    g_fault_from = from;
    g_fault_to = to;
}

int orc_sizeof_params(void) { return static_cast<int>(sizeof(OrcParams)); }
int orc_sizeof_ray(void) { return static_cast<int>(sizeof(OrcRay)); }

}  // extern "C"
