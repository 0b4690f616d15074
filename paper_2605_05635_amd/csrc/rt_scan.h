// rt_scan.h -- roots and extrema of the radial metric function (Sec. 2):
// the outer horizon as the largest root of Delta(R) = R^2 - F(R) + chi^2
// (eq. (33)), the ergosurface as the largest root with chi^2 cos^2(theta) in
// place of chi^2 (g_TT = 0), and the extremal spin chi_e^2 = max_R (F(R) -
// R^2), beyond which Delta has no root.  Host and device (the image set-up
// and the parameter-scan kernel use the same code).
#pragma once

#include "rt_device.h"

namespace rt {
namespace scan {

// R^2 - F(R) + a2 and its R-derivative.
__host__ __device__ inline void delta(const ImageConst& c, double a2, double R, double* D,
                                      double* dD) {
    double F, dF;
    mass_function_any(c, R, F, dF);
    *D = R * R - F + a2;
    *dD = 2.0 * R - dF;
}

// The largest root of R^2 - F(R) + a2 in (0.05, 50]: the function is sampled
// downward on a grid of spacing 1e-2; an interval counts when it changes sign
// across it, or when it has an interior minimum <= 0 (two close roots, near
// extremality).  The root is refined by bisection to the last representable
// bracket.  False when there is none.
__host__ __device__ inline bool largest_root(const ImageConst& c, double a2, double* root) {
    const double top = 50.0, step = 1e-2;
    double D_hi, dD_hi;
    delta(c, a2, top, &D_hi, &dD_hi);
    if (!(D_hi > 0.0)) return false;
    for (int k = 1; top - k * step >= 0.05 - 1e-12; ++k) {
        const double hi = top - (k - 1) * step, lo = top - k * step;
        double D_lo, dD_lo;
        delta(c, a2, lo, &D_lo, &dD_lo);
        double a = lo, b = hi;  // want D(a) <= 0 < D(b)
        bool bracket = D_lo <= 0.0;
        if (!bracket && dD_lo < 0.0 && dD_hi > 0.0) {
            // interior minimum: locate it where the derivative vanishes
            double u = lo, v = hi;
            for (int it = 0; it < 200; ++it) {
                const double m = 0.5 * (u + v);
                if (m <= u || m >= v) break;
                double Dm, dDm;
                delta(c, a2, m, &Dm, &dDm);
                if (dDm < 0.0) u = m; else v = m;
            }
            double Dm, dDm;
            delta(c, a2, 0.5 * (u + v), &Dm, &dDm);
            if (Dm <= 0.0) {
                a = 0.5 * (u + v);
                bracket = true;
            }
        }
        if (bracket) {
            for (int it = 0; it < 200; ++it) {
                const double m = 0.5 * (a + b);
                if (m <= a || m >= b) break;
                double Dm, dDm;
                delta(c, a2, m, &Dm, &dDm);
                if (Dm > 0.0) b = m; else a = m;
            }
            *root = 0.5 * (a + b);
            return true;
        }
        D_hi = D_lo;
        dD_hi = dD_lo;
    }
    return false;
}

// Extremal spin: chi_e^2 = -min_R (R^2 - F(R)) over the local minima of R^2 - F
// on (0.01, 50] (where 2R - F'(R) turns from negative to non-negative across a
// grid interval of 1e-3, refined by bisection), r_e the minimising radius.
// False when R^2 - F stays positive (no horizon for any spin).
__host__ __device__ inline bool extremal_spin(const ImageConst& c, double* chi_e, double* r_e) {
    const double step = 1e-3;
    double best = 0.0, best_r = 0.0;
    bool found = false;
    double a = 0.01, Va, Da;
    delta(c, 0.0, a, &Va, &Da);
    for (int k = 1; a < 50.0; ++k) {
        const double b = 0.01 + static_cast<double>(k) * step;
        double Vb, Db;
        delta(c, 0.0, b, &Vb, &Db);
        if (Da < 0.0 && Db >= 0.0) {
            double lo = a, hi = b;
            for (int it = 0; it < 200; ++it) {
                const double m = 0.5 * (lo + hi);
                if (m <= lo || m >= hi) break;
                double Vm, Dm;
                delta(c, 0.0, m, &Vm, &Dm);
                if (Dm < 0.0) lo = m; else hi = m;
            }
            const double rm = 0.5 * (lo + hi);
            double Vm, Dm;
            delta(c, 0.0, rm, &Vm, &Dm);
            if (Vm < best) {
                best = Vm;
                best_r = rm;
                found = true;
            }
        }
        a = b;
        Da = Db;
    }
    if (!found) return false;
    *chi_e = sqrt(-best);
    *r_e = best_r;
    return true;
}

}  // namespace scan
}  // namespace rt
