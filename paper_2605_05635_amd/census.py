"""Algorithmic operation census of the trace (for roofline accounting).

Counts the floating-point operations one right-hand-side evaluation, one
Dormand-Prince step attempt, the location of one crossing (trace kernel) and
the emission of one recorded crossing (emission pass) must perform, by
executing the kernels' formulas once with a counting scalar.
Convention: every +, -, *, / , sqrt, fabs/fmax/fmin and every special-function
value (sin, cos, exp, expm1, log1p, pow, tanh) counts as one flop; common
subexpressions are counted once, as the kernel computes them; comparisons and
integer bookkeeping are not counted.

Used only to turn measured per-ray step counts into FLOP/s; it computes nothing
the trace returns.  tests/test_census.py checks that the formulas below give
the same numbers as the oracle's right-hand side, so the census counts a
correct evaluation.
"""
from __future__ import annotations

import math


class Num:
    """A float that counts the arithmetic done on it."""
    ops = 0

    def __init__(self, v):
        self.v = float(v.v if isinstance(v, Num) else v)

    @staticmethod
    def _v(x):
        return x.v if isinstance(x, Num) else float(x)

    def _op(self, r):
        Num.ops += 1
        return Num(r)

    def __add__(self, o): return self._op(self.v + self._v(o))
    def __radd__(self, o): return self._op(self._v(o) + self.v)
    def __sub__(self, o): return self._op(self.v - self._v(o))
    def __rsub__(self, o): return self._op(self._v(o) - self.v)
    def __mul__(self, o): return self._op(self.v * self._v(o))
    def __rmul__(self, o): return self._op(self._v(o) * self.v)
    def __truediv__(self, o): return self._op(self.v / self._v(o))
    def __rtruediv__(self, o): return self._op(self._v(o) / self.v)
    def __neg__(self): return Num(-self.v)      # sign flips are free
    def __float__(self): return self.v


def f(name, *x):
    Num.ops += 1
    return Num(getattr(math, name)(*(Num._v(a) for a in x)))


def mass_function(metric: str, c: dict, R):
    if metric == "kerr":
        return 2.0 * R, Num(2.0)
    if metric == "einasto":
        x = R * c["inv_lam"]
        e = f("exp", -x)
        mu = 1.0 - e * (1.0 + x * (1.0 + 0.5 * x))
        dmu = 0.5 * e * x * x * c["inv_lam"]
        return 2.0 * R * mu, 2.0 * (mu + R * dmu)
    iR = 1.0 / R
    iRl = 1.0 / (R + c["lam_c"])
    lg = f("log1p", R * c["inv_lam_c"])
    ex = c["eta_lc"] * (iRl - 2.0 * iR * lg)
    dex = c["eta_lc"] * (2.0 * iR * (iR * lg - iRl) - iRl * iRl)
    em1 = f("expm1", ex)
    F = R * (2.0 - R * em1)
    dF = 2.0 - R * (2.0 * em1 + R * (em1 + 1.0) * dex)
    return F, dF


def rhs(metric: str, c: dict, E, L, R, th, pR, pth):
    s, co = f("sin", th), f("cos", th)
    F, dF = mass_function(metric, c, R)
    chi, chi2 = c["chi"], c["chi2"]
    R2 = R * R
    R2c = R2 + chi2
    Sig = R2 + chi2 * co * co
    Del = R2c - F
    dDel = 2.0 * R - dF
    iS, iD, is_ = 1.0 / Sig, 1.0 / Del, 1.0 / s
    P = R2c * E - chi * L
    PiD = P * iD
    Lis2 = L * is_ * is_
    chiE = chi * E
    W = L * is_ - chiE * s
    pR2 = pR * pR
    N = Del * pR2 + pth * pth - P * PiD + W * W
    dN = dDel * (pR2 + PiD * PiD) - 4.0 * R * E * PiD
    return [(PiD * R2c + chi * (L - chiE * s * s)) * iS,
            Del * pR * iS,
            pth * iS,
            (chi * PiD + Lis2 - chiE) * iS,
            (N * R * iS - 0.5 * dN) * iS,
            co * iS * (W * (Lis2 + chiE) - chi2 * s * N * iS)]


def _consts(metric, chi=0.5, halo=(0.1, 10.0)):
    return dict(chi=chi, chi2=chi * chi, inv_lam=1.0 / halo[0], lam_c=halo[1], inv_lam_c=1.0 / halo[1],
                eta_lc=halo[0] * halo[1])


def flops_rhs(metric: str) -> int:
    Num.ops = 0
    c = _consts(metric)
    rhs(metric, c, Num(1.0), Num(2.0), Num(7.0), Num(1.1), Num(0.3), Num(2.0))
    return Num.ops


def flops_step_overhead() -> int:
    """Everything in one attempt except the six right-hand sides: stage inputs
    of the four dynamical components (T and phi do not feed back), the 5th-order
    update, the RMS error norm and the step-size factor."""
    n = 0
    for j in range(2, 7):        # stages 2..6: y + h * sum_{i<j} a_ji k_i
        n += 4 * (2 * j - 1)
    n += 6 * 11                  # y_new = y + h * (5 weighted k's)
    n += 6 * (12 + 5 + 3)        # error term, scale atol + rtol max(|y|,|y_new|), q^2 sum
    n += 2 + 4                   # sqrt(mean), pow, safety, min/max
    return n


def flops_step_overhead32() -> int:
    """The binary32 attempt of the mixed-precision bulk: as
    flops_step_overhead, with each of the six state updates y + h sum b_i k_i
    done as an error-free (two-sum) addition into the compensated pair hi + lo
    (10 operations in place of the one addition)."""
    return flops_step_overhead() + 6 * 9


def flops_crossing(newton: int = 3) -> int:
    """Locating one crossing (trace kernel): dense coefficients for theta, R,
    p_theta, phi and T; the safeguarded Newton iteration on theta(s) (`newton`
    iterations: from the secant start it takes three on average, measured on
    the cored-NFW benchmark screen, at most four); the evaluations at the root
    and the trusted-crossing test."""
    dense_coeffs = 5 * (3 + 12 + 1)      # r2, r3, r4 and r5 = h sum d_i k_i
    start = 5 + 2                         # quartic coefficients, secant root
    per_iter = 9 + 9 + 2 + 2              # theta(s) - pi/2, derivative, update, bracket
    per_eval = 9                          # y0 + s (r2 + (1-s)(r3 + s (r4 + (1-s) r5)))
    at_root = 4 * per_eval + 2 + 4        # R, p_theta, phi, T; affine position; filter
    return dense_coeffs + start + newton * per_iter + at_root


def flops_emission(metric: str) -> int:
    """The emission of one recorded crossing (emission pass): the Keplerian
    redshift, the disc window and g^3 R^-p, added to the pixel's sum."""
    Num.ops = 0
    c = _consts(metric)
    R = Num(7.0)
    F, dF = mass_function(metric, c, R)
    iR = 1.0 / R
    FoR2 = F * iR * iR
    G = (dF - 2.0 * F * iR) * iR * iR
    disc = -2.0 * R * G
    Om = (c["chi"] * G + f("sqrt", disc)) / (2.0 * R + c["chi2"] * G)
    gTT, gTp = -(1.0 - FoR2), -c["chi"] * FoR2
    gpp = R * R + c["chi2"] + c["chi2"] * FoR2
    A = -(gTT + Om * (2.0 * gTp + Om * gpp))
    g = f("sqrt", A) / (1.0 - Om * 2.0)
    In = g * g * g * f("pow", R, -3.0)
    _ = In + 1.0
    return Num.ops


def flops_thick_source(metric: str) -> int:
    """One evaluation of the thick disc's source g^3 j at (R, theta) (Sec.
    5.1-5.2): sine and cosine, the emissivity of eq. (84) with tapers, the
    circular emitter's Omega (eq. (91)) at R and u^T from the metric at
    (R, theta), g^3 times j."""
    Num.ops = 0
    c = _consts(metric)
    R, th = Num(7.0), Num(1.4)
    s, co = f("sin", th), f("cos", th)
    rho, z = R * s, R * co
    w = (1.0 / (1.0 + f("exp", -2.0 * (rho - 2.0) / 0.5))) * (1.0 / (1.0 + f("exp", 2.0 * (rho - 20.0) / 0.5)))
    H = 0.2 + 0.1 * rho
    j = f("exp", -2.0 * f("log1p", rho / 2.0 - 1.0) - (rho - 2.0) / 8.0 - z * z / (2.0 * H * H)) * w
    F, dF = mass_function(metric, c, R)
    G = (dF - 2.0 * F / R) / (R * R)
    Om = (c["chi"] * G + f("sqrt", -2.0 * R * G)) / (2.0 * R + c["chi2"] * G)
    Sig = R * R + c["chi2"] * co * co
    s2 = s * s
    gTT = -(1.0 - F / Sig)
    gTp = -F * c["chi"] * s2 / Sig
    gpp = (R * R + c["chi2"] + F * c["chi2"] * s2 / Sig) * s2
    A = -(gTT + 2.0 * Om * gTp + Om * Om * gpp)
    g = f("sqrt", A) / (1.0 - Om * 2.0)
    _ = g * g * g * j
    return Num.ops


def flops_trace_ray(metric: str, attempts: float, crossings: float) -> float:
    """Algorithmic flops of the trace kernel for a ray with the given step
    attempts and trusted crossings (plus its start: screen map and one
    right-hand side)."""
    return (attempts * (6 * flops_rhs(metric) + flops_step_overhead())
            + crossings * flops_crossing() + 20 + flops_rhs(metric))


if __name__ == "__main__":
    for m in ("kerr", "einasto", "cnfw"):
        print(m, "rhs", flops_rhs(m), "step", flops_step_overhead(), "crossing",
              flops_crossing(), "emission", flops_emission(m), "thick source",
              flops_thick_source(m), "attempt",
              6 * flops_rhs(m) + flops_step_overhead())
