"""Coefficients of the polynomial kernels of rt_math.h.

Each kernel approximates a smooth auxiliary function on the reduced interval
its caller guarantees, by Chebyshev interpolation (mpmath.chebyfit, within a
small factor of the best uniform approximation of that degree) in 60-digit
arithmetic, the coefficients then rounded to binary64.  The printed bound is
the largest relative error of the resulting function value (before the
rounding of its binary64 evaluation), measured on a 4000-point grid:

    sin r = r + r z S(z),            z = r^2 in [0, (pi/2)^2]  (binary32: [0, (pi/4)^2])
    cos r = 1 + z C(z)               (its bound is absolute: cos r reaches 0)
    e^r - 1 = r + r^2 E(r),          |r| <= ln(2)/2 (+1e-9)
    e^x - 1 = x + x^2 EN(x),         x in [-0.34, 0] (+-1e-9; the cored-NFW exponent)
    log m = w (1 + v LW(v)),         w = 2 (m-1)/(m+1), m in [sqrt(1/2), sqrt(2)), v = w^2
    (binary32: log m = 2 (t + t z L(z)), t = w/2, z = t^2)

Run `python poly_coeffs.py` to print the tables in the order rt_math.h
evaluates them (highest degree first): the binary64 kernels, then the
lower-degree binary32 kernels of the single-precision bulk trace (coefficients
rounded to binary32).
"""
import mpmath as mp

mp.mp.dps = 60
PIO4_2 = (mp.pi / 4) ** 2 * (1 + mp.mpf("1e-12"))
PIO2_2 = (mp.pi / 2) ** 2 * (1 + mp.mpf("1e-12"))
LN2_2 = mp.log(2) / 2 + mp.mpf("1e-9")
T_MAX = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)
Z_LOG = T_MAX ** 2 * (1 + mp.mpf("1e-12"))
EX_NEAR = mp.mpf("0.34")


def _S(z):
    r = mp.sqrt(z)
    return (mp.sin(r) - r) / (r * z)


def _C(z):
    return (mp.cos(mp.sqrt(z)) - 1) / z


def _E(r):
    return mp.mpf(0.5) if r == 0 else (mp.expm1(r) - r) / (r * r)


def _L(z):
    t = mp.sqrt(z)
    return (mp.atanh(t) / t - 1) / z


def _LW(v):
    w = mp.sqrt(v)
    return (2 * mp.atanh(w / 2) / w - 1) / v


KERNELS = {   # name: (auxiliary function, interval, degree, value of the kernel's function)
    "S": (_S, (0, PIO2_2), 7, lambda x, p: (mp.sqrt(x) * (1 + x * p), mp.sin(mp.sqrt(x)))),
    "C": (_C, (0, PIO2_2), 7, lambda x, p: (1 + x * p, mp.cos(mp.sqrt(x)))),
    "E": (_E, (-LN2_2, LN2_2), 10, lambda x, p: (x + x * x * p, mp.expm1(x))),
    "EN": (_E, (-EX_NEAR - mp.mpf("1e-9"), mp.mpf("1e-9")), 8,
           lambda x, p: (x + x * x * p, mp.expm1(x))),
    "L": (_L, (0, Z_LOG), 6, lambda x, p: (2 * mp.sqrt(x) * (1 + x * p), 2 * mp.atanh(mp.sqrt(x)))),
    "LW": (_LW, (0, 4 * Z_LOG), 6,
           lambda x, p: (mp.sqrt(x) * (1 + x * p), 2 * mp.atanh(mp.sqrt(x) / 2))),
}
# The kernels of the binary64 functions (rt_math.h); L is binary32 only.
USED64 = ("S", "C", "E", "EN", "LW")
# Kernels whose bound is the absolute error of the function value.
ABSOLUTE = {"C"}

# Degrees of the binary32 kernels (the single-precision bulk trace, whose sine
# and cosine reduce by pi/2); their coefficients are rounded to binary32.
DEGREES32 = {"S": 3, "C": 3, "E": 5, "L": 2}
INTERVALS32 = {"S": (0, PIO4_2), "C": (0, PIO4_2)}


def interval(name, binary32=False):
    if binary32 and name in INTERVALS32:
        return INTERVALS32[name]
    return KERNELS[name][1]


def coefficients(name, binary32=False):
    f, _, deg, _ = KERNELS[name]
    a, b = interval(name, binary32)
    if binary32:
        deg = DEGREES32[name]
    cs = mp.chebyfit(f, [a, b], deg + 1)
    if binary32:
        import numpy as np
        return [float(np.float32(c)) for c in cs]
    return [float(c) for c in cs]


def max_rel_error(name, cs, n=4000, binary32=False):
    """The largest relative error (absolute for the kernels in ABSOLUTE)."""
    f, _, _, value = KERNELS[name]
    a, b = interval(name, binary32)
    worst = mp.mpf(0)
    for i in range(1, n):
        x = a + (b - a) * mp.mpf(i) / n
        if x == 0:
            continue
        p = mp.mpf(cs[0])
        for c in cs[1:]:
            p = p * x + mp.mpf(c)
        got, exact = value(x, p)
        worst = max(worst, abs(got - exact) if name in ABSOLUTE else abs((got - exact) / exact))
    return float(worst)


if __name__ == "__main__":
    for binary32 in (False, True):
        for name in (DEGREES32 if binary32 else USED64):
            cs = coefficients(name, binary32)
            kind = "binary32" if binary32 else "binary64"
            what = "abs" if name in ABSOLUTE else "rel"
            print(f"// {name} ({kind}): degree {len(cs) - 1}, "
                  f"max {what} err {max_rel_error(name, cs, binary32=binary32):.2e}")
            print("    " + ",\n    ".join(repr(c) + ("f" if binary32 else "") for c in cs))
