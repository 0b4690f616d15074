"""Accuracy of the trace kernels' compact elementary functions (rt_math.h),
compiled for the host from the same source, against mpmath at 40 digits.

Measured in units in the last place (ulp) of the exact result, over the
argument ranges the trace uses: theta in (-2 pi, 3 pi), exp of R/lambda_E
arguments down to underflow, expm1 of the cored-NFW exponent, log1p of
R/lambda_c, and the step controller's x^(-1/10)."""
import math
import os
import subprocess

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "devmath", "devmath_driver.cpp")
INC = os.path.join(ROOT, "paper_2605_05635_amd", "csrc")
mp.mp.dps = 40


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("devmath") / "devmath_driver")
    subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-I", INC, SRC, "-o", exe],
                   check=True, capture_output=True)
    return exe


def run(exe, fn, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = subprocess.run([exe, fn], input=x.tobytes(), capture_output=True, check=True).stdout
    return np.frombuffer(out, dtype=np.float64)


def ulp_err(got, exact):
    exact_f = np.array([float(e) for e in exact])
    ulp = np.spacing(np.abs(exact_f))
    ulp[ulp == 0] = np.spacing(0.0)
    d = np.array([float(abs(mp.mpf(g) - e)) for g, e in zip(got, exact)])
    return d / ulp


def test_sincos(driver):
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-2 * np.pi, 3 * np.pi, 3000),
                        np.pi / 2 * np.arange(-4, 7) + 1e-13, [0.0, 1e-300, 3.1e5]])
    out = run(driver, "sincos", x).reshape(-1, 2)
    es = [mp.sin(mp.mpf(v)) for v in x]
    ec = [mp.cos(mp.mpf(v)) for v in x]
    # absolute error relative to 1 (the magnitude of sin and cos)
    ds = np.array([float(abs(mp.mpf(g) - e)) for g, e in zip(out[:, 0], es)])
    dc = np.array([float(abs(mp.mpf(g) - e)) for g, e in zip(out[:, 1], ec)])
    assert ds.max() < 2.5e-16 and dc.max() < 2.5e-16
    # relative accuracy away from the zeros
    big = np.abs(np.array([float(e) for e in es])) > 1e-3
    assert ulp_err(out[big, 0], [e for e, b in zip(es, big) if b]).max() < 4


def test_sincos_near_multiples_of_pi(driver):
    # the doubles nearest k pi and their neighbours, |k| <= 16: sin must keep
    # its relative accuracy where it is tiny (pi is carried as two doubles)
    x = []
    for k in range(-16, 17):
        if k == 0:
            continue
        c = float(k * mp.pi)
        x += [np.nextafter(c, -np.inf), c, np.nextafter(c, np.inf)]
    x = np.array(x)
    out = run(driver, "sincos", x).reshape(-1, 2)
    es = [mp.sin(mp.mpf(v)) for v in x]
    assert ulp_err(out[:, 0], es).max() < 4


def test_exp(driver):
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-740, 700, 2000), rng.uniform(-1, 1, 1000),
                        [0.0, -744.0, -800.0, -1e5, 709.0]])
    out = run(driver, "exp", x)
    ex = [mp.exp(mp.mpf(v)) for v in x]
    normal = np.array([float(e) for e in ex]) > 2.3e-308
    assert ulp_err(out[normal], [e for e, n in zip(ex, normal) if n]).max() < 3
    assert out[x <= -800].max() == 0.0


def test_expm1(driver):
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(-0.6, 0.2, 3000), 10.0 ** rng.uniform(-20, -1, 500),
                        -(10.0 ** rng.uniform(-20, -1, 500)), -(10.0 ** rng.uniform(-1, 2.8, 500)),
                        10.0 ** rng.uniform(-1, 2.8, 500),
                        [0.0, 0.3465, -0.3466, 0.34657359027997264, -0.34657359027997264,
                         0.3465735902799727, 2.0, -700.0, 700.0]])
    out = run(driver, "expm1", x)
    ex = [mp.expm1(mp.mpf(v)) for v in x]
    nz = x != 0
    assert ulp_err(out[nz], [e for e, n in zip(ex, nz) if n]).max() < 4
    assert out[x == 0][0] == 0.0
    # the limit -1 far below zero
    assert np.all(run(driver, "expm1", np.array([-745.0, -800.0, -1e10])) == -1.0)


def test_expm1_near(driver):
    """The cored-NFW exponent's e^x - 1 on [-0.34, 0] (halos with
    0 <= eta <= 0.34), including the ends and tiny arguments."""
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.uniform(-0.34, 0.0, 3000), -(10.0 ** rng.uniform(-12, -0.5, 500)),
                        [-0.34, -1e-300, 0.0, -0.02, -1e-9]])
    out = run(driver, "expm1_near", x)
    ex = [mp.expm1(mp.mpf(v)) for v in x]
    assert ulp_err(out, ex).max() < 4


def test_log1p(driver):
    rng = np.random.default_rng(3)
    x = np.concatenate([10.0 ** rng.uniform(-3, 3.5, 3000), rng.uniform(-0.5, 0.5, 500),
                        [1e-17, 1.0, 3.0, 1e5]])
    out = run(driver, "log1p", x)
    ex = [mp.log1p(mp.mpf(v)) for v in x]
    assert ulp_err(out, ex).max() < 4


def test_log1p_fast(driver):
    """Without the correction for the rounding of 1 + u: the dropped term is at
    most half an ulp of 1 + u relative to 1 + u, i.e. 2^-53 absolute.  (The
    host build divides exactly; the device's one-step reciprocal adds 2.2e-15
    relative, measured on gfx950.)"""
    rng = np.random.default_rng(5)
    x = np.concatenate([10.0 ** rng.uniform(-3, 3.5, 3000), rng.uniform(-0.5, 0.5, 500),
                        [1e-17, 1.0, 3.0, 1e5]])
    out = run(driver, "log1p_fast", x)
    ex = [mp.log1p(mp.mpf(v)) for v in x]
    d = np.array([float(abs(mp.mpf(g) - e)) for g, e in zip(out, ex)])
    exf = np.abs(np.array([float(e) for e in ex]))
    assert np.all(d <= 2.0 ** -53 + 4 * np.spacing(exf))
    # relative to the result, the dropped term matters only where log1p(u) is
    # small; from u = 1 on it stays within a few ulp
    big = x >= 1.0
    assert ulp_err(out[big], [e for e, b in zip(ex, big) if b]).max() < 4


def test_cnfw_halo_terms(driver):
    """The cored-NFW mass function's 1/R, 1/(R + lambda_c) and
    log(1 + R/lambda_c) from one reciprocal and the integer split of
    1 + R/lambda_c (host build: exact division).  Bounds as log1p_fast's: the
    logarithm within half an ulp of 1 + R/lambda_c absolute plus a few ulp, the
    reciprocals within a few ulp; R over the traced range, lambda_c over the
    workloads' (including arguments right at the split's powers of two)."""
    rng = np.random.default_rng(6)
    R = np.concatenate([10.0 ** rng.uniform(-0.2, 3.1, 3000), [1.0, 1.5, 1100.0]])
    lc = np.concatenate([rng.uniform(2.0, 25.0, 3000), [10.0, 10.0, 10.0]])
    # 1 + R/lambda_c at and beside sqrt(2) 2^j and 2^j
    for j in range(0, 7):
        for m in (math.sqrt(2.0), 2.0):
            u = m * 2.0 ** j - 1.0
            for f in (1 - 1e-15, 1.0, 1 + 1e-15):
                R = np.append(R, 10.0 * u * f)
                lc = np.append(lc, 10.0)
    out = run(driver, "cnfw_terms", np.stack([R, lc], axis=1).ravel()).reshape(-1, 3)
    ex_iR = [1 / mp.mpf(r) for r in R]
    ex_iRl = [1 / (mp.mpf(r) + mp.mpf(l)) for r, l in zip(R, lc)]
    ex_lg = [mp.log1p(mp.mpf(r) / mp.mpf(l)) for r, l in zip(R, lc)]
    assert ulp_err(out[:, 0], ex_iR).max() < 4
    assert ulp_err(out[:, 1], ex_iRl).max() < 4
    d = np.array([float(abs(mp.mpf(g) - e)) for g, e in zip(out[:, 2], ex_lg)])
    exf = np.abs(np.array([float(e) for e in ex_lg]))
    assert np.all(d <= 2.0 ** -53 + 4 * np.spacing(exf))


def test_kernel_coefficients_match_generator():
    """The polynomial coefficients written in rt_math.h are the ones
    poly_coeffs.py generates (binary64 and binary32), in Horner order."""
    import importlib.util
    import re
    spec = importlib.util.spec_from_file_location("poly_coeffs", os.path.join(INC, "poly_coeffs.py"))
    pc = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(pc)
    src = open(os.path.join(INC, "rt_math.h")).read()
    nums = [float(v) for v in re.findall(r"fmaf?\(\w+, \w+, (-?[0-9.]+e?-?[0-9]*)f?\)", src)]
    inits = [float(v) for v in re.findall(r"(?:double|float) p\w* = (-?[0-9.]+e?-?[0-9]*)f?;", src)]
    for binary32 in (False, True):
        for name in (pc.DEGREES32 if binary32 else pc.USED64):
            cs = pc.coefficients(name, binary32)
            # the first coefficient initialises the accumulator, the others are
            # the additive terms of consecutive fused multiply-adds
            assert cs[0] in inits, (name, binary32)
            text = ", ".join(repr(c) for c in cs[1:])
            seq = [c for c in cs[1:]]
            found = any(nums[i:i + len(seq)] == seq for i in range(len(nums)))
            assert found, (name, binary32, text)


def test_rpow_tenth(driver):
    rng = np.random.default_rng(4)
    x = np.concatenate([10.0 ** rng.uniform(-12, 12, 3000), [1.0, 6.0, 1e-12, 1e12]])
    out = run(driver, "rpow_tenth", x)
    ex = [mp.power(mp.mpf(v), mp.mpf(-1) / 10) for v in x]
    # one Newton step from the binary32 estimate: relative error ~ (2e-7)^2
    rel = np.array([float(abs(mp.mpf(g) - e) / e) for g, e in zip(out, ex)])
    assert rel.max() < 1e-12


# ---------------------------------------------------------------- binary32
def ulp32_err(got, x32, fn):
    """Error in binary32 ulps of the exact value at the binary32 argument."""
    ex = np.array([float(fn(mp.mpf(float(v)))) for v in x32])
    ulp = np.spacing(np.abs(ex).astype(np.float32)).astype(np.float64)
    return np.abs(got - ex) / ulp


def test_binary32_sincos(driver):
    rng = np.random.default_rng(10)
    x = np.concatenate([rng.uniform(-2 * np.pi, 3 * np.pi, 3000), [0.0, 1e-30, 1.0, 100.0]])
    x32 = x.astype(np.float32)
    out = run(driver, "sincosf", x32.astype(np.float64)).reshape(-1, 2)
    es = np.array([float(mp.sin(mp.mpf(float(v)))) for v in x32])
    ec = np.array([float(mp.cos(mp.mpf(float(v)))) for v in x32])
    # absolute error against the magnitude 1 of sin and cos: below two binary32 ulps of 1
    assert np.abs(out[:, 0] - es).max() < 2.4e-7 and np.abs(out[:, 1] - ec).max() < 2.4e-7
    big = np.abs(es) > 1e-2
    assert ulp32_err(out[big, 0], x32[big], mp.sin).max() < 4


def test_binary32_exp_expm1_log1p(driver):
    rng = np.random.default_rng(11)
    xe = np.concatenate([rng.uniform(-80, 80, 2000), rng.uniform(-1, 1, 500), [0.0]]).astype(np.float32)
    assert ulp32_err(run(driver, "expf", xe.astype(np.float64)), xe, mp.exp).max() < 3
    xm = np.concatenate([rng.uniform(-0.6, 0.2, 2000), -(10.0 ** rng.uniform(-20, 1.5, 500)),
                         10.0 ** rng.uniform(-20, 1.5, 500)]).astype(np.float32)
    xm = xm[xm != 0]
    assert ulp32_err(run(driver, "expm1f", xm.astype(np.float64)), xm, mp.expm1).max() < 4
    xl = np.concatenate([10.0 ** rng.uniform(-3, 3.5, 2000), rng.uniform(-0.5, 0.5, 500)]).astype(np.float32)
    xl = xl[xl != 0]
    assert ulp32_err(run(driver, "log1pf", xl.astype(np.float64)), xl, mp.log1p).max() < 4
