"""The ray tracer's reverse-mode pieces (rt_vjp.h), compiled for the host from
the same source the adjoint kernel uses, against independent derivatives:

* rhs_vjp, the hand-derived reverse mode of the Hamiltonian right-hand side
  (Sec. 3.1, eqs. (57)-(62)), against the dual-number Jacobian of the forward
  right-hand side, and that Jacobian against central differences;
* reverse_step, the adjoint of one accepted Dormand-Prince step with a
  crossing located on its continuous extension (Sec. 3.3) and the emission of
  that crossing (Sec. 5.2, eqs. (89)-(91)), against central differences of the
  forward step attempt the trace kernels run, with the step size frozen;
* crossing_root, the equatorial crossing on a step's continuous extension
  (Sec. 3.3), against the root of the same quartic in 40-digit arithmetic.
"""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "adjoint", "vjp_driver.hip")
INC = [os.path.join(ROOT, "include"), os.path.join(ROOT, "paper_2605_05635_amd", "csrc")]

KERR, EINASTO, CNFW = 0, 1, 2


def build_driver(tmp_path_factory, defines=()):
    exe = str(tmp_path_factory.mktemp("vjp") / "vjp_driver")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-ffp-contract=on", *defines]
    for d in INC:
        cmd += ["-I", d]
    subprocess.run(cmd + [SRC, "-o", exe], check=True, capture_output=True)
    return exe


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    return build_driver(tmp_path_factory)


@pytest.fixture(scope="module", params=[5.96e-8, -5.96e-8])
def driver_rcp_err(tmp_path_factory, request):
    """The same driver with the device's reciprocal estimate emulated: every
    dm::recip_estimate off by 2^-24 relative (the hardware's is within
    2^-24.4), with either sign."""
    return build_driver(tmp_path_factory, [f"-DRT_HOST_RECIP_ESTIMATE_ERROR={request.param!r}"])


def run(exe, mode, rows, width_out):
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    out = subprocess.run([exe, mode], input=rows.tobytes(), capture_output=True,
                         check=True).stdout
    return np.frombuffer(out, dtype=np.float64).reshape(len(rows), width_out)


def mass_consts(metric, rng):
    if metric == EINASTO:
        return [1.0 / rng.uniform(0.1, 0.3), 0.0, 0.0]
    if metric == CNFW:
        lc = rng.uniform(5.0, 20.0)
        eta = rng.uniform(0.005, 0.05)
        return [lc, 1.0 / lc, eta * lc]
    return [0.0, 0.0, 0.0]


def rhs_rows(metric, n, seed):
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n):
        chi = rng.uniform(0.1, 0.95)
        rows.append([metric, chi, *mass_consts(metric, rng),
                     rng.uniform(0.8, 1.2), rng.uniform(-5, 5),          # E, l
                     rng.uniform(2.5, 40.0), rng.uniform(0.3, 2.8),       # R, theta
                     rng.uniform(-2, 2), rng.uniform(-4, 4),              # p_R, p_theta
                     *rng.normal(size=4)])
    return np.array(rows)


@pytest.mark.parametrize("metric", [KERR, EINASTO, CNFW])
def test_rhs_vjp_matches_dual_jacobian(driver, metric):
    rows = rhs_rows(metric, 200, 10 + metric)
    out = run(driver, "rhs", rows, 24)
    vjp, dual = out[:, :10], out[:, 10:20]
    scale = np.abs(dual).max(axis=1, keepdims=True)
    assert np.all(np.abs(vjp - dual) <= 1e-12 * scale + 1e-300)


@pytest.mark.parametrize("metric", [KERR, EINASTO, CNFW])
def test_rhs_dual_jacobian_matches_differences(driver, metric):
    rows = rhs_rows(metric, 20, 20 + metric)
    base = run(driver, "rhs", rows, 24)
    # input columns of (R, th, pR, pth, E, l, chi, m0, m1, m2)
    cols = [7, 8, 9, 10, 5, 6, 1, 2, 3, 4]
    g = rows[:, 11:15]
    for j, col in enumerate(cols):
        if metric == KERR and j >= 7:
            continue
        if metric == EINASTO and j >= 8:
            continue
        dv = 1e-6 * np.maximum(1.0, np.abs(rows[:, col]))
        up, dn = rows.copy(), rows.copy()
        up[:, col] += dv
        dn[:, col] -= dv
        fd = ((run(driver, "rhs", up, 24)[:, 20:] - run(driver, "rhs", dn, 24)[:, 20:])
              * g).sum(axis=1) / (2 * dv)
        ref = base[:, 10 + j]
        scale = np.abs(base[:, 10:20]).max(axis=1)
        assert np.all(np.abs(fd - ref) <= 2e-6 * scale), (j, np.abs(fd - ref).max())


def step_rows(metric, n, seed, crossing):
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n):
        chi = rng.uniform(0.1, 0.9)
        R = rng.uniform(4.0, 12.0)
        if crossing:
            th = np.pi / 2 - rng.uniform(0.005, 0.02)
            pth = rng.uniform(1.5, 3.0) * R * R / 36.0
        else:
            th = rng.uniform(0.4, 1.2)
            pth = rng.uniform(-1, 1)
        rows.append([metric, chi, *mass_consts(metric, rng),
                     rng.uniform(1.5, 3.0), 20.0, 0.5, 0.5, 3.0,     # window and emissivity
                     rng.uniform(0.95, 1.05), rng.uniform(-2, 2),     # E, l
                     R, th, rng.uniform(-0.5, 0.5), pth,
                     rng.uniform(0.5, 1.0) * (R / 6.0) ** 1.5,        # h
                     rng.normal(), *rng.normal(size=4)])
    return np.array(rows)


@pytest.mark.parametrize("metric", [KERR, EINASTO, CNFW])
@pytest.mark.parametrize("crossing", [True, False])
def test_reverse_step_matches_differences(driver, metric, crossing):
    rows = step_rows(metric, 16, 30 + metric + 3 * crossing, crossing)
    base = run(driver, "step", rows, 14)
    keep = base[:, 1] == 1.0
    keep &= base[:, 2] == (1.0 if crossing else 0.0)
    assert keep.sum() >= 8
    rows, base = rows[keep], base[keep]
    grad = base[:, 3:]
    # columns of (R, th, pR, pth, E, l, chi, m0, m1, m2, r_in)
    cols = [12, 13, 14, 15, 10, 11, 1, 2, 3, 4, 5]
    scale = np.abs(grad).max(axis=1)
    for j, col in enumerate(cols):
        dv = 1e-6 * np.maximum(1.0, np.abs(rows[:, col]))
        up, dn = rows.copy(), rows.copy()
        up[:, col] += dv
        dn[:, col] -= dv
        ou, od = run(driver, "step", up, 14), run(driver, "step", dn, 14)
        # the frozen decisions must not move under the perturbation
        assert np.array_equal(ou[:, 1:3], base[:, 1:3]) and np.array_equal(od[:, 1:3], base[:, 1:3])
        fd = (ou[:, 0] - od[:, 0]) / (2 * dv)
        assert np.all(np.abs(fd - grad[:, j]) <= 1e-6 * scale), (j, np.abs(fd - grad[:, j]).max())
    if crossing:
        # the crossing's emission reaches the inner-edge adjoint (exactly zero
        # only where the taper has saturated)
        assert np.any(grad[:, 10] != 0.0)
    else:
        assert np.all(grad[:, 10] == 0.0)


def test_crossing_root_with_inexact_reciprocal(driver_rcp_err):
    """The plain Newton steps divide through the hardware reciprocal estimate;
    with a 2^-24 error in every such reciprocal the roots keep the exact
    division's accuracy."""
    test_crossing_root(driver_rcp_err)


def test_crossing_root(driver):
    """The root of theta(s) = pi/2 on the quartic extension, to a few ulp of s
    (its conditioning here: one ulp of pi/2 over |dtheta/ds| ~ 0.08).  Among the
    cases are extensions on which the Newton iteration lands on a point where
    the extension evaluates to exactly pi/2, from which it once fell back to
    bisection and stopped up to 1e-10 away, and extensions that turn near the
    crossing, where the plain Newton steps hand over to the safeguarded
    search."""
    import mpmath as mp
    mp.mp.dps = 40
    half_pi = 1.5707963267948966
    rng = np.random.default_rng(7)
    rows = []
    for _ in range(400):
        d0 = rng.uniform(1e-4, 0.05) * rng.choice([-1.0, 1.0])   # theta(0) - pi/2
        c1 = -np.sign(d0) * rng.uniform(abs(d0) * 1.05, 0.15)    # crosses inside (0, 1)
        c2, c3, c4 = rng.normal(0, 1e-4), rng.normal(0, 1e-4), rng.normal(0, 1e-6)
        # back to the extension's coefficients: c4 = r5, c3 = -r4 - 2 r5,
        # c2 = r4 + r5 - r3, c1 = r2 + r3
        r5 = c4
        r4 = -c3 - 2.0 * r5
        r3 = r4 + r5 - c2
        r2 = c1 - r3
        rows.append([half_pi + d0, r2, r3, r4, r5, 1.0 if d0 >= 0 else 0.0])
    # extensions that flatten out at the crossing: f = A (s - s0)^3 + eps (s - s0),
    # on which Newton's steps shrink the error only by ~2/3 each until they reach
    # sqrt(eps/A), so four plain steps do not pin the root down
    for _ in range(60):
        A, s0, eps = rng.uniform(0.02, 0.2), rng.uniform(0.2, 0.8), rng.uniform(1e-4, 1e-3)
        sg = rng.choice([-1.0, 1.0])
        f0, c1, c2, c3 = sg * (-A * s0 ** 3 - eps * s0), sg * (3 * A * s0 ** 2 + eps), sg * (-3 * A * s0), sg * A
        r5 = 0.0
        r4 = -c3 - 2.0 * r5
        r3 = r4 + r5 - c2
        r2 = c1 - r3
        rows.append([half_pi + f0, r2, r3, r4, r5, 1.0 if f0 >= 0 else 0.0])
    rows = np.array(rows)
    s = run(driver, "root", rows, 1)[:, 0]
    for row, got in zip(rows, s):
        y0, r2, r3, r4, r5 = row[:5]
        c1, c2, c3, c4 = r2 + r3, r4 + r5 - r3, -r4 - 2.0 * r5, r5   # as the kernel forms them
        f = lambda x: (mp.mpf(y0) + x * (mp.mpf(c1) + x * (mp.mpf(c2) + x * (mp.mpf(c3) + x * mp.mpf(c4))))
                       - mp.mpf(half_pi))
        exact = mp.findroot(f, (mp.mpf(0), mp.mpf(1)), solver="anderson")
        # the evaluation's rounding (a few ulp of its largest term) over the
        # slope at the root: 1e-14 for the first cases, more where it flattens
        slope = abs(float(mp.diff(f, exact)))
        tol = 1e-14 + 8 * 2.0 ** -53 * (abs(c1) + abs(c2) + abs(c3) + abs(c4)) / slope
        assert 0.0 < got < 1.0
        assert abs(got - float(exact)) < tol, (row, got, float(exact), tol)
