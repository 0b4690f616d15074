"""Pins of the oracle's shadow-boundary search (paper Sec. 4.1, eqs. (78)-(79)).

The transition between captured and escaping rays along a screen direction is
compared with closed forms that do not use the oracle's ray tracer:

* non-rotating metrics: the critical impact parameter b_crit = min_R R/sqrt(f),
  f = 1 - F/R^2 (Sec. 2, Delta = R^2 - F at chi = 0), seen by the static
  observer at R_o under the angle sin(alpha) = b_crit sqrt(f(R_o))/R_o, i.e. at
  screen radius R_o tan(alpha) in every direction (Schwarzschild: b_crit = 3 sqrt(3));
* Kerr: the critical curve of the spherical photon orbits (Bardeen 1973), the
  constants xi(r) = l/E and eta(r) = Q/E^2 of the orbit at radius r mapped to
  the screen of the ZAMO at (R_o, theta_o) exactly (no large-distance limit):
  X = R_o p^(phi)/p^(R), Y = R_o p^(theta)/p^(R);
* the reflection symmetry Y -> -Y of the boundary (the metrics are symmetric
  under theta -> pi - theta and separable).

The search's own tolerance is 1e-9; the integrated flow places the transition
within about 1e-8 relative of the exact one (Dormand-Prince at rtol = atol =
1e-8), so the pins use 2e-7 relative.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq, minimize_scalar

from paper_2605_05635_amd import workloads as W

TOL_B = 1e-9
REL = 2e-7


def dirs_of(psi):
    psi = np.asarray(psi, dtype=np.float64)
    return np.stack([np.cos(psi), np.sin(psi)], axis=1)


def static_shadow_radius(orc, img):
    """R_o tan(alpha_c) for the non-rotating metric of img."""
    f = lambda R: 1.0 - orc.radial(img, R)["F"] / (R * R)
    g = lambda R: R / math.sqrt(f(R))
    r_plus = orc.horizon(img)
    Rs = np.linspace(1.05 * r_plus, 4.0 * r_plus, 600)
    i = int(np.argmin([g(R) for R in Rs]))
    res = minimize_scalar(g, bracket=(Rs[i - 1], Rs[i], Rs[i + 1]), tol=1e-12)
    b_crit = res.fun
    Ro = img["r_obs"]
    return Ro * math.tan(math.asin(b_crit * math.sqrt(f(Ro)) / Ro)), b_crit


def test_schwarzschild_closed_form(orc):
    img = W.image(metric="kerr", spin=0.0, incl=math.radians(60))
    psi = np.array([0.0, 0.9, 2.5, 4.0])
    lo, hi, ok = orc.shadow_boundary(img, dirs_of(psi), 4.0, 7.0, TOL_B)
    assert ok.all() and np.all(hi - lo <= TOL_B)
    Ro = img["r_obs"]
    exact = Ro * math.tan(math.asin(math.sqrt(27.0) * math.sqrt(1.0 - 2.0 / Ro) / Ro))
    assert np.all(np.abs(0.5 * (lo + hi) / exact - 1.0) < REL)
    # the closed form of the helper for the same metric
    assert static_shadow_radius(orc, img)[1] == pytest.approx(math.sqrt(27.0), rel=1e-10)


@pytest.mark.parametrize("img", [
    W.image(metric="einasto", spin=0.0, halo=(0.3, 0.0), incl=math.radians(60)),
    W.image(metric="cnfw", spin=0.0, halo=(0.02, 10.0), incl=math.radians(60)),
    W.image(metric="cnfw", spin=0.0, halo=(0.3, 4.0), incl=math.radians(120), r_obs=400.0),
])
def test_static_halo_closed_form(orc, img):
    psi = np.array([0.3, 2.0, 5.1])
    lo, hi, ok = orc.shadow_boundary(img, dirs_of(psi), 4.0, 9.0, TOL_B)
    assert ok.all()
    exact, _ = static_shadow_radius(orc, img)
    assert np.all(np.abs(0.5 * (lo + hi) / exact - 1.0) < REL)


def kerr_critical_point(chi, th_o, Ro, psi):
    """Screen point of the Kerr critical curve in direction psi, exactly for
    the ZAMO at (Ro, th_o) (M = 1, E = 1)."""
    a = chi
    s, c = math.sin(th_o), math.cos(th_o)
    Sig = Ro * Ro + a * a * c * c
    Del = Ro * Ro - 2.0 * Ro + a * a
    A = (Ro * Ro + a * a) ** 2 - a * a * Del * s * s
    g_phph = A * s * s / Sig

    def xy(r):
        xi = -(r ** 3 - 3.0 * r * r + a * a * r + a * a) / (a * (r - 1.0))
        eta = r ** 3 * (4.0 * a * a - r * (r - 3.0) ** 2) / (a * a * (r - 1.0) ** 2)
        Rr = (Ro * Ro + a * a - a * xi) ** 2 - Del * (eta + (xi - a) ** 2)
        Th = eta + a * a * c * c - xi * xi * c * c / (s * s)
        p_r = -math.sqrt(Rr) / math.sqrt(Sig * Del)        # frame components, inward
        p_ph = xi / math.sqrt(g_phph)
        p_th = math.sqrt(max(Th, 0.0)) / math.sqrt(Sig)
        return Ro * p_ph / p_r, abs(Ro * p_th / p_r), Th

    # the visible arc: Theta(th_o) >= 0 between the two photon-orbit radii
    rp = 2.0 * (1.0 + math.cos(2.0 / 3.0 * math.acos(-a)))
    rm = 2.0 * (1.0 + math.cos(2.0 / 3.0 * math.acos(a)))
    rs = np.linspace(rp + 1e-9, rm - 1e-9, 20001)
    th = np.array([xy(r)[2] for r in rs])
    vis = np.where(th >= 0)[0]
    r1 = brentq(lambda r: xy(r)[2], rs[vis[0] - 1], rs[vis[0]], xtol=1e-15) if vis[0] > 0 else rs[0]
    r2 = brentq(lambda r: xy(r)[2], rs[vis[-1]], rs[vis[-1] + 1], xtol=1e-15) if vis[-1] < len(rs) - 1 else rs[-1]
    sign = 1.0 if math.sin(psi) >= 0 else -1.0   # Y = R_o p^(th)/p^(R): p^(th) of either sign
    cross = lambda r: xy(r)[0] * math.sin(psi) - sign * xy(r)[1] * math.cos(psi)
    grid = np.linspace(r1, r2, 4001)
    vals = np.array([cross(r) for r in grid])
    k = np.where(np.sign(vals[:-1]) != np.sign(vals[1:]))[0]
    for kk in k:
        r = brentq(cross, grid[kk], grid[kk + 1], xtol=1e-15)
        X, Yabs, _ = xy(r)
        Y = sign * Yabs
        if X * math.cos(psi) + Y * math.sin(psi) > 0:
            return math.hypot(X, Y)
    raise AssertionError("no critical point in that direction")


@pytest.mark.parametrize("chi,incl", [(0.5, 60.0), (0.9, 60.0), (0.94, 163.0)])
def test_kerr_critical_curve(orc, chi, incl):
    img = W.image(metric="kerr", spin=chi, incl=math.radians(incl))
    psi = np.array([0.2, 1.3, 2.9, 3.6, 4.9])
    lo, hi, ok = orc.shadow_boundary(img, dirs_of(psi), 2.0, 9.0, TOL_B)
    assert ok.all()
    for p, b in zip(psi, 0.5 * (lo + hi)):
        exact = kerr_critical_point(chi, math.radians(incl), img["r_obs"], p)
        assert abs(b / exact - 1.0) < REL, (chi, incl, p, b, exact)


def test_reflection_symmetry_and_bad_bracket(orc):
    img = W.image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=math.radians(163))
    psi = np.array([0.7, -0.7, 2.2, -2.2])
    lo, hi, ok = orc.shadow_boundary(img, dirs_of(psi), 2.0, 9.0, TOL_B)
    assert ok.all()
    b = 0.5 * (lo + hi)
    assert abs(b[0] / b[1] - 1.0) < REL and abs(b[2] / b[3] - 1.0) < REL
    # a bracket that does not hold the transition is reported, not searched
    lo, hi, ok = orc.shadow_boundary(img, dirs_of([0.7, 0.7]), [9.0, 2.0][0], 12.0, TOL_B)
    assert not ok.any() and np.all(lo == 9.0) and np.all(hi == 12.0)
