"""Pins of the oracle's spacetime functions (paper Sec. 2 and Sec. 3.1).

Each check compares the oracle with something other than its own formulas:
textbook Kerr, the static seed form, a matrix inverse, numerical derivatives,
the mass-density relation of the seeds, and the extremal spin the paper prints.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from paper_2605_05635_amd import workloads as W

RNG = np.random.default_rng(1234)


def kerr_textbook(R, th, a):
    """Kerr in Boyer-Lindquist coordinates, M = 1 (any GR textbook)."""
    S = R * R + a * a * math.cos(th) ** 2
    D = R * R - 2 * R + a * a
    s2 = math.sin(th) ** 2
    return dict(g_TT=-(1 - 2 * R / S), g_Tph=-2 * a * R * s2 / S, g_RR=S / D, g_thth=S,
                g_phph=(R * R + a * a + 2 * a * a * R * s2 / S) * s2)


def imgs():
    return [W.image(metric="kerr", spin=0.7),
            W.image(metric="einasto", spin=0.6, halo=(0.25, 0.0)),
            W.image(metric="cnfw", spin=0.9, halo=(0.03, 8.0))]


def test_kerr_metric_is_textbook_kerr(orc):
    for a in (0.0, 0.3, 0.9, -0.5):
        img = W.image(metric="kerr", spin=a)
        for _ in range(20):
            R, th = RNG.uniform(2.5, 50), RNG.uniform(0.05, math.pi - 0.05)
            m, k = orc.metric(img, R, th), kerr_textbook(R, th, a)
            for key, v in k.items():
                assert m[key] == pytest.approx(v, rel=1e-13, abs=1e-15), key


def test_halo_metrics_reduce_to_kerr_bitwise(orc):
    """Sec. 2.2: H = 1 - 2/R gives F = 2R.  cNFW with eta = 0, and Einasto with
    lambda_E so small that exp(-R/lambda_E) underflows, are Kerr exactly."""
    for R in (1.2, 2.0, 7.5, 1000.0):
        for th in (0.3, 1.2):
            k = orc.metric(W.image(metric="kerr", spin=0.5), R, th)
            c = orc.metric(W.image(metric="cnfw", spin=0.5, halo=(0.0, 10.0)), R, th)
            e = orc.metric(W.image(metric="einasto", spin=0.5, halo=(0.001, 0.0)), R, th)
            for key in k:
                assert c[key] == k[key], key
                assert e[key] == k[key], key


def test_continuity_small_halo(orc):
    """eta -> 0 approaches Kerr continuously (difference O(eta))."""
    k = orc.metric(W.image(metric="kerr", spin=0.5), 6.0, 1.0)
    for eta in (1e-4, 1e-6, 1e-8):
        c = orc.metric(W.image(metric="cnfw", spin=0.5, halo=(eta, 10.0)), 6.0, 1.0)
        assert abs(c["F"] - k["F"]) < 1e3 * eta


def test_zero_spin_is_static_seed(orc):
    """Sec. 2.2: chi -> 0 gives the static seed, eq. (3)."""
    for img in imgs():
        img = dict(img, spin=0.0)
        for _ in range(10):
            R, th = RNG.uniform(2.5, 40), RNG.uniform(0.1, 3.0)
            m, r = orc.metric(img, R, th), orc.radial(img, R)
            H = r["H"]
            assert m["g_TT"] == pytest.approx(-H, rel=1e-13)
            assert m["g_RR"] == pytest.approx(1 / H, rel=1e-13)
            assert m["g_thth"] == pytest.approx(R * R, rel=1e-14)
            assert m["g_phph"] == pytest.approx(R * R * math.sin(th) ** 2, rel=1e-13)
            assert m["g_Tph"] == 0.0


def test_inverse_metric_is_matrix_inverse(orc):
    """eqs. (49)-(53) are the inverse of eqs. (27)-(31)."""
    for img in imgs():
        for _ in range(25):
            R, th = RNG.uniform(2.2, 200), RNG.uniform(0.05, math.pi - 0.05)
            m = orc.metric(img, R, th)
            g = np.zeros((4, 4))
            g[0, 0], g[0, 3], g[3, 0] = m["g_TT"], m["g_Tph"], m["g_Tph"]
            g[1, 1], g[2, 2], g[3, 3] = m["g_RR"], m["g_thth"], m["g_phph"]
            gi = np.linalg.inv(g)
            want = dict(u_TT=gi[0, 0], u_Tph=gi[0, 3], u_RR=gi[1, 1], u_thth=gi[2, 2],
                        u_phph=gi[3, 3])
            for key, v in want.items():
                assert m[key] == pytest.approx(v, rel=1e-10, abs=1e-14), key


def _richardson(f, x, h):
    d1 = (f(x + h) - f(x - h)) / (2 * h)
    d2 = (f(x + h / 2) - f(x - h / 2)) / h
    return (4 * d2 - d1) / 3


def test_radial_derivatives_match_numerical(orc):
    for img in imgs():
        for R in (1.7, 3.0, 11.0, 300.0):
            r = orc.radial(img, R)
            dF = _richardson(lambda x: orc.radial(img, x)["F"], R, 1e-3 * R)
            dH = _richardson(lambda x: orc.radial(img, x)["H"], R, 1e-3 * R)
            assert r["dF"] == pytest.approx(dF, rel=1e-8, abs=1e-11)
            assert r["dH"] == pytest.approx(dH, rel=1e-8, abs=1e-11)


def test_inverse_metric_derivatives_match_numerical(orc):
    keys = ("TT", "Tph", "RR", "thth", "phph")
    for img in imgs():
        for _ in range(8):
            R, th = RNG.uniform(2.5, 30), RNG.uniform(0.3, math.pi - 0.3)
            m = orc.metric(img, R, th)
            for k in keys:
                dR = _richardson(lambda x: orc.metric(img, x, th)["u_" + k], R, 1e-3)
                dt = _richardson(lambda x: orc.metric(img, R, x)["u_" + k], th, 1e-3)
                assert m["dR_" + k] == pytest.approx(dR, rel=1e-7, abs=1e-11), k
                assert m["dt_" + k] == pytest.approx(dt, rel=1e-7, abs=1e-11), k


def test_einasto_seed_is_exponential_density_of_unit_mass(orc):
    """eqs. (7), (9), (15): the Einasto-type mass function has dmu/dR = 4 pi R^2 rho
    with an exponential density rho ~ exp(-R/lambda_E); mu(0) = 0 (regular centre)
    and mu(infinity) = 1 (asymptotic Schwarzschild, H -> 1 - 2/R)."""
    for lam in (0.1, 0.3, 0.7):
        img = W.image(metric="einasto", halo=(lam, 0.0))
        ratios = []
        for R in (0.05, 0.3, 1.0, 2.0, 4.0):
            r = orc.radial(img, R)
            ratios.append(r["dmu"] / (R * R * math.exp(-R / lam)))
        assert np.ptp(ratios) < 1e-12 * max(ratios)
        # normalisation: total mass 1 <=> 4 pi rho0 int R^2 e^{-R/lam} = 8 pi lam^3 rho0 = 1
        assert ratios[0] == pytest.approx(1 / (2 * lam ** 3), rel=1e-13)
        assert orc.radial(img, 1e-3 * lam)["mu"] < 1e-9
        assert orc.radial(img, 60 * lam)["mu"] == pytest.approx(1.0, abs=1e-20)


def test_cnfw_lapse_exponent_is_enclosed_cored_nfw_mass(orc):
    """eqs. (11), (13), (14): with H = exp(E(R)) - 2/R, the halo exponent obeys
    dE/dR = 2 m(R)/R^2 where m is the mass of the cored-NFW density
    rho0 (1 + R/lambda_c)^-3 inside R (eta = 4 pi rho0 lambda_c^2), and E -> 0 at
    infinity."""
    for eta, lc in ((0.02, 10.0), (0.05, 5.0), (0.01, 20.0)):
        img = W.image(metric="cnfw", halo=(eta, lc))
        rho0 = eta / (4 * math.pi * lc * lc)
        for R in (0.5, 2.0, 9.0, 40.0, 500.0):
            r = orc.radial(img, R)
            e = r["H"] + 2 / R                   # exp(E)
            dE = (r["dH"] - 2 / (R * R)) / e      # E'
            m, _ = quad(lambda x: 4 * math.pi * x * x * rho0 * (1 + x / lc) ** -3, 0, R,
                        epsabs=0, epsrel=1e-13)
            assert dE == pytest.approx(2 * m / (R * R), rel=1e-9)
        far = orc.radial(img, 1e9)
        assert abs(math.log(far["H"] + 2e-9)) < 1e-6


def test_outer_horizon_kerr_closed_form(orc):
    for a in (0.0, 0.3, 0.5, 0.94, 0.999):
        r = orc.horizon(W.image(metric="kerr", spin=a))
        assert r == pytest.approx(1 + math.sqrt(1 - a * a), rel=1e-14)


def test_outer_horizon_is_largest_root(orc):
    for img in imgs():
        rp = orc.horizon(img)
        d = lambda R: orc.metric(img, R, 1.0)["Delta"]  # noqa: E731
        assert abs(d(rp)) < 1e-12
        Rs = np.linspace(rp * (1 + 1e-9), 60, 4000)
        assert all(d(R) > 0 for R in Rs)


def test_extremal_spin_paper_value(orc):
    """Sec. 2.2 (Fig. 2 caption): extremal spin 0.640 for the Einasto case and 1 for
    Kerr.  lambda_E = 0.3 is the Einasto scale the paper uses elsewhere (Fig. 5)."""
    chi_e, r_e = orc.extremal_spin(W.image(metric="einasto", halo=(0.3, 0.0)))
    assert chi_e == pytest.approx(0.640, abs=1e-3)
    chi_k, r_k = orc.extremal_spin(W.image(metric="kerr"))
    assert chi_k == pytest.approx(1.0, abs=1e-12) and r_k == pytest.approx(1.0, abs=1e-9)
    # just below / above the extremal spin the horizon appears / disappears
    base = W.image(metric="einasto", halo=(0.3, 0.0))
    assert orc.horizon(dict(base, spin=chi_e - 1e-6)) is not None
    assert orc.horizon(dict(base, spin=chi_e + 1e-6)) is None
    assert orc.extremal_spin(W.image(metric="einasto", halo=(0.45, 0.0))) is None
