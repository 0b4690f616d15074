"""Pins of the oracle's image diagnostics (paper Sec. 6.2, and the bright-peak
scale of Sec. 6.3) on synthetic intensity maps with closed-form answers.

* A circular Gaussian I = exp(-rho^2 / (2 s^2)) centred at (x0, y0): the
  centroid is (x0, y0), the flux 2 pi s^2, and rho about the centroid is
  Rayleigh distributed: rho_bar = s sqrt(pi/2), w = s sqrt(2 - pi/2); by
  mirror symmetry about a pixel column A_LR = 0.
* A uniform disc: P = 1 (the peak equals the emitting mean).
* A thin Gaussian ring of radius r0 about the origin: the radial profile
  peaks in the bin holding r0.
* Invariances: a constant factor changes only F and the intensities; an
  asymmetric brightness gives the sign of A_LR the closed form of two
  half-discs fixes.
"""
import math

import numpy as np
import pytest

from paper_2605_05635_amd import workloads as W


def screen(n=801, half=20.0):
    return W.image(nx=n, ny=n, x_min=-half, x_max=half, y_min=-half, y_max=half)


def grid(img):
    dx = (img["x_max"] - img["x_min"]) / img["nx"]
    X = img["x_min"] + (np.arange(img["nx"]) + 0.5) * dx
    dy = (img["y_max"] - img["y_min"]) / img["ny"]
    Y = img["y_min"] + (np.arange(img["ny"]) + 0.5) * dy
    return np.meshgrid(X, Y)


def test_gaussian_moments(orc):
    img = screen()
    Xg, Yg = grid(img)
    dx = (img["x_max"] - img["x_min"]) / img["nx"]
    x0, y0, s = 3.5 * dx, -5 * dx, 2.0      # x0 between two pixel columns
    I = np.exp(-((Xg - x0) ** 2 + (Yg - y0) ** 2) / (2 * s * s))
    d = orc.image_diagnostics(img, I, 0.1, 300)
    assert d["F"] == pytest.approx(2 * math.pi * s * s, rel=1e-10)
    assert d["X_c"] == pytest.approx(x0, abs=1e-10) and d["Y_c"] == pytest.approx(y0, abs=1e-10)
    assert d["C"] == pytest.approx(math.hypot(x0, y0), abs=1e-10)
    # midpoint sums of smooth rapidly decaying integrands: spectrally accurate
    # except for rho's kink at the centroid (a pixel-scale correction)
    assert d["rho_bar"] == pytest.approx(s * math.sqrt(math.pi / 2), rel=2e-4)
    assert d["d_img"] == pytest.approx(2 * s * math.sqrt(math.pi / 2), rel=2e-4)
    assert d["w_img"] == pytest.approx(s * math.sqrt(2 - math.pi / 2), rel=2e-3)
    assert d["w_over_d"] == pytest.approx(math.sqrt(2 - math.pi / 2) / (2 * math.sqrt(math.pi / 2)), rel=2e-3)
    assert abs(d["A_LR"]) < 1e-12


def test_uniform_disc_contrast_and_scale_invariance(orc):
    img = screen(401, 10.0)
    Xg, Yg = grid(img)
    I = ((Xg - 1.0) ** 2 + Yg ** 2 < 16.0).astype(np.float64)
    d = orc.image_diagnostics(img, I, 0.25, 100)
    assert d["P"] == 1.0 and d["I_max"] == 1.0 and d["I_mean_emitting"] == 1.0
    # the disc's mean radius about its centre: 2/3 of the radius
    assert d["rho_bar"] == pytest.approx(2 * 4.0 / 3, rel=2e-3)
    d7 = orc.image_diagnostics(img, 7.0 * I, 0.25, 100)
    for k in ("X_c", "Y_c", "C", "rho_bar", "d_img", "w_img", "w_over_d", "A_LR", "P", "rho_peak"):
        assert d7[k] == pytest.approx(d[k], rel=1e-13, abs=1e-15), k
    assert d7["F"] == pytest.approx(7 * d["F"], rel=1e-13)


def test_ring_peak_and_half_disc_asymmetry(orc):
    img = screen(601, 15.0)
    Xg, Yg = grid(img)
    r0 = 6.37
    rho0 = np.hypot(Xg, Yg)
    I = np.exp(-((rho0 - r0) ** 2) / (2 * 0.15 ** 2))
    bw = 0.2
    d = orc.image_diagnostics(img, I, bw, 80)
    assert d["rho_peak"] == pytest.approx((math.floor(r0 / bw) + 0.5) * bw, abs=1e-12)
    assert d["d_peak"] == pytest.approx(2 * d["rho_peak"], abs=1e-15)
    # a disc of radius R twice as bright on its right half: centroid
    # x_c = 4R/(9 pi); F_R = 2 seg(x_c), F_L = 2 (A/2 - seg(x_c)) + A/2 with
    # seg(c) = R^2 acos(c/R) - c sqrt(R^2 - c^2) the area beyond x = c
    R = 5.0
    disc = (rho0 < R).astype(np.float64)
    d2 = orc.image_diagnostics(img, disc * np.where(Xg > 0, 2.0, 1.0), bw, 80)
    xc = 4 * R / (9 * math.pi)
    seg = R * R * math.acos(xc / R) - xc * math.sqrt(R * R - xc * xc)
    A = math.pi * R * R
    FR, FL = 2 * seg, 2 * (A / 2 - seg) + A / 2
    assert d2["X_c"] == pytest.approx(xc, abs=5e-3)
    # on the pixel grid the column nearest X_c falls wholly on one side: up to
    # one column's share of the flux, 2 (2 R dx)/(1.5 pi R^2) = 0.0085 here (a
    # reference at the origin instead of X_c would give 1/3, swapped halves -0.094)
    assert d2["A_LR"] == pytest.approx((FR - FL) / (FR + FL), abs=0.01)
