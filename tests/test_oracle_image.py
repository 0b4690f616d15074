"""Pins of the oracle's per-image reductions (paper Sec. 6.2 and 6.4) against
closed forms for Gaussian images, and of the screen pixel convention."""
import math

import numpy as np
import pytest

from paper_2605_05635_amd import workloads as W


def gaussian_image(img, x0, y0, s):
    X = img["x_min"] + (np.arange(img["nx"]) + 0.5) * (img["x_max"] - img["x_min"]) / img["nx"]
    Y = img["y_min"] + (np.arange(img["ny"]) + 0.5) * (img["y_max"] - img["y_min"]) / img["ny"]
    return np.exp(-((X[None, :] - x0) ** 2 + (Y[:, None] - y0) ** 2) / (2 * s * s))


def test_flux_and_centroid_of_gaussian(orc):
    img = W.image(nx=201, ny=173, x_min=-14, x_max=14, y_min=-15, y_max=13)
    I = gaussian_image(img, 1.3, -2.1, 1.2)
    F, Xc, Yc = orc.flux_centroid(img, I)
    assert F == pytest.approx(2 * math.pi * 1.2 ** 2, rel=1e-10)
    assert Xc == pytest.approx(1.3, abs=1e-10) and Yc == pytest.approx(-2.1, abs=1e-10)


def test_visibility_of_gaussian(orc):
    """|V(u,v)|/|V(0,0)| of a Gaussian of width s is exp(-2 pi^2 s^2 q^2), and a
    shift only changes the phase."""
    img = W.image(nx=160, ny=150, x_min=-12, x_max=12, y_min=-12, y_max=12)
    s = 1.6
    I = gaussian_image(img, 0.7, 0.4, s)
    uv = W.uv_points(11, 40)
    amp = orc.visibility_amplitude(img, I, uv)
    q2 = (uv ** 2).sum(1)
    assert np.allclose(amp, np.exp(-2 * math.pi ** 2 * s * s * q2), rtol=0, atol=1e-10)


def test_pixel_centres_and_workloads(batch64):
    img = W.kerr_small()
    assert (img["x_max"] - img["x_min"]) / img["nx"] == 0.375
    from oracle import oracle as O
    X, Y = O.pixel_xy(img, np.array([0, 63, 64, 4095]))
    assert X[0] == -12 + 0.1875 and X[1] == 12 - 0.1875 and Y[2] == -12 + 0.375 + 0.1875
    assert Y[3] == 12 - 0.1875
    a, b = W.einasto_512(), W.einasto_512()
    assert a == b and 0.10 <= a["halo"][0] <= 0.18
    batch = batch64
    assert len(batch) == 64 and {d["metric"] for d in batch} == {"kerr", "einasto", "cnfw"}
    assert all(d["nx"] in (128, 256, 512, 768) for d in batch)
    # the Einasto halos span the drawn range, each with a horizon at its spin
    from conftest import oracle_einasto_extremal_spin as ce
    lam = [d["halo"][0] for d in batch if d["metric"] == "einasto"]
    assert min(lam) < 0.08 and max(lam) > 0.25
    assert all(ce(d["halo"][0]) >= d["spin"] + 0.005 for d in batch if d["metric"] == "einasto")


def elliptical_gaussian(img, x0, y0, sx, sy):
    X = img["x_min"] + (np.arange(img["nx"]) + 0.5) * (img["x_max"] - img["x_min"]) / img["nx"]
    Y = img["y_min"] + (np.arange(img["ny"]) + 0.5) * (img["y_max"] - img["y_min"]) / img["ny"]
    return np.exp(-(X[None, :] - x0) ** 2 / (2 * sx * sx) - (Y[:, None] - y0) ** 2 / (2 * sy * sy))


def test_ring_average_and_cut_of_gaussians(orc):
    """Sec. 6.4's summaries.  A circular Gaussian of width s: V(q) = V(|u|, 0) =
    exp(-2 pi^2 s^2 q^2).  An elliptical one (sx, sy): the cut is
    exp(-2 pi^2 sx^2 q^2) and the angular mean of exp(-2 pi^2 q^2 (sx^2 cos^2 +
    sy^2 sin^2)) is exp(-pi^2 q^2 (sx^2 + sy^2)) I_0(pi^2 q^2 (sx^2 - sy^2))."""
    from scipy.special import i0
    img = W.image(nx=150, ny=140, x_min=-12, x_max=12, y_min=-11, y_max=11)
    q = np.linspace(0.0, 0.45, 10)
    avg, cut = orc.visibility_rings(img, gaussian_image(img, 0.5, -0.4, 1.3), q, 48)
    want = np.exp(-2 * math.pi ** 2 * 1.3 ** 2 * q ** 2)
    assert np.allclose(avg, want, atol=1e-10) and np.allclose(cut, want, atol=1e-10)
    sx, sy = 1.1, 0.6
    avg, cut = orc.visibility_rings(img, elliptical_gaussian(img, -0.3, 0.2, sx, sy), q, 48)
    a, b = math.pi ** 2 * q ** 2 * (sx * sx + sy * sy), math.pi ** 2 * q ** 2 * (sx * sx - sy * sy)
    assert np.allclose(cut, np.exp(-2 * math.pi ** 2 * sx * sx * q ** 2), atol=1e-10)
    assert np.allclose(avg, np.exp(-a) * i0(b), atol=1e-10)
    # the mean is over directions, not one point: the image is widest along X,
    # so the cut along u is the lowest of all directions
    assert np.all(avg[1:] > cut[1:])


def test_relative_deviation_of_gaussian_diagnostics(orc):
    """delta Q (Sec. 6.2) of a Gaussian image of width 1.5 s against one of width
    s: the flux scales as the width squared (delta F = 1.25), the mean radius
    and the width with it (delta = 0.5), the relative width not at all; a model
    equal to its reference has delta Q = 0 throughout."""
    img = W.image(nx=220, ny=200, x_min=-14, x_max=14, y_min=-13, y_max=13)
    s = 1.2
    d1 = orc.image_diagnostics(img, gaussian_image(img, 0.4, 0.3, s), 0.1, 100)
    d2 = orc.image_diagnostics(img, gaussian_image(img, 0.4, 0.3, 1.5 * s), 0.1, 100)
    keys = ("F", "rho_bar", "d_img", "w_img", "w_over_d")
    delta = orc.relative_to_reference([d2[k] for k in keys], [d1[k] for k in keys])
    assert delta == pytest.approx([1.25, 0.5, 0.5, 0.5, 0.0], abs=2e-3)
    assert np.all(orc.relative_to_reference([d1[k] for k in keys], [d1[k] for k in keys]) == 0.0)
