"""Pins of the oracle's image gradient (the derivative of the frozen discrete
map, by forward-mode dual numbers).

It is checked against central finite differences of the same frozen map
(each ray's attempt sequence replayed at perturbed parameters, plain double
arithmetic), which must agree to the differencing error, and against finite
differences of the full adaptive trace, which agree only to ~tol/h because the
controller's choices move with the parameters."""
import math

import numpy as np
import pytest

from paper_2605_05635_amd import workloads as W

CASES = [
    W.image(metric="kerr", spin=0.6, incl=math.radians(50), nx=24, ny=20),
    W.image(metric="einasto", spin=0.8, halo=(0.15, 0.0), incl=math.radians(70), nx=24, ny=20,
            sigma_in=0.5, sigma_out=0.5),
    W.image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=math.radians(60), nx=24, ny=20,
            x_min=-10, x_max=10, y_min=-10, y_max=10, sigma_in=0.5, sigma_out=0.5),
]


def _pixels(img, count=40, seed=3):
    return W.random_pixels(img["nx"], img["ny"], count, seed)


@pytest.mark.parametrize("img", CASES, ids=["kerr", "einasto-taper", "cnfw-taper"])
def test_dual_gradient_matches_frozen_finite_differences(orc, img):
    idx = _pixels(img)
    I, G = orc.trace_grad_pixels(img, idx)
    base_I = orc.trace_pixels(img, idx)["intensity"]
    assert np.array_equal(I, base_I)          # value part = the double trace, bitwise
    used = 0
    for j in range(4):
        if img["metric"] == "kerr" and j >= 2:
            assert np.all(G[:, j] == 0)
            continue
        if img["metric"] == "einasto" and j == 3:
            assert np.all(G[:, j] == 0)
            continue
        q = [img["spin"], img["incl"], *img["halo"]][j]
        d = 1e-6 * max(abs(q), 1e-2)
        Ip = orc.replay_pixels(img, orc.perturbed(img, j, d), idx)
        Im = orc.replay_pixels(img, orc.perturbed(img, j, -d), idx)
        fd = (Ip - Im) / (2 * d)
        scale = np.abs(G[:, j]).max() + 1e-300
        assert np.allclose(G[:, j], fd, rtol=2e-5, atol=2e-6 * scale), j
        used += 1
    assert used >= 2


def test_frozen_gradient_approximates_adaptive_derivative(orc):
    """Against differences of the full adaptive trace (the controller re-decides),
    the frozen-map derivative agrees to ~tol/h of the image's scale."""
    img = CASES[2]
    idx = _pixels(img, 30, 5)
    _, G = orc.trace_grad_pixels(img, idx)
    for j in (0, 1, 2, 3):
        q = [img["spin"], img["incl"], *img["halo"]][j]
        d = 1e-4 * abs(q)
        Ip = orc.trace_pixels(orc.perturbed(img, j, d), idx)["intensity"]
        Im = orc.trace_pixels(orc.perturbed(img, j, -d), idx)["intensity"]
        fd = (Ip - Im) / (2 * d)
        assert np.abs(G[:, j].sum() - fd.sum()) <= 2e-2 * np.abs(G[:, j]).sum() + 1e-12, j
