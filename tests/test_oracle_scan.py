"""Pins of the oracle's parameter scan (Sec. 2): Kerr's closed forms R_+ =
1 + sqrt(1 - chi^2), the ergosurface 1 + sqrt(1 - chi^2 cos^2 theta) and the
extremal spin 1 at r_e = 1; the ergosurface meets the horizon at the poles
and lies at R = 2 on the equator for every spin; the paper's printed extremal
spin 0.640 of the Einasto seed with lambda_E = 0.3 (Fig. 2 caption);
R_+ < ergosurface <= the static limit of the non-rotating metric."""
import math

import numpy as np
import pytest


def test_kerr_closed_forms(orc):
    pts = [("kerr", chi, 0.0, 0.0, th) for chi in (0.0, 0.3, 0.7, 0.95) for th in (0.2, 1.0, math.pi / 2)]
    out = orc.parameter_scan(pts)
    for (m, chi, _, _, th), (rp, rerg, ce, re) in zip(pts, out):
        assert rp == pytest.approx(1 + math.sqrt(1 - chi * chi), rel=1e-12)
        assert rerg == pytest.approx(1 + math.sqrt(1 - chi * chi * math.cos(th) ** 2), rel=1e-12)
        assert ce == pytest.approx(1.0, rel=1e-12) and re == pytest.approx(1.0, rel=1e-6)
    eq = orc.parameter_scan([("kerr", 0.9, 0.0, 0.0, math.pi / 2)])[0]
    assert eq[1] == pytest.approx(2.0, rel=1e-12)
    pole = orc.parameter_scan([("kerr", 0.9, 0.0, 0.0, 0.0)])[0]
    assert pole[1] == pytest.approx(pole[0], rel=1e-12)
    beyond = orc.parameter_scan([("kerr", 1.05, 0.0, 0.0, 1.0)])[0]
    assert math.isnan(beyond[0]) and beyond[2] == pytest.approx(1.0, rel=1e-12)


def test_halo_metrics(orc):
    out = orc.parameter_scan([("einasto", 0.5, 0.3, 0.0, 1.0), ("cnfw", 0.9, 0.02, 10.0, 0.7),
                              ("cnfw", 0.0, 0.05, 5.0, 1.3)])
    assert out[0, 2] == pytest.approx(0.640, abs=5e-4)
    for rp, rerg, ce, re in out:
        assert rp < rerg or math.isclose(rp, rerg, rel_tol=1e-12)
        assert ce > 0 and 0 < re < rp + 1.0
