"""Screen points and the screen refinement near lensing-band boundaries
(rt_trace_points, rt_refine_points; Sec. 4, bands of Sec. 4.2) on the GPU:
point rays against the oracle's trace of the same points (the parity bar of
parity_util), the marking and subpixel centres against the oracle's
refinement of the same maps, and sub = 1 against the image trace bit for bit."""
import sys

import numpy as np
import pytest

from paper_2605_05635_amd import workloads as W
from parity_util import compare, gpu_to_numpy, summary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_2605_05635_amd import rt as mod
    return mod


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def points_numpy(outs: dict) -> dict:
    """Point outputs -> numpy: per-point arrays (n) and records (3, n)."""
    return {k: t.cpu().numpy() if t.ndim == 2 else t.cpu().numpy().reshape(-1)
            for k, t in outs.items()}


def refine_gpu(rt, img, nc, st, sub, max_points=None):
    import torch
    d = torch.device("cuda")
    nc_t = torch.as_tensor(nc, device=d).contiguous()
    st_t = torch.as_tensor(st, device=d).contiguous()
    if max_points is None:
        return rt.refine_points(img, nc_t, st_t, sub)
    xy = torch.full((max(max_points, 1), 2), -7.0, dtype=torch.float64, device=d)
    pix = torch.full((max(max_points // (sub * sub), 1),), -1, dtype=torch.int64, device=d)
    n = torch.zeros(1, dtype=torch.int64, device=d)
    rt.rt_refine_points(rt.params_from(img), nc_t, st_t, sub, max_points, xy, pix, n)
    torch.cuda.synchronize()
    return xy.cpu().numpy(), pix.cpu().numpy(), int(n.item())


@pytest.mark.parametrize("label,img", [
    ("cnfw", W.cnfw_1024()),
    ("kerr", W.image(metric="kerr", spin=0.9, incl=1.2)),
    ("einasto", W.image(metric="einasto", spin=0.8, halo=(0.2, 0.0), incl=0.6, sigma_in=0.5,
                        sigma_out=0.5)),
])
def test_points_match_oracle(rt, orc, label, img):
    import torch
    pts = W.screen_points(7, 600)
    say(f"[refine] {label}: 600 seeded screen points")
    outs = rt.trace_points(img, pts)
    torch.cuda.synchronize()
    g = points_numpy(outs)
    o = orc.trace_points(img, pts)
    check_points(orc, img, g, o)
    assert (g["ncross"] >= 2).sum() > 20      # the annulus reaches the higher-order images


def check_points(orc, img, g, o):
    """The parity bar of parity_util, with g_n held to its 1e-9 relative bar
    after propagating the record's R_n difference (itself within 1e-6)
    through the oracle's emitter g(R) at the ray's E and l: near the photon
    ring a rounding-level difference of the trajectory, amplified over the
    turns before the third crossing, moves R_2 by more than g's bar allows."""
    ge = {k: v for k, v in g.items() if k != "g_em"}
    bad = compare(ge, o)
    assert not bad, "\n".join(bad) + "\n" + summary(g, o)
    same = (g["ncross"].astype(int) == o["ncross"]) & (g["status"].astype(int) == o["status"])
    rec = np.minimum(o["ncross"], 3)
    for j in range(3):
        for k in np.nonzero(same & (rec > j))[0]:
            go, Ro = o["g_em"][j, k], o["r_em"][j, k]
            shift = abs(orc.redshift(img, float(g["r_em"][j, k]), o["E"][k], o["L"][k]) - go)
            assert abs(g["g_em"][j, k] - go) <= 1e-15 + 1e-9 * abs(go) + shift, (j, k, Ro)
        none = same & (rec <= j)
        assert np.isnan(g["g_em"][j][none]).all()


@pytest.mark.parametrize("nx,ny,sub", [(37, 23, 3), (1, 17, 2), (29, 1, 1), (64, 48, 4)])
def test_marks_and_subpixels_match_oracle(rt, orc, nx, ny, sub):
    img = W.image(nx=nx, ny=ny, x_min=-7.0, x_max=5.0, y_min=-4.0, y_max=8.0)
    nc, st = W.band_maps(nx * 1000 + ny, nx, ny)
    xy, pix = refine_gpu(rt, img, nc, st, sub)
    pix_o, xy_o = orc.refine_points(img, nc, st, sub)
    assert np.array_equal(pix.cpu().numpy(), pix_o)
    # the same centres up to the rounding of one fused multiply-add
    assert np.allclose(xy.cpu().numpy(), xy_o, rtol=0.0, atol=2e-15 * 8.0)


def test_capacity_truncates_in_pixel_order(rt, orc):
    img = W.image(nx=40, ny=30)
    nc, st = W.band_maps(5, 40, 30)
    pix_o, xy_o = orc.refine_points(img, nc, st, 2)
    assert len(pix_o) > 20
    xy, pix, n = refine_gpu(rt, img, nc, st, 2, max_points=4 * 20 + 3)   # room for 20 pixels
    assert n == len(pix_o)
    assert np.array_equal(pix[:20], pix_o[:20]) and (pix[20:] == -1).all()
    assert np.allclose(xy[:80], xy_o[:80], rtol=0.0, atol=1e-13) and (xy[80:] == -7.0).all()
    xy, pix, n = refine_gpu(rt, img, np.zeros((30, 40), np.uint8), np.ones((30, 40), np.uint8), 2,
                            max_points=16)
    assert n == 0 and (pix == -1).all() and (xy == -7.0).all()


def test_sub1_retraces_the_image_bitwise(rt):
    """Refining with one subpixel per pixel gives the band-edge pixels' own
    centres; their rays reproduce the image's outputs there bit for bit."""
    import torch
    img = W.image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=1.2, nx=96, ny=80,
                  x_min=-10.0, x_max=10.0, y_min=-9.0, y_max=9.0)
    outs = rt.trace(img)
    xy, pix = rt.refine_points(img, outs["ncross"], outs["status"], 1)
    assert pix.numel() > 100
    pts = rt.trace_points(img, xy)
    torch.cuda.synchronize()
    p = pix.cpu().numpy()
    g_img, g_pts = gpu_to_numpy(outs, p), points_numpy(pts)
    for k, a in g_pts.items():
        assert np.array_equal(a, g_img[k], equal_nan=True), k


def test_refined_band_edges_end_to_end(rt, orc):
    """The oracle's own image, refined four-fold near its band edges by both
    sides, and the subpixel rays traced by both."""
    import torch
    img = W.image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=1.2, nx=30, ny=24,
                  x_min=-8.0, x_max=8.0, y_min=-7.0, y_max=7.0)
    o_img = orc.trace_pixels(img)
    nc = o_img["ncross"].astype(np.uint8).reshape(24, 30)
    st = o_img["status"].astype(np.uint8).reshape(24, 30)
    xy, pix = refine_gpu(rt, img, nc, st, 2)
    pix_o, xy_o = orc.refine_points(img, nc, st, 2)
    assert np.array_equal(pix.cpu().numpy(), pix_o) and len(pix_o) > 50
    say(f"[refine] end to end: {len(pix_o)} band-edge pixels, {4 * len(pix_o)} subpixel rays")
    pts = rt.trace_points(img, xy)
    torch.cuda.synchronize()
    g = points_numpy(pts)
    o = orc.trace_points(img, xy_o)
    check_points(orc, img, g, o)
