"""Parity of the HIP path (through the C ABI) with the CPU oracle, on the GPU.

Small screens are compared on every pixel (several tiles plus a ragged tail);
the full-size workloads are traced exactly as bench.py launches them and
compared on seeded pixel samples the oracle computes one by one.
"""
import math
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


def run_full(rt, orc, img, emission=True):
    import torch
    say(f"[parity] full screen {img['metric']} {img['nx']}x{img['ny']} chi={img['spin']}")
    outs = rt.trace(img, emission=emission)
    torch.cuda.synchronize()
    g = gpu_to_numpy(outs)
    o = orc.trace_pixels(img)
    return g, o


def assert_parity(g, o, emission=True):
    bad = compare(g, o, emission)
    assert not bad, "\n".join(bad) + "\n" + summary(g, o)


def test_kerr_small_full_screen(rt, orc):
    """Kerr chi=0.5, theta_o=17 deg, 64x64 over +-12 M: every pixel."""
    img = W.kerr_small()
    g, o = run_full(rt, orc, img)
    assert_parity(g, o)
    say(summary(g, o))


@pytest.mark.parametrize("img", [
    W.image(metric="einasto", spin=0.9, halo=(0.14, 0.0), incl=math.radians(60),
            nx=97, ny=61, x_min=-10, x_max=10, y_min=-10, y_max=10),
    W.image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=math.radians(163),
            nx=83, ny=71, x_min=-10, x_max=10, y_min=-10, y_max=10),
    W.image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=math.radians(60),
            nx=67, ny=59, x_min=-10, x_max=10, y_min=-10, y_max=10, sigma_in=0.5, sigma_out=0.5),
    W.image(metric="kerr", spin=0.99, incl=math.radians(85), nx=75, ny=49),
    W.image(metric="einasto", spin=0.3, halo=(0.3, 0.0), incl=math.radians(30), nx=1, ny=1),
    W.image(metric="kerr", spin=0.0, incl=math.radians(45), nx=129, ny=1, y_min=-0.1, y_max=0.1),
    W.image(metric="cnfw", spin=-0.6, halo=(0.05, 5.0), incl=math.radians(120), nx=1, ny=77),
    W.image(metric="cnfw", spin=0.5, halo=(0.6, 4.0), incl=math.radians(70), nx=41, ny=37,
            x_min=-14, x_max=14, y_min=-14, y_max=14),
    W.image(metric="cnfw", spin=0.7, halo=(0.33, 3.0), incl=math.radians(110), nx=39, ny=35,
            x_min=-12, x_max=12, y_min=-12, y_max=12),
], ids=["einasto-ragged", "cnfw-163-ragged", "cnfw-taper", "kerr-0.99-edge-on", "one-pixel",
        "one-row", "one-column-retrograde", "cnfw-dense-halo", "cnfw-eta-0.33"])
def test_ragged_screens(rt, orc, img):
    g, o = run_full(rt, orc, img)
    assert_parity(g, o)
    say(summary(g, o))


@pytest.mark.parametrize("k", range(16))
def test_random_configurations(rt, orc, k):
    """Seeded draws over metrics, spins (prograde and retrograde),
    inclinations, observer radii, tolerances and emission windows: every
    pixel at the parity bar."""
    img = W.random_small_images(21, 16)[k]
    say(f"[parity] random {k}: incl {math.degrees(img['incl']):.1f} deg, r_obs {img['r_obs']:.0f}, "
        f"tol {img['rtol']:.1e}, halo {img['halo']}, taper {img['sigma_in']:.2f}")
    g, o = run_full(rt, orc, img)
    assert_parity(g, o)


@pytest.mark.parametrize("img", [
    W.image(metric="kerr", spin=0.5, incl=math.radians(17), nx=1, ny=97, y_min=-10, y_max=10),
    W.image(metric="kerr", spin=0.0, incl=math.radians(60), nx=1, ny=64),
    W.image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=math.radians(163), nx=3, ny=61,
            x_min=-0.1, x_max=0.1, y_min=-10, y_max=10),
], ids=["kerr-17-axis", "schwarzschild-60-axis", "cnfw-163-axis"])
def test_rays_over_the_pole(rt, orc, img):
    """Screens whose centre column is X = 0 exactly: those photons have l = 0
    and may pass over a pole, where theta leaves (0, pi); their crossings
    continue on the equator's far side (azimuth phi + pi)."""
    g, o = run_full(rt, orc, img)
    assert_parity(g, o)
    # the case holds rays whose theta leaves (0, pi) (logged by the oracle)
    X, Y = orc.pixel_xy(img, np.arange(img["nx"] * img["ny"]))
    axis = X == 0.0
    assert axis.sum() >= img["ny"]
    over = 0
    for x, y in zip(X[axis][::2], Y[axis][::2]):
        _, log = orc.trace_ray(img, x, y, log_cap=20000)
        over += bool(((log[:, 4] <= 0.0) | (log[:, 4] >= math.pi)).any())
    assert over >= 5, "no ray passes over a pole in this case"
    say(summary(g, o) + f"; {over} sampled rays over a pole")


def test_transfer_maps_only(rt, orc):
    img = W.image(metric="cnfw", spin=0.7, halo=(0.03, 12.0), incl=math.radians(50), nx=40,
                  ny=36)
    g, o = run_full(rt, orc, img, emission=False)
    assert_parity(g, o, emission=False)
    assert "intensity" not in g


def test_step_budget_and_edge_cases(rt, orc):
    """max_attempts = 5 ends every ray with STEP_LIMIT; a tiny budget and a
    screen entirely inside the shadow still agree pixel by pixel."""
    for img in (W.image(nx=16, ny=16, max_attempts=5),
                W.image(nx=16, ny=16, max_attempts=60),
                W.image(nx=33, ny=17, x_min=-1, x_max=1, y_min=-1, y_max=1)):
        g, o = run_full(rt, orc, img)
        assert_parity(g, o)
    assert (g["status"] == 1).all() and (g["ncross"] >= 0).all()


def _sampled(rt, orc, img, count, seed):
    import torch
    say(f"[parity] full-size {img['metric']} {img['nx']}x{img['ny']}, {count} sampled pixels")
    outs = rt.trace(img)
    torch.cuda.synchronize()
    idx = W.random_pixels(img["nx"], img["ny"], count, seed)
    g = gpu_to_numpy(outs, idx)
    o = orc.trace_pixels(img, idx)
    return g, o, outs


def test_einasto_512_sampled(rt, orc):
    img = W.einasto_512()
    g, o, outs = _sampled(rt, orc, img, 1500, 21)
    assert_parity(g, o)
    say(summary(g, o))


def test_cnfw_1024_sampled(rt, orc):
    img = W.cnfw_1024()
    g, o, outs = _sampled(rt, orc, img, 1500, 31)
    assert_parity(g, o)
    say(summary(g, o))
    # properties of the whole image, at any size
    nc = outs["ncross"].cpu().numpy()
    st = outs["status"].cpu().numpy()
    assert set(np.unique(st).tolist()) <= {1, 2}
    r = outs["r_em"].cpu().numpy()
    assert np.isnan(r[0][nc == 0]).all() and np.isfinite(r[0][nc >= 1]).all()
    I = outs["intensity"].cpu().numpy()
    assert np.isfinite(I).all() and (I >= 0).all()


@pytest.mark.parametrize("shape", [(1_048_579, 3), (3, 1_048_579)])
def test_long_thin_screens_sampled(rt, orc, shape):
    """Screens of 3.1 M pixels, one side 2^20 + 3 and the other 3 (ragged
    tiles clamped to the short side), sampled against the oracle."""
    nx, ny = shape
    wide = nx > ny
    img = dict(W.cnfw_1024(), nx=nx, ny=ny,
               x_min=-10.0 if wide else -0.4, x_max=10.0 if wide else 0.4,
               y_min=-0.4 if wide else -10.0, y_max=0.4 if wide else 10.0)
    g, o, outs = _sampled(rt, orc, img, 400, 41 if wide else 43)
    assert_parity(g, o)
    say(summary(g, o))
    st = outs["status"].cpu().numpy()
    assert set(np.unique(st).tolist()) <= {1, 2}
    I = outs["intensity"].cpu().numpy()
    assert np.isfinite(I).all() and (I >= 0).all()


def test_reduce_flux_centroid(rt, orc):
    img = W.image(metric="einasto", spin=0.9, halo=(0.14, 0.0), incl=math.radians(60),
                  nx=96, ny=80, x_min=-10, x_max=10, y_min=-10, y_max=10)
    import torch
    outs = rt.trace(img)
    torch.cuda.synchronize()
    g = gpu_to_numpy(outs)
    F, Xc, Yc = orc.flux_centroid(img, g["intensity"])
    assert g["reduce"][0] == pytest.approx(F, rel=1e-12)
    assert g["reduce"][1] == pytest.approx(Xc, rel=1e-12, abs=1e-12)
    assert g["reduce"][2] == pytest.approx(Yc, rel=1e-12, abs=1e-12)
    o = orc.trace_image(img)
    F2, Xc2, Yc2 = orc.flux_centroid(img, o["intensity"])
    assert g["reduce"][0] == pytest.approx(F2, rel=1e-6)
    assert g["reduce"][1] == pytest.approx(Xc2, abs=1e-6)


def test_deterministic_and_batched_equals_single(rt):
    """Two runs are bitwise equal, and each image of a multi-image call equals its
    single-image call bit for bit."""
    import torch
    imgs = [W.image(metric="kerr", spin=0.3, nx=48, ny=40),
            W.image(metric="cnfw", spin=0.8, halo=(0.02, 8.0), incl=1.0, nx=31, ny=50),
            W.image(metric="einasto", spin=0.5, halo=(0.2, 0.0), incl=2.0, nx=64, ny=64),
            W.image(metric="cnfw", spin=0.5, halo=(0.6, 4.0), incl=1.2, nx=29, ny=33)]
    singles = [rt.trace(i) for i in imgs]
    again = [rt.trace(i) for i in imgs]
    many = rt.trace_many(imgs)
    torch.cuda.synchronize()
    for a, b, c in zip(singles, again, many):
        for k in a:
            x, y, z = (t.cpu().numpy() for t in (a[k], b[k], c[k]))
            assert np.array_equal(x, y, equal_nan=True), k
            assert np.array_equal(x, z, equal_nan=True), k


def test_intensity_without_crossing_outputs(rt):
    """The emission pass reads the crossing counts and radii: a call that asks
    for the intensities only (no ncross, no r_em) gets them from scratch
    buffers and returns the same intensities, for a single image, a batch with
    one such image and a mixed-precision image."""
    import torch
    imgs = [W.image(metric="cnfw", spin=0.9, halo=(0.03, 7.0), incl=1.2, nx=45, ny=38),
            W.image(metric="kerr", spin=0.4, incl=0.7, nx=33, ny=29),
            W.image(metric="einasto", spin=0.6, halo=(0.2, 0.0), incl=2.2, nx=26, ny=40,
                    precision="mixed")]
    ref = [rt.trace(i) for i in imgs]

    def lean(img):
        outs = rt.alloc_outputs(img)
        return {k: v for k, v in outs.items() if k not in ("ncross", "r_em")}

    say("[parity] intensities without ncross and r_em")
    single = lean(imgs[0])
    rt.rt_trace_image([rt.params_from(imgs[0])], [rt.out_from(single)])
    batch = [lean(imgs[0]), rt.alloc_outputs(imgs[1])]
    rt.rt_trace_image([rt.params_from(i) for i in imgs[:2]], [rt.out_from(o) for o in batch])
    mixed = lean(imgs[2])
    rt.rt_trace_image([rt.params_from(imgs[2])], [rt.out_from(mixed)])
    torch.cuda.synchronize()
    for got, want in ((single, ref[0]), (batch[0], ref[0]), (batch[1], ref[1]), (mixed, ref[2])):
        for k in got:
            assert np.array_equal(got[k].cpu().numpy(), want[k].cpu().numpy(), equal_nan=True), k


def test_launch_config_does_not_change_results(rt):
    """Chunk size, tile shape and order (screen or ring-out) and occupancy cap
    only move rays between lanes."""
    import torch
    img = W.image(metric="cnfw", spin=0.9, halo=(0.03, 7.0), incl=1.2, nx=45, ny=38)
    rt.rt_set_launch_config(reset=True)
    ref = rt.trace(img)
    torch.cuda.synchronize()
    try:
        screen = rt.RT_ORDER_SCREEN
        for cfg in (dict(chunk=1, order=screen), dict(chunk=7, tile_w=8, tile_h=8, order=screen),
                    dict(chunk=256, tile_w=16, tile_h=4, blocks_per_cu=1, order=screen),
                    dict(chunk=33, tile_w=50, tile_h=50, order=screen),
                    dict(tile_w=3, tile_h=5), dict(tile_w=64, tile_h=1, blocks_per_cu=1),
                    dict(tile_w=50, tile_h=50)):
            say(f"[parity] launch config {cfg}")
            rt.rt_set_launch_config(**cfg)
            got = rt.trace(img)
            torch.cuda.synchronize()
            for k in ref:
                assert np.array_equal(ref[k].cpu().numpy(), got[k].cpu().numpy(),
                                      equal_nan=True), (cfg, k)
    finally:
        rt.rt_set_launch_config(reset=True)


def test_large_mixed_batch_equals_single_images(rt):
    """130 small images of all metrics: two batched launches (128 + 2 images),
    each image bit-identical to its own single-image trace."""
    import torch
    from conftest import oracle_einasto_extremal_spin
    base = W.batch_64(oracle_einasto_extremal_spin, seed=9, n_images=64)
    imgs = []
    for j in range(130):
        b = dict(base[j % 64])
        b.update(nx=5 + j % 7, ny=4 + j % 5)
        imgs.append(b)
    say("[parity] 130-image batch")
    many = rt.trace_many(imgs)
    singles = [rt.trace(i) for i in imgs]
    torch.cuda.synchronize()
    for j, (a, b) in enumerate(zip(singles, many)):
        for k in a:
            assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy(), equal_nan=True), (j, k)


def test_batch_64_workload_sampled(rt, orc, batch64):
    """The benchmark's 64-image batch (14 M rays, all three metrics, Einasto
    halos up to lambda_E = 0.3) traced as bench.py traces it -- one persistent
    launch under the autotuned launch configuration -- on 24 seeded pixels of
    every image against the oracle.  The library's own draw of the workload
    (its extremal spin deciding the Einasto rejections) is the same list."""
    import torch
    from paper_2605_05635_amd import autotune
    assert W.batch_64(rt.einasto_extremal_spin) == batch64
    say("[parity] batch_64: autotune, one launch, 24 pixels per image")
    best = autotune.tune(batch64, log=say)
    try:
        many = rt.trace_many(batch64)
        torch.cuda.synchronize()
    finally:
        rt.rt_set_launch_config(reset=True)
    say(f"[parity] batch_64 traced with {best}")
    for j, (img, outs) in enumerate(zip(batch64, many)):
        idx = W.random_pixels(img["nx"], img["ny"], 24, 500 + j)
        g = gpu_to_numpy(outs, idx)
        o = orc.trace_pixels(img, idx)
        bad = compare(g, o)
        assert not bad, (j, img["metric"], bad)


def test_batch_parity_with_oracle(rt, orc):
    """A batch of three metrics against the oracle, every pixel."""
    import torch
    imgs = [W.image(metric="kerr", spin=0.99, incl=1.4, nx=23, ny=19),
            W.image(metric="einasto", spin=0.7, halo=(0.2, 0.0), incl=0.5, nx=31, ny=17),
            W.image(metric="cnfw", spin=0.3, halo=(0.05, 5.0), incl=2.7, nx=19, ny=29)]
    many = rt.trace_many(imgs)
    torch.cuda.synchronize()
    for img, outs in zip(imgs, many):
        g = gpu_to_numpy(outs)
        o = orc.trace_pixels(img)
        assert_parity(g, o)


def test_visibility_gaussian_closed_form(rt):
    """|V|/|V(0,0)| of a Gaussian image is exp(-2 pi^2 s^2 q^2) (Sec. 6.4)."""
    import torch
    img = W.image(nx=181, ny=157, x_min=-12, x_max=12, y_min=-12, y_max=12)
    X = img["x_min"] + (np.arange(img["nx"]) + 0.5) * 24 / img["nx"]
    Y = img["y_min"] + (np.arange(img["ny"]) + 0.5) * 24 / img["ny"]
    s = 1.4
    I = np.exp(-((X[None, :] - 0.6) ** 2 + (Y[:, None] + 0.3) ** 2) / (2 * s * s))
    uv = W.uv_points(5, 2000)
    amp = rt.visibility(img, torch.tensor(I, device="cuda"), uv).cpu().numpy()
    q2 = (uv ** 2).sum(1)
    assert np.allclose(amp, np.exp(-2 * np.pi ** 2 * s * s * q2), rtol=0, atol=1e-10)


def test_visibility_of_traced_image_matches_oracle(rt, orc):
    import torch
    img = W.image(metric="einasto", spin=0.9, halo=(0.14, 0.0), incl=math.radians(60),
                  nx=96, ny=80, x_min=-10, x_max=10, y_min=-10, y_max=10)
    outs = rt.trace(img)
    uv = W.uv_points(6, 300)
    amp = rt.visibility(img, outs["intensity"], uv).cpu().numpy()
    torch.cuda.synchronize()
    I = outs["intensity"].cpu().numpy()
    want = orc.visibility_amplitude(img, I, uv)
    assert np.allclose(amp, want, rtol=1e-11, atol=1e-13)
    # and against the oracle's own traced image, to the trace parity bar
    o = orc.trace_image(img)
    want2 = orc.visibility_amplitude(img, o["intensity"], uv)
    assert np.allclose(amp, want2, rtol=1e-6, atol=1e-9)
