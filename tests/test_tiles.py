"""The trace kernels' hand-out of screen pixels (rt_ray.h, compiled for the
host): quotient(a, b) = floor(a / b) without an integer division, and the
tile order of a screen, against plain integer arithmetic written out here.

The host build of quotient uses the division for its reciprocal's starting
value, or that value perturbed by 2^-24 relative (worse than the hardware
estimate's 2^-24.4 on gfx950), so the one Newton step and the 1/(2b) margin
the device relies on are exercised on the CPU.
"""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "tiles", "tile_driver.hip")
INC = [os.path.join(ROOT, "include"), os.path.join(ROOT, "paper_2605_05635_amd", "csrc")]
EST = 2.0 ** -24


@pytest.fixture(scope="module", params=[None, EST, -EST], ids=["exact", "est+", "est-"])
def driver(request, tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tiles") / "tile_driver")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17"]
    if request.param is not None:
        cmd += [f"-DRT_HOST_RECIP1_ESTIMATE_ERROR=({request.param!r})"]
    for d in INC:
        cmd += ["-I", d]
    subprocess.run(cmd + [SRC, "-o", exe], check=True, capture_output=True)
    return exe


def run(exe, mode, rows):
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = subprocess.run([exe, mode], input=rows.tobytes(), capture_output=True, check=True).stdout
    return np.frombuffer(out, dtype=np.int64)


def tile_pixel_ref(p, nx, ny, tw, th):
    """The p-th pixel of the tile order, by integer division."""
    band = th * nx
    r = p // band
    h = th if (r + 1) * th <= ny else ny - r * th
    q = p - r * band
    full = nx // tw
    j = q // (tw * h)
    if j < full:
        off = q - j * tw * h
        return (r * th + off // tw) * nx + j * tw + off % tw
    w = nx - full * tw
    off = q - full * tw * h
    return (r * th + off // w) * nx + full * tw + off % w


def test_quotient(driver):
    rng = np.random.default_rng(0)
    top = 2 ** 31 - 1
    b = np.concatenate([rng.integers(1, top, 4000), rng.integers(1, 2 ** 16, 4000),
                        2 ** np.arange(31), 2 ** np.arange(1, 31) - 1, [1, 2, 3, 7, top]])
    a = []
    for bb in b:
        k = int(rng.integers(0, top // bb + 1))
        a += [min(k * bb, top), max(k * bb - 1, 0), min(k * bb + bb - 1, top),
              int(rng.integers(0, top))]
    b = np.repeat(b, 4)
    a = np.array(a, dtype=np.int64)
    got = run(driver, "quotient", np.stack([a, b], axis=1))
    assert np.array_equal(got, a // b)


@pytest.mark.parametrize("nx,ny,tw,th", [
    (64, 64, 8, 8), (97, 61, 8, 8), (83, 71, 16, 4), (1, 77, 8, 8), (129, 1, 8, 8),
    (13, 11, 13, 1), (31, 29, 5, 7), (768, 768, 8, 8), (300, 7, 32, 32),
])
def test_tile_order_is_the_bijection(driver, nx, ny, tw, th):
    n = nx * ny
    p = np.arange(n)
    rows = np.stack([p, np.full(n, nx), np.full(n, ny), np.full(n, tw), np.full(n, th)], axis=1)
    got = run(driver, "tile", rows).reshape(n, 2)
    ref = np.array([tile_pixel_ref(int(k), nx, ny, tw, th) for k in p])
    for j in range(2):   # integer division, quotient()
        assert np.array_equal(got[:, j], ref)
        assert np.array_equal(np.sort(got[:, j]), p)


def test_tile_order_on_the_largest_screens(driver):
    rng = np.random.default_rng(1)
    rows, ref = [], []
    # (the launch clamps the tile to the screen: tw <= nx, th <= ny)
    for nx, ny, tw, th in ((46340, 46340, 8, 8), (2 ** 16 - 1, 32767, 7, 9),
                           (1, 2 ** 31 - 1, 1, 8), (2 ** 31 - 1, 1, 8, 1)):
        for k in np.concatenate([rng.integers(0, nx * ny, 2000), [0, nx * ny - 1]]):
            rows.append([int(k), nx, ny, tw, th])
            ref.append(tile_pixel_ref(int(k), nx, ny, tw, th))
    got = run(driver, "tile", np.array(rows)).reshape(len(rows), 2)
    assert np.array_equal(got[:, 0], np.array(ref)) and np.array_equal(got[:, 1], np.array(ref))
