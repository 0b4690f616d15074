"""The oracle's screen refinement near the lensing-band boundaries (Sec. 4,
bands of Sec. 4.2): its vectorised marking against the definition written as
loops over each pixel's 4-neighbours, the subpixel centres against the pixel
geometry, and its point trace against its pixel trace at pixel centres."""
import numpy as np

from oracle import oracle as O
from paper_2605_05635_amd import workloads as W


def marked_by_loops(nc, st):
    ny, nx = nc.shape
    out = []
    for iy in range(ny):
        for ix in range(nx):
            for jx, jy in ((ix - 1, iy), (ix + 1, iy), (ix, iy - 1), (ix, iy + 1)):
                if 0 <= jx < nx and 0 <= jy < ny and (nc[jy, jx] != nc[iy, ix] or
                                                      st[jy, jx] != st[iy, ix]):
                    out.append(iy * nx + ix)
                    break
    return np.array(out, dtype=np.int64)


def test_marking_matches_the_definition():
    rng = np.random.default_rng(3)
    for nx, ny in ((1, 1), (1, 9), (7, 1), (13, 11), (32, 17)):
        img = W.image(nx=nx, ny=ny)
        for _ in range(3):
            # blocky maps (runs of equal values), so both marked and unmarked pixels occur
            nc = np.repeat(np.repeat(rng.integers(0, 3, ((ny + 2) // 3, (nx + 2) // 3)), 3, 0), 3, 1)[:ny, :nx]
            st = np.repeat(np.repeat(rng.integers(1, 3, ((ny + 3) // 4, (nx + 3) // 4)), 4, 0), 4, 1)[:ny, :nx]
            pix, xy = O.refine_points(img, nc.astype(np.uint8), st.astype(np.uint8), 2)
            assert np.array_equal(pix, marked_by_loops(nc, st))
            assert xy.shape == (4 * len(pix), 2)


def test_uniform_map_marks_nothing():
    img = W.image(nx=9, ny=5)
    pix, xy = O.refine_points(img, np.ones((5, 9), np.uint8), np.full((5, 9), 2, np.uint8), 3)
    assert len(pix) == 0 and xy.shape == (0, 2)


def test_subpixel_centres():
    img = W.image(nx=6, ny=4, x_min=-3.0, x_max=9.0, y_min=-2.0, y_max=6.0)
    nc = np.zeros((4, 6), np.uint8)
    nc[:, 3:] = 1                                    # a vertical band edge between columns 2 and 3
    st = np.ones((4, 6), np.uint8)
    pix1, xy1 = O.refine_points(img, nc, st, 1)
    assert set((pix1 % 6).tolist()) == {2, 3}
    X, Y = O.pixel_xy(img, pix1)
    assert np.array_equal(xy1[:, 0], X) and np.array_equal(xy1[:, 1], Y)   # sub = 1: the centres
    for sub in (2, 3, 5):
        pix, xy = O.refine_points(img, nc, st, sub)
        assert np.array_equal(pix, pix1)
        c = xy.reshape(len(pix), sub * sub, 2)
        # the subpixel centres average to the pixel centre and lie inside the pixel,
        # 1/sub of a pixel apart
        assert np.allclose(c.mean(axis=1), xy1, rtol=0, atol=1e-13)
        ix, iy = pix % 6, pix // 6
        assert np.all(c[:, :, 0] > (-3.0 + 2.0 * ix)[:, None]) and np.all(c[:, :, 0] < (-1.0 + 2.0 * ix)[:, None])
        assert np.all(c[:, :, 1] > (-2.0 + 2.0 * iy)[:, None]) and np.all(c[:, :, 1] < (2.0 * iy)[:, None])
        assert np.allclose(np.diff(c[:, :sub, 0], axis=1), 2.0 / sub)          # first row, along X
        assert np.allclose(c[:, sub, 1] - c[:, 0, 1], 2.0 / sub)               # next row, along Y


def test_point_trace_equals_pixel_trace_at_centres():
    img = W.image(nx=6, ny=5)
    idx = np.arange(30)
    X, Y = O.pixel_xy(img, idx)
    a = O.trace_points(img, np.stack([X, Y], axis=1), threads=4)
    b = O.trace_pixels(img, idx, threads=4)
    assert np.all(a["E"] > 0.0)
    for k in ("ncross", "status", "attempts", "intensity"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("r_em", "phi_em", "t_em", "g_em", "i_n"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
