"""The mixed-precision trace (precision RT_MIXED) on the GPU.

What must hold exactly: a ray traced again in binary64 (two crossings, or the
step budget) has outputs bit-identical to the binary64 trace of that pixel;
the mixed image is deterministic; in a batch, each image equals its own
single-image trace.  What is measured and bounded: the difference of the mixed
image from the binary64 one.  The bulk integrates at max(tol, 1e-6) in
binary32 with a compensated state, so its crossing radii differ from binary64
ones at the level the looser tolerance allows (MIX_R_P99 M at the 99th
percentile) and crossing counts differ only for rays that graze a crossing
(at most MIX_NC_FRAC of the pixels).  The same bounds hold against the
binary64 oracle: every pixel of three screens and 1500 seeded pixels of the
1024x1024 benchmark screen; there the rays traced again in binary64 meet the
binary64 parity bar.
"""
import math
import sys

import numpy as np
import pytest

from paper_2605_05635_amd import workloads as W
from parity_util import compare, gpu_to_numpy

pytestmark = pytest.mark.gpu

# Bounds about 2.5-6 times the measured values (MI355X: p99 |dI|/max I at most
# 1.6e-6, p99 |dR_em| at most 7.3e-5 M, at most 2 of 23,040 counts differing),
# the same against the GPU's binary64 trace and against the oracle.
MIX_R_P99 = 2e-4      # p99 of |dR_em| [M] over the recorded crossings of equal pixels
MIX_I_P99 = 4e-6      # p99 of |dI| / max I over pixels with equal count and status
MIX_NC_FRAC = 5e-4    # pixels whose crossing count (or status) differs
ORC_I_P99, ORC_R_P99, ORC_NC_FRAC = MIX_I_P99, MIX_R_P99, MIX_NC_FRAC


@pytest.fixture(scope="module")
def rt():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_2605_05635_amd import rt as mod
    return mod


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def np_outs(outs):
    return {k: v.cpu().numpy() for k, v in outs.items()}


def report(g64, gmx):
    nc64, ncm = g64["ncross"].ravel(), gmx["ncross"].ravel()
    st64, stm = g64["status"].ravel(), gmx["status"].ravel()
    same = (nc64 == ncm) & (st64 == stm)
    I64, Im = g64["intensity"].ravel(), gmx["intensity"].ravel()
    dI = np.abs(Im - I64) / max(np.abs(I64).max(), 1e-300)
    r64, rm = g64["r_em"].reshape(3, -1), gmx["r_em"].reshape(3, -1)
    have = (np.arange(3)[:, None] < np.minimum(nc64, 3)[None, :]) & same[None, :]
    dR = np.abs(rm - r64)[have]
    rep = dict(pixels=nc64.size, ncross_mismatch=int((nc64 != ncm).sum()),
               status_mismatch=int((st64 != stm).sum()),
               dI_p50=float(np.quantile(dI[same], 0.5)), dI_p99=float(np.quantile(dI[same], 0.99)),
               dI_max=float(dI[same].max()),
               dR_p99=float(np.quantile(dR, 0.99)) if dR.size else 0.0,
               dR_max=float(dR.max()) if dR.size else 0.0)
    return rep, same


@pytest.mark.parametrize("img,label", [
    (W.image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=math.radians(163), nx=160,
             ny=144), "cnfw-163"),
    (W.image(metric="einasto", spin=0.9, halo=(0.14, 0.0), incl=math.radians(60), nx=128,
             ny=96), "einasto-60"),
    (W.image(metric="kerr", spin=0.5, incl=math.radians(17), nx=96, ny=96, x_min=-12, x_max=12,
             y_min=-12, y_max=12), "kerr-17"),
], ids=["cnfw-163", "einasto-60", "kerr-17"])
def test_mixed_against_binary64(rt, img, label):
    import torch
    say(f"[mixed] {label} {img['nx']}x{img['ny']}")
    g64 = np_outs(rt.trace(img))
    mixed = dict(img, precision="mixed")
    gm = np_outs(rt.trace(mixed))
    stats = rt.rt_mixed_stats()
    rt.rt_set_launch_config(chunk=3, tile_w=16, tile_h=2, order=rt.RT_ORDER_SCREEN)
    try:
        gm2 = np_outs(rt.trace(mixed))
    finally:
        rt.rt_set_launch_config(reset=True)
    torch.cuda.synchronize()
    for k in gm:
        assert np.array_equal(gm[k], gm2[k], equal_nan=True), f"{k} depends on the hand-out"
    rep, same = report(g64, gm)
    say(f"[mixed] {label}: {rep} binary64 {stats['binary64']} (reruns {stats['rerun']})")
    # rays traced again in binary64 equal the binary64 trace exactly
    rerun = gm["ncross"].ravel() >= 2
    assert rerun.sum() <= stats["rerun"]
    for k in ("ncross", "status", "attempts", "intensity"):
        a, b = gm[k].reshape(-1), g64[k].reshape(-1)
        assert np.array_equal(a[rerun], b[rerun]), k
    for k in ("r_em", "phi_em", "t_em", "g_em", "intensity_n"):
        a, b = gm[k].reshape(3, -1)[:, rerun], g64[k].reshape(3, -1)[:, rerun]
        assert np.array_equal(a, b, equal_nan=True), k
    assert rep["ncross_mismatch"] <= MIX_NC_FRAC * rep["pixels"] + 1
    assert rep["status_mismatch"] <= MIX_NC_FRAC * rep["pixels"] + 1
    assert rep["dR_p99"] <= MIX_R_P99
    assert rep["dI_p99"] <= MIX_I_P99
    # every pixel written: no NaN intensity, records NaN exactly beyond the count
    assert np.all(np.isfinite(gm["intensity"]))
    nrec = np.minimum(gm["ncross"].ravel(), 3)
    r = gm["r_em"].reshape(3, -1)
    for j in range(3):
        assert np.all(np.isfinite(r[j][nrec > j])) and np.all(np.isnan(r[j][nrec <= j]))


def test_mixed_in_batch(rt):
    import torch
    say("[mixed] batch of binary64 and mixed images")
    imgs = [W.image(metric="kerr", spin=0.3, incl=math.radians(40), nx=48, ny=40),
            W.image(metric="cnfw", spin=0.8, halo=(0.03, 9.0), incl=math.radians(120), nx=56,
                    ny=50, precision="mixed"),
            W.image(metric="einasto", spin=0.6, halo=(0.2, 0.0), incl=math.radians(70), nx=40,
                    ny=44),
            W.image(metric="kerr", spin=0.9, incl=math.radians(80), nx=36, ny=30,
                    precision="mixed")]
    many = rt.trace_many(imgs)
    single = [rt.trace(i) for i in imgs]
    torch.cuda.synchronize()
    for a, b in zip(many, single):
        for k in a:
            assert torch.equal(torch.nan_to_num(a[k].double(), nan=-7.0),
                               torch.nan_to_num(b[k].double(), nan=-7.0)), k


@pytest.mark.parametrize("img,label", [
    (W.image(metric="einasto", spin=0.3, halo=(0.3, 0.0), incl=math.radians(30), nx=1, ny=1),
     "one-pixel"),
    (W.image(metric="kerr", spin=0.7, incl=math.radians(40), nx=23, ny=17, x_min=-2, x_max=2,
             y_min=-2, y_max=2), "inside-shadow"),
    (W.image(metric="cnfw", spin=-0.6, halo=(0.05, 5.0), incl=math.radians(120), nx=77, ny=1),
     "one-row-retrograde"),
], ids=["one-pixel", "inside-shadow", "one-row-retrograde"])
def test_mixed_edge_screens(rt, img, label):
    """Degenerate screens run through both passes and agree with binary64 on
    crossing counts and status."""
    import torch
    say(f"[mixed] edge screen {label}")
    g64 = np_outs(rt.trace(img))
    gm = np_outs(rt.trace(dict(img, precision="mixed")))
    torch.cuda.synchronize()
    assert np.array_equal(gm["ncross"], g64["ncross"])
    assert np.array_equal(gm["status"], g64["status"])
    rep, same = report(g64, gm)
    assert rep["dR_max"] <= 1e-3


def oracle_report(g, o):
    """Per-pixel error of the mixed image g (numpy, flattened) against the
    oracle's o on the same pixels."""
    nc_g, nc_o = g["ncross"].astype(np.int64), o["ncross"].astype(np.int64)
    st_g, st_o = g["status"].astype(np.int64), o["status"].astype(np.int64)
    same = (nc_g == nc_o) & (st_g == st_o)
    dI = np.abs(g["intensity"] - o["intensity"]) / max(np.abs(o["intensity"]).max(), 1e-300)
    have = (np.arange(3)[:, None] < np.minimum(nc_o, 3)[None, :]) & same[None, :]
    dR = np.abs(g["r_em"] - o["r_em"])[have]
    return dict(pixels=int(nc_o.size), ncross_mismatch=int((nc_g != nc_o).sum()),
                status_mismatch=int((st_g != st_o).sum()),
                dI_p99=float(np.quantile(dI[same], 0.99)), dI_max=float(dI[same].max()),
                dR_p99=float(np.quantile(dR, 0.99)) if dR.size else 0.0,
                dR_max=float(dR.max()) if dR.size else 0.0), same


def check_against_oracle(g, o, label):
    rep, same = oracle_report(g, o)
    say(f"[mixed vs oracle] {label}: {rep}")
    assert rep["ncross_mismatch"] + rep["status_mismatch"] <= ORC_NC_FRAC * rep["pixels"] + 1
    assert rep["dI_p99"] <= ORC_I_P99
    assert rep["dR_p99"] <= ORC_R_P99
    # the rays the mixed trace finished by a binary64 trace from the screen (two
    # crossings) meet the binary64 parity bar against the oracle
    rerun = (g["ncross"] >= 2) & (o["ncross"] >= 2)
    sub = lambda d: {k: (v[:, rerun] if v.ndim == 2 else v[rerun]) for k, v in d.items()  # noqa: E731
                     if k != "reduce"}
    bad = compare(sub(g), sub(o))
    assert not bad, "\n".join(bad)
    return rep


@pytest.mark.parametrize("img,label", [
    (W.image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=math.radians(163), nx=160,
             ny=144), "cnfw-163"),
    (W.image(metric="einasto", spin=0.9, halo=(0.14, 0.0), incl=math.radians(60), nx=128,
             ny=96), "einasto-60"),
    (W.image(metric="kerr", spin=0.5, incl=math.radians(17), nx=96, ny=96), "kerr-17"),
], ids=["cnfw-163", "einasto-60", "kerr-17"])
def test_mixed_against_oracle_full_screens(rt, orc, img, label):
    """Every pixel of three screens in mixed precision against the binary64
    oracle at the image's tolerance (1e-8)."""
    import torch
    say(f"[mixed vs oracle] {label} {img['nx']}x{img['ny']}, every pixel")
    gm = gpu_to_numpy(rt.trace(dict(img, precision="mixed")))
    torch.cuda.synchronize()
    o = orc.trace_pixels(img)
    check_against_oracle(gm, o, label)


def test_mixed_against_oracle_benchmark_screen(rt, orc):
    """The 1024x1024 cored-NFW screen in mixed precision, launched as bench.py
    launches it, on 1500 seeded pixels against the oracle."""
    import torch
    img = W.cnfw_1024("mixed")
    say("[mixed vs oracle] cnfw 1024x1024 mixed, 1500 seeded pixels")
    outs = rt.trace(img)
    torch.cuda.synchronize()
    idx = W.random_pixels(img["nx"], img["ny"], 1500, 41)
    g = gpu_to_numpy(outs, idx)
    o = orc.trace_pixels(W.cnfw_1024(), idx)
    check_against_oracle(g, o, "cnfw-1024")
