"""The image diagnostics' entry point that allocates nothing
(rt_image_diagnostics_noalloc) against rt_image_diagnostics, through the C
ABI: the same kernels on a file-scope work array instead of stream-ordered
scratch, so the outputs must be identical bit for bit.  Two calls in a row,
the second on a smaller image (the array keeps the first call's contents),
with and without a caller profile buffer; the size limit is an argument
error."""
import math
import sys

import numpy as np
import pytest

from paper_2605_05635_amd import workloads as W

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


def ring_image(img, r0, w, tilt):
    X = img["x_min"] + (np.arange(img["nx"]) + 0.5) * (img["x_max"] - img["x_min"]) / img["nx"]
    Y = img["y_min"] + (np.arange(img["ny"]) + 0.5) * (img["y_max"] - img["y_min"]) / img["ny"]
    rho = np.hypot(X[None, :] - 0.4, Y[:, None] + 0.2)
    I = np.exp(-0.5 * ((rho - r0) / w) ** 2) * (1.0 + tilt * X[None, :] / 10.0)
    I[I < 1e-3] = 0.0
    return I


def both(rt, img, I, bw, n_bins, with_profile):
    import torch
    p = rt.params_from(img)
    dev = torch.tensor(I, dtype=torch.float64, device="cuda")
    out_a = torch.full((rt.RT_DIAG_COUNT,), -7.0, dtype=torch.float64, device="cuda")
    out_b = torch.full_like(out_a, -9.0)
    prof_a = torch.full((n_bins,), -7.0, dtype=torch.float64, device="cuda") if with_profile else None
    prof_b = torch.full((n_bins,), -9.0, dtype=torch.float64, device="cuda") if with_profile else None
    rt.rt_image_diagnostics(dev, p, bw, n_bins, out_a, prof_a)
    rt.rt_image_diagnostics_noalloc(dev, p, bw, n_bins, out_b, prof_b)
    torch.cuda.synchronize()
    a, b = out_a.cpu().numpy(), out_b.cpu().numpy()
    assert np.array_equal(a, b, equal_nan=True), (a, b)
    assert np.isfinite(a).all()
    if with_profile:
        pa, pb = prof_a.cpu().numpy(), prof_b.cpu().numpy()
        assert np.array_equal(pa, pb, equal_nan=True)
    return a


@pytest.mark.parametrize("with_profile", [False, True])
def test_noalloc_matches_allocating_entry(rt, with_profile):
    import torch
    big = W.image(nx=512, ny=384, x_min=-12, x_max=12, y_min=-10, y_max=10)
    small = W.image(nx=97, ny=61, x_min=-9, x_max=11, y_min=-8, y_max=8)
    say(f"[no-alloc] diagnostics 512x384 then 97x61, profile given: {with_profile}")
    a1 = both(rt, big, ring_image(big, 5.0, 0.6, 0.7), 0.05, 300, with_profile)
    a2 = both(rt, small, ring_image(small, 3.0, 0.4, -0.5), 0.1, 90, with_profile)
    assert not np.array_equal(a1, a2)


def test_noalloc_traced_image_and_limits(rt):
    import torch
    img = W.image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=math.radians(60), nx=48,
                  ny=40, x_min=-10, x_max=10, y_min=-10, y_max=10)
    say("[no-alloc] diagnostics of a traced 48x40 cored-NFW image")
    outs = rt.trace(img)
    torch.cuda.synchronize()
    I = outs["intensity"].cpu().numpy()
    both(rt, img, I, 0.2, rt.RT_DIAG_NOALLOC_MAX_BINS, False)
    p = rt.params_from(img)
    out = torch.empty(rt.RT_DIAG_COUNT, dtype=torch.float64, device="cuda")
    with pytest.raises(rt.RTError) as e:
        rt.rt_image_diagnostics_noalloc(outs["intensity"], p, 0.2,
                                        rt.RT_DIAG_NOALLOC_MAX_BINS + 1, out)
    assert e.value.code == rt.RT_ERR_ARG
    # with a caller profile the bin count is not limited by the array
    prof = torch.empty(rt.RT_DIAG_NOALLOC_MAX_BINS + 1, dtype=torch.float64, device="cuda")
    rt.rt_image_diagnostics_noalloc(outs["intensity"], p, 0.2,
                                    rt.RT_DIAG_NOALLOC_MAX_BINS + 1, out, prof)
    torch.cuda.synchronize()
