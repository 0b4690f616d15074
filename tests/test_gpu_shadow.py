"""The shadow-boundary search (rt_shadow_boundary, Sec. 4.1, eqs. (78)-(79))
on the GPU against the oracle's plain bisection in b along each direction, and
against the exact finite-distance Kerr critical curve.

Tolerance.  The GPU narrows its bracket by multisection, the oracle by
bisection: different sample points, the same transition.  Each final bracket
holds the transition of its own traced flow and is at most its b_tol wide;
the two flows are the same discrete algorithm and differ only in rounding,
which moves the fate of a ray only within about 1e-14 of the transition.  So
the two midpoints differ by at most (b_tol_gpu + b_tol_oracle)/2, held here to
b_tol_gpu + b_tol_oracle.  Against the exact Kerr curve the integrated flow's
transition lies within ~3e-8 relative (rtol = atol = 1e-8): held to 2e-7, as
the oracle's pins are.
"""
import math
import sys

import numpy as np
import pytest

from paper_2605_05635_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_B = 1e-9     # the GPU search's bracket width
TOL_ORC = 1e-9   # the oracle bisection's


@pytest.fixture(scope="module")
def rt():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_2605_05635_amd import rt as mod
    return mod


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dirs_of(psi):
    psi = np.asarray(psi, dtype=np.float64)
    return np.stack([np.cos(psi), np.sin(psi)], axis=1)


FIG3 = dict(spin=0.5, incl=math.radians(60.0))   # the parameters of the paper's shadow figure
CASES = [
    ("kerr", W.image(metric="kerr", **FIG3)),
    ("einasto", W.image(metric="einasto", halo=(0.3, 0.0), **FIG3)),
    ("cnfw", W.image(metric="cnfw", halo=(0.02, 10.0), **FIG3)),
    ("cnfw-bench", W.cnfw_1024()),
]


@pytest.mark.parametrize("label,img", CASES)
def test_boundary_matches_oracle(rt, orc, label, img):
    import torch
    psi = np.linspace(0.0, 2.0 * np.pi, 24, endpoint=False) + 0.05
    d = dirs_of(psi)
    say(f"[shadow] {label}: 24 directions, b in [2, 9], b_tol {TOL_B}")
    out, st = rt.shadow_boundary(img, d, 2.0, 9.0, TOL_B)
    torch.cuda.synchronize()
    out, st = out.cpu().numpy(), st.cpu().numpy()
    lo, hi, ok = orc.shadow_boundary(img, d, 2.0, 9.0, TOL_ORC)
    assert np.all(st == 0) and ok.all()
    assert np.all(out[:, 1] - out[:, 0] <= TOL_B) and np.all(out[:, 1] > out[:, 0])
    mid_g, mid_o = out.mean(axis=1), 0.5 * (lo + hi)
    assert np.abs(mid_g - mid_o).max() <= TOL_B + TOL_ORC, np.abs(mid_g - mid_o).max()


def test_kerr_boundary_against_critical_curve(rt):
    import torch
    from tests.test_oracle_shadow import kerr_critical_point
    img = W.image(metric="kerr", spin=0.9, incl=math.radians(60.0))
    psi = np.array([0.2, 1.3, 2.9, 3.6, 4.9])
    out, st = rt.shadow_boundary(img, dirs_of(psi), 2.0, 9.0, TOL_B)
    torch.cuda.synchronize()
    b = out.cpu().numpy().mean(axis=1)
    assert np.all(st.cpu().numpy() == 0)
    for p, bb in zip(psi, b):
        exact = kerr_critical_point(0.9, math.radians(60.0), img["r_obs"], p)
        assert abs(bb / exact - 1.0) < 2e-7


def test_bad_bracket_and_unnormalised_directions(rt, orc):
    import torch
    img = W.image(metric="cnfw", halo=(0.02, 10.0), **FIG3)
    d = dirs_of([0.4, 2.0, 4.4])
    # b_lo already escapes: reported, bracket left as given
    out, st = rt.shadow_boundary(img, d, 9.0, 12.0, TOL_B)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 1)
    assert np.all(out.cpu().numpy() == np.array([9.0, 12.0]))
    # b_hi still captured
    out, st = rt.shadow_boundary(img, d, 1.0, 2.0, TOL_B)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 1)
    # a direction of length 2 finds half the impact parameter; a bracket
    # already narrower than b_tol is returned as given
    out2, st2 = rt.shadow_boundary(img, 2.0 * d, 1.0, 4.5, TOL_B)
    out1, st1 = rt.shadow_boundary(img, d, 2.0, 9.0, TOL_B)
    torch.cuda.synchronize()
    assert np.all(st2.cpu().numpy() == 0) and np.all(st1.cpu().numpy() == 0)
    assert np.abs(2.0 * out2.cpu().numpy().mean(axis=1) - out1.cpu().numpy().mean(axis=1)).max() < 4 * TOL_B
    lo1, hi1 = (float(v) for v in out1.cpu().numpy()[0])
    out3, st3 = rt.shadow_boundary(img, d[:1], lo1, hi1, 2e-9)
    torch.cuda.synchronize()
    assert st3.cpu().numpy()[0] == 0
    assert np.all(out3.cpu().numpy()[0] == np.array([lo1, hi1]))


def test_many_directions_sampled(rt, orc):
    """The benchmark's launch: 4096 directions of the cored-NFW benchmark
    spacetime at b_tol 1e-10; eight of them against the oracle."""
    import torch
    img = W.cnfw_1024()
    n = 4096
    psi = (np.arange(n) + 0.5) * (2.0 * np.pi / n)
    d = dirs_of(psi)
    say(f"[shadow] cnfw-bench: {n} directions, b_tol 1e-10")
    out, st = rt.shadow_boundary(img, d, 2.0, 9.0, 1e-10)
    torch.cuda.synchronize()
    out, st = out.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0) and np.all(out[:, 1] - out[:, 0] <= 1e-10)
    b = out.mean(axis=1)
    # a closed curve without jumps: neighbouring directions differ by O(dpsi)
    assert np.abs(np.diff(np.r_[b, b[0]])).max() < 0.05
    pick = np.arange(0, n, n // 8) + 17
    lo, hi, ok = orc.shadow_boundary(img, d[pick], 2.0, 9.0, 1e-10)
    assert ok.all() and np.abs(b[pick] - 0.5 * (lo + hi)).max() <= 2e-10


def test_attempt_counts_do_not_change_results(rt):
    import torch
    img = W.image(metric="einasto", halo=(0.3, 0.0), **FIG3)
    d = torch.tensor(dirs_of(np.linspace(0.1, 6.0, 40)), device="cuda")
    p = rt.params_from(img)
    out1 = torch.empty(40, 2, dtype=torch.float64, device="cuda")
    out2 = torch.empty_like(out1)
    st1 = torch.empty(40, dtype=torch.int32, device="cuda")
    st2 = torch.empty_like(st1)
    att = torch.full((40,), -1, dtype=torch.int64, device="cuda")
    rt.rt_shadow_boundary(p, d, 2.0, 9.0, TOL_B, out1, st1)
    rt.rt_shadow_boundary(p, d, 2.0, 9.0, TOL_B, out2, st2, att)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2) and torch.equal(st1, st2)
    passes = math.ceil(math.log(7.0 / TOL_B) / math.log(65.0))
    # every traced ray takes at least a few dozen attempts from R_o = 1000
    assert int(att.min()) >= (64 * passes + 2) * 20


@pytest.mark.parametrize("samples", [32, 16])
def test_fewer_samples_per_direction(rt, orc, samples):
    """Two or four directions per wavefront, 32 or 16 samples each, against the
    oracle's bisection (an odd count of directions leaves a partly filled
    wavefront)."""
    import torch
    img = W.cnfw_1024()
    psi = np.linspace(0.0, 2.0 * np.pi, 13, endpoint=False) + 0.1
    d = dirs_of(psi)
    out, st = rt.shadow_boundary(img, d, 2.0, 9.0, TOL_B, samples=samples)
    torch.cuda.synchronize()
    out, st = out.cpu().numpy(), st.cpu().numpy()
    lo, hi, ok = orc.shadow_boundary(img, d, 2.0, 9.0, TOL_ORC)
    assert np.all(st == 0) and ok.all()
    assert np.all(out[:, 1] - out[:, 0] <= TOL_B)
    assert np.abs(out.mean(axis=1) - 0.5 * (lo + hi)).max() <= TOL_B + TOL_ORC
    # the same transition as with 64 samples
    out64, _ = rt.shadow_boundary(img, d, 2.0, 9.0, TOL_B)
    assert np.abs(out.mean(axis=1) - out64.cpu().numpy().mean(axis=1)).max() <= 2 * TOL_B
    # a bracket without the transition in one group only
    out2, st2 = rt.shadow_boundary(img, np.concatenate([d[:1], 3.0 * d[1:2]]), 2.0, 9.0, TOL_B,
                                   samples=samples)
    torch.cuda.synchronize()
    assert st2.cpu().numpy().tolist() == [0, 1]


def test_sample_count_rule(rt):
    """The library's sample count: the largest of 64, 32, 16 whose n S rays fit
    one wavefront per SIMD of the device, else 16."""
    import torch
    lanes = torch.cuda.get_device_properties(0).multi_processor_count * 4 * 64
    for n in (1, lanes // 64, lanes // 64 + 1, lanes // 32, lanes // 32 + 1, lanes // 16,
              lanes, 1 << 24):
        want = next((s for s in (64, 32) if n * s <= lanes), 16)
        assert rt.rt_shadow_boundary_samples(n) == want, n
