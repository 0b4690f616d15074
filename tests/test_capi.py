"""Host-side checks of the C ABI library (no GPU needed): it loads, exports every
function include/rt.h declares, its structs match the header's layout, and
invalid arguments are rejected before any device work."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import oracle_einasto_extremal_spin
from paper_2605_05635_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt.h")


@pytest.fixture(scope="module")
def rt():
    from paper_2605_05635_amd import rt as mod
    return mod


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(rt):
    names = declared_functions()
    assert {"rt_trace_image", "rt_transfer_maps", "rt_last_error", "rt_version"} <= set(names)
    lib = C.CDLL(rt.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", rt.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (rt_[a-z0-9_]+)\b", out))
    assert set(names) <= exported


def test_version(rt):
    m = re.search(r"#define RT_VERSION (\d+)", open(HEADER).read())
    assert rt.rt_version() == int(m.group(1))


def test_struct_layout_matches_header(rt, tmp_path):
    """ctypes mirrors of rt_image_params / rt_image_out have the C layout."""
    fields_p = [f for f, _ in rt.rt_image_params._fields_]
    fields_o = [f for f, _ in rt.rt_image_out._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "rt.h"', "int main(void){",
           'printf("%zu\\n", sizeof(rt_image_params));',
           'printf("%zu\\n", sizeof(rt_image_out));']
    src += [f'printf("%zu\\n", offsetof(rt_image_params, {f}));' for f in fields_p]
    src += [f'printf("%zu\\n", offsetof(rt_image_out, {f}));' for f in fields_o]
    src += ["return 0;}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)],
                   check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == C.sizeof(rt.rt_image_params)
    assert vals[1] == C.sizeof(rt.rt_image_out)
    offs_p = [getattr(rt.rt_image_params, f).offset for f in fields_p]
    offs_o = [getattr(rt.rt_image_out, f).offset for f in fields_o]
    assert vals[2:] == offs_p + offs_o


def _err(rt, img_or_params, n=None, outs=None):
    p = img_or_params if isinstance(img_or_params, rt.rt_image_params) else rt.params_from(img_or_params)
    with pytest.raises(rt.RTError) as e:
        rt.rt_trace_image([p] if n is None else [p] * n, outs or [rt.rt_image_out()], 0)
    return e.value.code


@pytest.mark.parametrize("change", [
    dict(incl=0.0), dict(incl=math.pi), dict(spin=float("nan")), dict(nx=0), dict(ny=-3),
    dict(rtol=0.0), dict(atol=-1.0), dict(h0=0.0), dict(r_stop_fac=1.0), dict(r_esc_fac=0.5),
    dict(max_attempts=0), dict(x_min=1.0, x_max=1.0), dict(r_obs=15.0),
    dict(metric="einasto", halo=(0.0, 0.0)), dict(metric="cnfw", halo=(0.02, 0.0)),
    dict(metric="cnfw", halo=(-0.1, 10.0)), dict(r_in=25.0),
    # screens of 2^31 pixels or more (pixel indices are 32-bit in the kernels)
    dict(nx=65536, ny=32768), dict(nx=46341, ny=46341), dict(nx=2**31 - 1, ny=2),
])
def test_invalid_arguments_rejected(rt, change):
    assert _err(rt, W.image(**change)) == rt.RT_ERR_ARG
    assert rt.rt_last_error()


def test_bad_enum_and_reserved_fields(rt):
    for field, value in (("metric", 7), ("precision", 5), ("reserved", 1)):
        p = rt.params_from(W.kerr_small())
        setattr(p, field, value)
        assert _err(rt, p) == rt.RT_ERR_ARG


def test_null_pointers_and_counts(rt):
    lib = rt.lib()
    p = rt.params_from(W.kerr_small())
    o = rt.rt_image_out()
    assert lib.rt_trace_image(None, 1, C.byref(o), None) == rt.RT_ERR_ARG
    assert lib.rt_trace_image(C.byref(p), 1, None, None) == rt.RT_ERR_ARG
    assert lib.rt_trace_image(C.byref(p), 0, C.byref(o), None) == rt.RT_ERR_ARG
    assert lib.rt_transfer_maps(C.byref(p), -1, C.byref(o), None) == rt.RT_ERR_ARG
    assert lib.rt_image_setup(C.byref(p), None) == rt.RT_ERR_ARG
    # argument checks come before any device query
    assert lib.rt_shadow_boundary_samples(0) == rt.RT_ERR_ARG
    assert lib.rt_shadow_boundary_samples(-5) == rt.RT_ERR_ARG


def test_no_horizon_beyond_extremal_spin(rt):
    """Einasto lambda_E = 0.3 has extremal spin 0.640 (Sec. 2.2, Fig. 2)."""
    assert _err(rt, W.image(metric="einasto", halo=(0.3, 0.0), spin=0.65)) == rt.RT_ERR_NO_HORIZON
    assert _err(rt, W.image(metric="kerr", spin=1.01)) == rt.RT_ERR_NO_HORIZON
    assert _err(rt, W.image(metric="einasto", halo=(0.5, 0.0), spin=0.0)) == rt.RT_ERR_NO_HORIZON
    # a batch fails as a whole when any image has no horizon
    good, bad = rt.params_from(W.kerr_small()), rt.params_from(W.image(spin=1.2))
    with pytest.raises(rt.RTError) as e:
        rt.rt_trace_image([good, bad], [rt.rt_image_out()] * 2, 0)
    assert e.value.code == rt.RT_ERR_NO_HORIZON and "image 1" in str(e.value)


def test_image_setup_matches_oracle(rt, orc):
    """The library's host setup finds the same outer horizon as the oracle."""
    cases = [(W.kerr_small(), 1e-14), (W.einasto_512(), 1e-14), (W.cnfw_1024(), 1e-14),
             (W.cnfw_adjoint_256(), 1e-14)] + [(b, 1e-14) for b in W.batch_64(oracle_einasto_extremal_spin)[:12]]
    # 1e-4 below the extremal spin Delta is nearly a double root, and rounding
    # noise in Delta moves its zero by ~sqrt(eps) relative
    cases.append((W.image(metric="einasto", halo=(0.3, 0.0), spin=0.6395), 1e-7))
    for img, tol in cases:
        mine = rt.rt_image_setup(rt.params_from(img))
        ref = orc.image_setup(img)
        for k in ("r_plus", "r_stop", "r_esc", "r_in"):
            assert mine[k] == pytest.approx(ref[k], rel=tol, abs=0), (img["metric"], k)


def test_launch_config_roundtrip_and_validation(rt):
    rt.rt_set_launch_config(128, 8, 8, 1, rt.RT_ORDER_SCREEN)
    assert rt.rt_get_launch_config() == dict(chunk=128, tile_w=8, tile_h=8, blocks_per_cu=1,
                                             order=rt.RT_ORDER_SCREEN)
    for bad in (dict(chunk=-1), dict(tile_w=8), dict(tile_h=4), dict(blocks_per_cu=99),
                dict(chunk=70000), dict(order=2), dict(order=-1)):
        with pytest.raises(rt.RTError) as e:
            rt.rt_set_launch_config(**bad)
        assert e.value.code == rt.RT_ERR_ARG
    rt.rt_set_launch_config(reset=True)
    assert rt.rt_get_launch_config() == dict(chunk=0, tile_w=0, tile_h=0, blocks_per_cu=0,
                                             order=rt.RT_ORDER_CENTRE)


def test_autotune_signature_and_cache(tmp_path, monkeypatch):
    from paper_2605_05635_amd import autotune
    monkeypatch.setenv("RT_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    a = [W.kerr_small(), W.cnfw_1024()]
    assert autotune.signature(a) == autotune.signature([dict(x) for x in a])
    assert autotune.signature(a) != autotune.signature(a[::-1])
    autotune._store({"k": {"chunk": 64}})
    assert autotune._load() == {"k": {"chunk": 64}}


def test_visibility_argument_errors(rt):
    lib = rt.lib()
    p = rt.params_from(W.kerr_small())
    assert lib.rt_visibility_dft(None, C.byref(p), None, 10, None, None, None) == rt.RT_ERR_ARG
    assert lib.rt_visibility_dft(C.c_void_p(8), C.byref(p), C.c_void_p(8), 0, C.c_void_p(8),
                                 None, None) == rt.RT_ERR_ARG
    bad = rt.params_from(W.image(nx=0))
    assert lib.rt_visibility_dft(C.c_void_p(8), C.byref(bad), C.c_void_p(8), 5, C.c_void_p(8),
                                 None, None) == rt.RT_ERR_ARG


def test_batch_visibility_layout_and_errors(rt, tmp_path):
    """rt_vis_image has the header's layout; batched and ring calls reject bad
    arguments before any device work."""
    fields = [f for f, _ in rt.rt_vis_image._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "rt.h"', "int main(void){",
           'printf("%zu\\n", sizeof(rt_vis_image));']
    src += [f'printf("%zu\\n", offsetof(rt_vis_image, {f}));' for f in fields]
    src += ["return 0;}"]
    c = tmp_path / "vis.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "vis"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == C.sizeof(rt.rt_vis_image)
    assert vals[1:] == [getattr(rt.rt_vis_image, f).offset for f in fields]
    lib = rt.lib()
    d = C.c_void_p(8)
    good = dict(intensity=8, uv=8, amp=8, vis=None, nx=4, ny=4, K=3, reserved=0, x_min=-1.0,
                x_max=1.0, y_min=-1.0, y_max=1.0)
    for change in (dict(intensity=None), dict(K=0), dict(K=(1 << 22) + 1), dict(nx=0),
                   dict(reserved=1), dict(x_max=-2.0), dict(amp=None), dict(y_min=float("nan"))):
        arr = (rt.rt_vis_image * 2)(rt.rt_vis_image(**good), rt.rt_vis_image(**dict(good, **change)))
        assert lib.rt_visibility_dft_batch(arr, 2, None) == rt.RT_ERR_ARG, change
        assert "image 1" in rt.rt_last_error()
    arr = (rt.rt_vis_image * 1)(rt.rt_vis_image(**good))
    assert lib.rt_visibility_dft_batch(arr, 0, None) == rt.RT_ERR_ARG
    assert lib.rt_visibility_dft_batch(None, 1, None) == rt.RT_ERR_ARG
    p = rt.params_from(W.kerr_small())
    assert lib.rt_visibility_rings(None, C.byref(p), d, 4, 8, d, d, None) == rt.RT_ERR_ARG
    assert lib.rt_visibility_rings(d, C.byref(p), d, 0, 8, d, d, None) == rt.RT_ERR_ARG
    assert lib.rt_visibility_rings(d, C.byref(p), d, 4, 0, d, d, None) == rt.RT_ERR_ARG
    assert lib.rt_visibility_rings(d, C.byref(p), d, 4, 8, None, None, None) == rt.RT_ERR_ARG
    assert lib.rt_visibility_rings(d, C.byref(p), d, 1 << 12, 1 << 11, d, d, None) == rt.RT_ERR_ARG


def test_vjp_argument_errors(rt):
    lib = rt.lib()
    cn = rt.params_from(W.cnfw_adjoint_256())
    kerr = rt.params_from(W.kerr_small())
    d = C.c_void_p(8)
    assert lib.rt_image_vjp(None, d, 0, d, None, None) == rt.RT_ERR_ARG
    assert lib.rt_image_vjp(C.byref(cn), None, 0, d, None, None) == rt.RT_ERR_ARG
    assert lib.rt_image_vjp(C.byref(cn), d, 0, None, None, None) == rt.RT_ERR_ARG
    assert lib.rt_image_vjp(C.byref(cn), d, 7, d, None, None) == rt.RT_ERR_ARG
    assert lib.rt_image_vjp(C.byref(kerr), d, rt.RT_GRAD_DENSITY, d, None, None) == rt.RT_ERR_ARG
    assert "cored-NFW" in rt.rt_last_error()
    bad = rt.params_from(W.image(nx=0))
    assert lib.rt_image_vjp(C.byref(bad), d, 0, d, None, None) == rt.RT_ERR_ARG
    nohz = rt.params_from(W.image(metric="kerr", spin=1.01))
    assert lib.rt_image_vjp(C.byref(nohz), d, 0, d, None, None) == rt.RT_ERR_NO_HORIZON
    assert lib.rt_set_checkpoint_budget(1000) == rt.RT_ERR_ARG
    assert lib.rt_set_checkpoint_budget(16 << 30) == rt.RT_OK
    assert lib.rt_vjp_stats(None) == rt.RT_ERR_ARG


def test_shadow_boundary_argument_errors(rt):
    lib = rt.lib()
    p = rt.params_from(W.kerr_small())
    d = C.c_void_p(8)
    call = lambda params, dirs, n, lo, hi, tol, out, st, s=64: lib.rt_shadow_boundary(
        params, dirs, n, s, lo, hi, tol, out, st, None, None)
    assert call(None, d, 4, 2.0, 9.0, 1e-9, d, d) == rt.RT_ERR_ARG
    assert call(C.byref(p), None, 4, 2.0, 9.0, 1e-9, d, d) == rt.RT_ERR_ARG
    assert call(C.byref(p), d, 4, 2.0, 9.0, 1e-9, None, d) == rt.RT_ERR_ARG
    assert call(C.byref(p), d, 4, 2.0, 9.0, 1e-9, d, None) == rt.RT_ERR_ARG
    assert call(C.byref(p), d, 0, 2.0, 9.0, 1e-9, d, d) == rt.RT_ERR_ARG
    assert call(C.byref(p), d, (1 << 24) + 1, 2.0, 9.0, 1e-9, d, d) == rt.RT_ERR_ARG
    assert call(C.byref(p), d, 4, 0.0, 9.0, 1e-9, d, d) == rt.RT_ERR_ARG
    assert call(C.byref(p), d, 4, 9.0, 2.0, 1e-9, d, d) == rt.RT_ERR_ARG
    assert call(C.byref(p), d, 4, 2.0, float("inf"), 1e-9, d, d) == rt.RT_ERR_ARG
    assert call(C.byref(p), d, 4, 2.0, 9.0, 1e-14, d, d) == rt.RT_ERR_ARG
    assert "b_tol" in rt.rt_last_error()
    assert call(C.byref(p), d, 4, 2.0, 9.0, 1e-9, d, d, 48) == rt.RT_ERR_ARG
    mixed = rt.params_from(W.image(precision="mixed"))
    assert call(C.byref(mixed), d, 4, 2.0, 9.0, 1e-9, d, d) == rt.RT_ERR_ARG
    nohz = rt.params_from(W.image(metric="kerr", spin=1.01))
    assert call(C.byref(nohz), d, 4, 2.0, 9.0, 1e-9, d, d) == rt.RT_ERR_NO_HORIZON


def test_image_diagnostics_argument_errors(rt):
    lib = rt.lib()
    p = rt.params_from(W.kerr_small())
    d = C.c_void_p(8)
    call = lambda I, params, bw, nb, out: lib.rt_image_diagnostics(I, params, bw, nb, out, None, None)
    assert call(None, C.byref(p), 0.1, 10, d) == rt.RT_ERR_ARG
    assert call(d, None, 0.1, 10, d) == rt.RT_ERR_ARG
    assert call(d, C.byref(p), 0.1, 10, None) == rt.RT_ERR_ARG
    assert call(d, C.byref(p), 0.0, 10, d) == rt.RT_ERR_ARG
    assert call(d, C.byref(p), float("nan"), 10, d) == rt.RT_ERR_ARG
    assert call(d, C.byref(p), 0.1, 0, d) == rt.RT_ERR_ARG
    assert call(d, C.byref(p), 0.1, (1 << 20) + 1, d) == rt.RT_ERR_ARG
    bad = rt.params_from(W.image(nx=0))
    assert call(d, C.byref(bad), 0.1, 10, d) == rt.RT_ERR_ARG
    assert "screen" in rt.rt_last_error()


def test_scan_point_layout_and_argument_errors(rt, tmp_path):
    fields = [f for f, _ in rt.rt_scan_point._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "rt.h"', "int main(void){",
           'printf("%zu\\n", sizeof(rt_scan_point));']
    src += [f'printf("%zu\\n", offsetof(rt_scan_point, {f}));' for f in fields]
    src += ["return 0;}"]
    c = tmp_path / "scan.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "scan"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == C.sizeof(rt.rt_scan_point)
    assert vals[1:] == [getattr(rt.rt_scan_point, f).offset for f in fields]
    lib = rt.lib()
    d = C.c_void_p(8)
    assert lib.rt_parameter_scan(None, 4, d, None) == rt.RT_ERR_ARG
    assert lib.rt_parameter_scan(d, 4, None, None) == rt.RT_ERR_ARG
    assert lib.rt_parameter_scan(d, 0, d, None) == rt.RT_ERR_ARG
    assert lib.rt_parameter_scan(d, (1 << 24) + 1, d, None) == rt.RT_ERR_ARG


def test_thick_disc_argument_errors(rt):
    lib = rt.lib()
    p = rt.params_from(W.kerr_small())
    d = C.c_void_p(8)
    good = rt.rt_thick_disc(8.0, 0.2, 0.1)
    o = rt.rt_image_out()
    o.intensity = 8
    assert lib.rt_trace_thick(None, C.byref(good), C.byref(o), None) == rt.RT_ERR_ARG
    assert lib.rt_trace_thick(C.byref(p), None, C.byref(o), None) == rt.RT_ERR_ARG
    for bad in (rt.rt_thick_disc(0.0, 0.2, 0.1), rt.rt_thick_disc(8.0, 0.0, 0.1),
                rt.rt_thick_disc(8.0, 0.2, -0.1), rt.rt_thick_disc(float("nan"), 0.2, 0.1)):
        assert lib.rt_trace_thick(C.byref(p), C.byref(bad), C.byref(o), None) == rt.RT_ERR_ARG
    none = rt.rt_image_out()
    assert lib.rt_trace_thick(C.byref(p), C.byref(good), C.byref(none), None) == rt.RT_ERR_ARG
    o2 = rt.rt_image_out()
    o2.intensity, o2.g_em = 8, 8
    assert lib.rt_trace_thick(C.byref(p), C.byref(good), C.byref(o2), None) == rt.RT_ERR_ARG
    mixed = rt.params_from(W.image(precision="mixed"))
    assert lib.rt_trace_thick(C.byref(mixed), C.byref(good), C.byref(o), None) == rt.RT_ERR_ARG


def test_screen_point_and_refinement_argument_errors(rt):
    lib = rt.lib()
    p = rt.params_from(W.kerr_small())
    d = C.c_void_p(8)
    o = rt.rt_image_out()
    o.ncross, o.r_em = 8, 8
    E = rt.RT_ERR_ARG
    assert lib.rt_trace_points(None, d, 4, C.byref(o), None) == E
    assert lib.rt_trace_points(C.byref(p), None, 4, C.byref(o), None) == E
    assert lib.rt_trace_points(C.byref(p), d, 4, None, None) == E
    for n in (0, -1, 2**31):
        assert lib.rt_trace_points(C.byref(p), d, n, C.byref(o), None) == E
    red = rt.rt_image_out()
    red.ncross, red.r_em, red.intensity, red.reduce = 8, 8, 8, 8
    assert lib.rt_trace_points(C.byref(p), d, 4, C.byref(red), None) == E
    em = rt.rt_image_out()
    em.intensity = 8                       # emission without ncross and r_em
    assert lib.rt_trace_points(C.byref(p), d, 4, C.byref(em), None) == E
    mixed = rt.params_from(W.image(precision="mixed"))
    assert lib.rt_trace_points(C.byref(mixed), d, 4, C.byref(o), None) == E
    for sub, mx, xy in ((0, 4, d), (17, 4, d), (2, -1, d), (2, 4, None)):
        assert lib.rt_refine_points(C.byref(p), d, d, sub, mx, xy, None, d, None) == E
    assert lib.rt_refine_points(C.byref(p), None, d, 2, 4, d, None, d, None) == E
    assert lib.rt_refine_points(C.byref(p), d, d, 2, 4, d, None, None, None) == E
    assert lib.rt_refine_points(None, d, d, 2, 4, d, None, d, None) == E


def test_image_setup_repeats_and_interleaves(rt):
    """The host keeps the horizons of recent spacetimes: repeated and
    interleaved set-ups (more spacetimes than it keeps) give the first
    call's values bit for bit."""
    lib = rt.lib()
    imgs = [W.image(metric=m, spin=float(s), halo=h)
            for s in np.linspace(0.05, 0.95, 50)
            for m, h in (("kerr", (0.0, 0.0)), ("einasto", (0.2, 0.0)), ("cnfw", (0.02, 10.0)))]
    def setup(img):
        buf = (C.c_double * 4)()
        rc = lib.rt_image_setup(C.byref(rt.params_from(img)), buf)
        assert rc in (rt.RT_OK, rt.RT_ERR_NO_HORIZON)
        return rc, list(buf) if rc == rt.RT_OK else None

    first = [setup(img) for img in imgs]
    assert sum(rc == rt.RT_OK for rc, _ in first) >= 120
    for rep in range(2):
        for img, want in zip(imgs[::-1] if rep else imgs, first[::-1] if rep else first):
            assert setup(img) == want
    # beyond the extremal spin: no horizon, also when asked again
    over = rt.params_from(W.image(spin=1.2))
    for _ in range(2):
        assert lib.rt_image_setup(C.byref(over), (C.c_double * 4)()) == rt.RT_ERR_NO_HORIZON
