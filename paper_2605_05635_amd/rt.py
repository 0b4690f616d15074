"""Python binding of the C ABI in include/rt.h (argument marshalling only).

Every entry point of the library has a function of the same name here that
takes ctypes structures (or workload dicts) and device tensors, and calls the
shared library; the computation happens in the gfx950 kernels.  PyTorch is
used only for device buffers and the current stream.

If the shared library is missing this module raises ImportError: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgeodesic_rt.so")

RT_KERR, RT_EINASTO, RT_CNFW = 0, 1, 2
RT_FP64, RT_MIXED = 0, 1
RT_OK, RT_ERR_ARG, RT_ERR_NO_HORIZON, RT_ERR_HIP, RT_ERR_ALLOC = 0, -1, -2, -3, -4
RT_RAY_CAPTURED, RT_RAY_ESCAPED, RT_RAY_STEP_LIMIT, RT_RAY_NONFINITE = 1, 2, 3, 4
RT_GRAD_NATIVE, RT_GRAD_DENSITY = 0, 1
RT_ORDER_CENTRE, RT_ORDER_SCREEN = 0, 1
METRIC_ID = {"kerr": RT_KERR, "einasto": RT_EINASTO, "cnfw": RT_CNFW}
PRECISION_ID = {"fp64": RT_FP64, "mixed": RT_MIXED}


class rt_image_params(C.Structure):
    _fields_ = [
        ("metric", C.c_int32), ("precision", C.c_int32),
        ("spin", C.c_double), ("halo", C.c_double * 2),
        ("incl", C.c_double), ("r_obs", C.c_double),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("x_min", C.c_double), ("x_max", C.c_double),
        ("y_min", C.c_double), ("y_max", C.c_double),
        ("rtol", C.c_double), ("atol", C.c_double),
        ("r_stop_fac", C.c_double), ("r_esc_fac", C.c_double),
        ("r_in", C.c_double), ("r_out", C.c_double), ("emis_pow", C.c_double),
        ("sigma_in", C.c_double), ("sigma_out", C.c_double), ("h0", C.c_double),
        ("max_attempts", C.c_int32), ("reserved", C.c_int32),
    ]


class rt_image_out(C.Structure):
    _fields_ = [
        ("ncross", C.c_void_p), ("status", C.c_void_p),
        ("r_em", C.c_void_p), ("phi_em", C.c_void_p), ("t_em", C.c_void_p),
        ("g_em", C.c_void_p), ("intensity", C.c_void_p), ("intensity_n", C.c_void_p),
        ("attempts", C.c_void_p), ("reduce", C.c_void_p),
    ]


class rt_launch_config(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("order", C.c_int32)]


class rt_thick_disc(C.Structure):
    _fields_ = [("r_scale", C.c_double), ("h0", C.c_double), ("h_slope", C.c_double)]


class rt_scan_point(C.Structure):
    _fields_ = [("metric", C.c_int32), ("reserved", C.c_int32), ("spin", C.c_double),
                ("halo", C.c_double * 2), ("theta", C.c_double)]


class rt_vis_image(C.Structure):
    _fields_ = [("intensity", C.c_void_p), ("uv", C.c_void_p), ("amp", C.c_void_p),
                ("vis", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32), ("K", C.c_int32),
                ("reserved", C.c_int32), ("x_min", C.c_double), ("x_max", C.c_double),
                ("y_min", C.c_double), ("y_max", C.c_double)]


class RTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rt error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2605_05635_amd.build` "
            "(there is no non-GPU fallback)")
    lib = C.CDLL(LIB_PATH)
    P, O = C.POINTER(rt_image_params), C.POINTER(rt_image_out)
    for name in ("rt_trace_image", "rt_transfer_maps"):
        f = getattr(lib, name)
        f.argtypes = [P, C.c_int32, O, C.c_void_p]
        f.restype = C.c_int
    lib.rt_image_setup.argtypes = [P, C.POINTER(C.c_double)]
    lib.rt_image_setup.restype = C.c_int
    lib.rt_visibility_dft.argtypes = [C.c_void_p, C.POINTER(rt_image_params), C.c_void_p,
                                      C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.rt_visibility_dft.restype = C.c_int
    lib.rt_visibility_dft_batch.argtypes = [C.POINTER(rt_vis_image), C.c_int32, C.c_void_p]
    lib.rt_visibility_dft_batch.restype = C.c_int
    lib.rt_visibility_rings.argtypes = [C.c_void_p, C.POINTER(rt_image_params), C.c_void_p,
                                        C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p]
    lib.rt_visibility_rings.restype = C.c_int
    lib.rt_trace_points.argtypes = [P, C.c_void_p, C.c_int64, O, C.c_void_p]
    lib.rt_trace_points.restype = C.c_int
    lib.rt_refine_points.argtypes = [P, C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]
    lib.rt_refine_points.restype = C.c_int
    lib.rt_trace_thick.argtypes = [P, C.POINTER(rt_thick_disc), O, C.c_void_p]
    lib.rt_trace_thick.restype = C.c_int
    lib.rt_parameter_scan.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    lib.rt_parameter_scan.restype = C.c_int
    lib.rt_image_diagnostics.argtypes = [C.c_void_p, P, C.c_double, C.c_int32, C.c_void_p,
                                         C.c_void_p, C.c_void_p]
    lib.rt_image_diagnostics.restype = C.c_int
    lib.rt_relative_deviation.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                          C.c_void_p]
    lib.rt_relative_deviation.restype = C.c_int
    lib.rt_image_diagnostics_noalloc.argtypes = lib.rt_image_diagnostics.argtypes
    lib.rt_image_diagnostics_noalloc.restype = C.c_int
    lib.rt_shadow_boundary.argtypes = [P, C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                       C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.rt_shadow_boundary.restype = C.c_int
    lib.rt_shadow_boundary_samples.argtypes = [C.c_int32]
    lib.rt_shadow_boundary_samples.restype = C.c_int
    lib.rt_set_launch_config.argtypes = [C.POINTER(rt_launch_config)]
    lib.rt_set_launch_config.restype = C.c_int
    lib.rt_get_launch_config.argtypes = [C.POINTER(rt_launch_config)]
    lib.rt_get_launch_config.restype = C.c_int
    lib.rt_set_kernel_timing.argtypes = [C.c_void_p, C.c_void_p]
    lib.rt_set_kernel_timing.restype = C.c_int
    lib.rt_set_split_timing.argtypes = [C.c_void_p]
    lib.rt_set_split_timing.restype = C.c_int
    lib.rt_image_vjp.argtypes = [P, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.rt_image_vjp.restype = C.c_int
    lib.rt_mixed_stats.argtypes = [C.POINTER(C.c_int64)]
    lib.rt_mixed_stats.restype = C.c_int
    lib.rt_set_checkpoint_budget.argtypes = [C.c_int64]
    lib.rt_set_checkpoint_budget.restype = C.c_int
    lib.rt_vjp_stats.argtypes = [C.POINTER(C.c_int64)]
    lib.rt_vjp_stats.restype = C.c_int
    lib.rt_last_error.argtypes = []
    lib.rt_last_error.restype = C.c_char_p
    lib.rt_version.argtypes = []
    lib.rt_version.restype = C.c_int
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc: int) -> None:
    if rc != RT_OK:
        raise RTError(rc, _lib.rt_last_error().decode())


def params_from(img: dict) -> rt_image_params:
    """rt_image_params of a workload dict (paper_2605_05635_amd.workloads)."""
    p = rt_image_params()
    p.metric = METRIC_ID[img["metric"]]
    p.precision = PRECISION_ID[img.get("precision", "fp64")]
    p.spin = img["spin"]
    p.halo[0], p.halo[1] = img["halo"]
    for k in ("incl", "r_obs", "x_min", "x_max", "y_min", "y_max", "rtol", "atol",
              "r_stop_fac", "r_esc_fac", "r_in", "r_out", "emis_pow", "sigma_in",
              "sigma_out", "h0"):
        setattr(p, k, float(img[k]))
    p.nx, p.ny = int(img["nx"]), int(img["ny"])
    p.max_attempts = int(img["max_attempts"])
    p.reserved = 0
    return p


def out_from(tensors: dict) -> rt_image_out:
    o = rt_image_out()
    for name, _ in rt_image_out._fields_:
        t = tensors.get(name)
        setattr(o, name, None if t is None else t.data_ptr())
    return o


def _stream_handle(stream):
    """hipStream_t of `stream`: a torch stream, a raw handle (int), or None for
    torch's current stream."""
    if isinstance(stream, int):
        return C.c_void_p(stream)
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _array(cls, items):
    arr = (cls * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


def rt_trace_image(params: list, outs: list, stream=None) -> None:
    """Calls rt_trace_image on lists of rt_image_params / rt_image_out."""
    _check(_lib.rt_trace_image(_array(rt_image_params, params), len(params),
                               _array(rt_image_out, outs), _stream_handle(stream)))


def rt_transfer_maps(params: list, outs: list, stream=None) -> None:
    _check(_lib.rt_transfer_maps(_array(rt_image_params, params), len(params),
                                 _array(rt_image_out, outs), _stream_handle(stream)))


def rt_image_setup(params: rt_image_params) -> dict:
    buf = (C.c_double * 4)()
    _check(_lib.rt_image_setup(C.byref(params), buf))
    return dict(r_plus=buf[0], r_stop=buf[1], r_esc=buf[2], r_in=buf[3])


def rt_set_kernel_timing(start_event, stop_event) -> None:
    """Bracket the trace kernels of later calls on this thread with two
    torch.cuda.Event objects (or raw hipEvent_t ints); None, None switches off."""
    def h(ev):
        if ev is None:
            return None
        return C.c_void_p(ev if isinstance(ev, int) else ev.cuda_event)
    _check(_lib.rt_set_kernel_timing(h(start_event), h(stop_event)))


def rt_visibility_dft(intensity, params: rt_image_params, uv, amp=None, vis=None,
                      stream=None) -> None:
    """Calls rt_visibility_dft on device tensors: intensity [ny][nx] f64,
    uv [K][2] f64, amp [K] f64 and/or vis [K][2] f64 (outputs)."""
    K = int(uv.shape[0])
    _check(_lib.rt_visibility_dft(C.c_void_p(intensity.data_ptr()), C.byref(params),
                                  C.c_void_p(uv.data_ptr()), K,
                                  None if amp is None else C.c_void_p(amp.data_ptr()),
                                  None if vis is None else C.c_void_p(vis.data_ptr()),
                                  _stream_handle(stream)))


def visibility(img: dict, intensity, uv, stream=None):
    """Normalised amplitudes |V|/|V(0,0)| of a traced image at the (u, v) points
    uv (a numpy array or tensor [K][2]); returns a device tensor [K]."""
    import torch
    uv_t = torch.as_tensor(uv, dtype=torch.float64, device=intensity.device).contiguous()
    amp = torch.empty(uv_t.shape[0], dtype=torch.float64, device=intensity.device)
    rt_visibility_dft(intensity.contiguous(), params_from(img), uv_t, amp=amp, stream=stream)
    return amp


def rt_visibility_dft_batch(images: list, stream=None) -> None:
    """Calls rt_visibility_dft_batch on a list of rt_vis_image descriptors."""
    arr = _array(rt_vis_image, images)
    _check(_lib.rt_visibility_dft_batch(arr, len(images), _stream_handle(stream)))


def vis_image_from(img: dict, intensity, uv, amp=None, vis=None) -> rt_vis_image:
    """The batched-visibility descriptor of a traced image (device tensors)."""
    return rt_vis_image(
        intensity=intensity.data_ptr(), uv=uv.data_ptr(),
        amp=None if amp is None else amp.data_ptr(), vis=None if vis is None else vis.data_ptr(),
        nx=int(img["nx"]), ny=int(img["ny"]), K=int(uv.shape[0]), reserved=0,
        x_min=img["x_min"], x_max=img["x_max"], y_min=img["y_min"], y_max=img["y_max"])


def visibility_many(imgs: list, intensities: list, uvs: list, stream=None) -> list:
    """Normalised amplitudes of several images in one batched call; returns a
    device tensor [K_i] per image."""
    import torch
    keep, descs, amps = [], [], []
    for img, I, uv in zip(imgs, intensities, uvs):
        uv_t = torch.as_tensor(uv, dtype=torch.float64, device=I.device).contiguous()
        amp = torch.empty(uv_t.shape[0], dtype=torch.float64, device=I.device)
        Ic = I.contiguous()
        keep += [uv_t, Ic]
        amps.append(amp)
        descs.append(vis_image_from(img, Ic, uv_t, amp=amp))
    rt_visibility_dft_batch(descs, stream)
    return amps


def rt_visibility_rings(intensity, params: rt_image_params, q, n_angles: int, avg=None, cut=None,
                        stream=None) -> None:
    """Calls rt_visibility_rings on device tensors: q [n_q] f64, avg and/or cut
    [n_q] f64 (outputs)."""
    _check(_lib.rt_visibility_rings(C.c_void_p(intensity.data_ptr()), C.byref(params),
                                    C.c_void_p(q.data_ptr()), int(q.shape[0]), int(n_angles),
                                    None if avg is None else C.c_void_p(avg.data_ptr()),
                                    None if cut is None else C.c_void_p(cut.data_ptr()),
                                    _stream_handle(stream)))


def visibility_rings(img: dict, intensity, q, n_angles: int = 64, stream=None):
    """The azimuthally averaged amplitude V(q) over n_angles directions and the
    horizontal cut V(|u|, 0) of a traced image at radii q; returns (avg, cut)
    device tensors [n_q]."""
    import torch
    q_t = torch.as_tensor(q, dtype=torch.float64, device=intensity.device).contiguous()
    avg = torch.empty_like(q_t)
    cut = torch.empty_like(q_t)
    rt_visibility_rings(intensity.contiguous(), params_from(img), q_t, n_angles, avg, cut, stream)
    return avg, cut


def rt_trace_thick(params: rt_image_params, thick: rt_thick_disc, out: rt_image_out,
                   stream=None) -> None:
    """Calls rt_trace_thick (one image)."""
    _check(_lib.rt_trace_thick(C.byref(params), C.byref(thick), C.byref(out),
                               _stream_handle(stream)))


def trace_thick(img: dict, r_scale: float, h0: float, h_slope: float, stream=None) -> dict:
    """The thick-disc image of img (Sec. 5.1-5.2): device tensors intensity,
    status, attempts, ncross and the transfer maps."""
    outs = alloc_outputs(img, reduce=False)
    for k in ("g_em", "intensity_n", "reduce"):
        outs.pop(k, None)
    o = out_from(outs)
    rt_trace_thick(params_from(img), rt_thick_disc(r_scale, h0, h_slope), o, stream)
    return outs


def rt_parameter_scan(points, out, stream=None) -> None:
    """Calls rt_parameter_scan on device tensors: points a uint8 tensor holding
    n rt_scan_point structs (packed by parameter_scan), out [n][4] f64."""
    n = int(out.shape[0])
    _check(_lib.rt_parameter_scan(C.c_void_p(points.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                  _stream_handle(stream)))


def parameter_scan(metric, spin, halo0, halo1, theta, stream=None):
    """R_+, the ergosurface radius at theta, chi_e and r_e for each parameter
    point (array-likes of one length; metric as "kerr"/"einasto"/"cnfw" or the
    RT_* codes): returns a device tensor [n][4]."""
    import numpy as np
    import torch
    codes = {"kerr": RT_KERR, "einasto": RT_EINASTO, "cnfw": RT_CNFW}
    seq = list(metric) if isinstance(metric, (list, tuple)) else list(np.atleast_1d(metric))
    m = [codes[str(x)] if isinstance(x, (str, np.str_)) else int(x) for x in seq]
    n = len(m)
    host = (rt_scan_point * n)()
    cols = [np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)) for v in (spin, halo0, halo1, theta)]
    for i in range(n):
        host[i].metric = m[i]
        host[i].reserved = 0
        host[i].spin = float(cols[0][i])
        host[i].halo[0] = float(cols[1][i])
        host[i].halo[1] = float(cols[2][i])
        host[i].theta = float(cols[3][i])
    raw = torch.frombuffer(bytearray(bytes(host)), dtype=torch.uint8).to("cuda")
    out = torch.empty(n, 4, dtype=torch.float64, device="cuda")
    rt_parameter_scan(raw, out, stream)
    return out


def einasto_extremal_spin(lam_e: float) -> float:
    """The extremal spin of the Einasto seed with lambda_E = lam_e, from
    rt_parameter_scan (synchronous); 0 when no horizon exists at any spin."""
    import math
    v = float(parameter_scan(["einasto"], 0.0, lam_e, 0.0, 1.0)[0, 2].item())
    return v if math.isfinite(v) else 0.0


RT_DIAG_COUNT = 14
RT_DIAG_NOALLOC_MAX_BINS = 65536
DIAG_KEYS = ("F", "X_c", "Y_c", "C", "rho_bar", "d_img", "w_img", "w_over_d", "A_LR",
             "I_max", "I_mean_emitting", "P", "rho_peak", "d_peak")


def rt_image_diagnostics(intensity, params: rt_image_params, bin_width: float, n_bins: int,
                         out, profile=None, stream=None) -> None:
    """Calls rt_image_diagnostics on device tensors: intensity [ny][nx] f64,
    out [RT_DIAG_COUNT] f64 and optionally profile [n_bins] f64 (outputs)."""
    _check(_lib.rt_image_diagnostics(C.c_void_p(intensity.data_ptr()), C.byref(params),
                                     bin_width, n_bins, C.c_void_p(out.data_ptr()),
                                     None if profile is None else C.c_void_p(profile.data_ptr()),
                                     _stream_handle(stream)))


def rt_image_diagnostics_noalloc(intensity, params: rt_image_params, bin_width: float,
                                 n_bins: int, out, profile=None, stream=None) -> None:
    """Calls rt_image_diagnostics_noalloc (the entry point that allocates
    nothing) on device tensors, as rt_image_diagnostics."""
    _check(_lib.rt_image_diagnostics_noalloc(
        C.c_void_p(intensity.data_ptr()), C.byref(params), bin_width, n_bins,
        C.c_void_p(out.data_ptr()), None if profile is None else C.c_void_p(profile.data_ptr()),
        _stream_handle(stream)))


def rt_relative_deviation(q, ref, delta, stream=None) -> None:
    """Calls rt_relative_deviation on device f64 tensors of equal length."""
    _check(_lib.rt_relative_deviation(C.c_void_p(q.data_ptr()), C.c_void_p(ref.data_ptr()),
                                      int(q.numel()), C.c_void_p(delta.data_ptr()),
                                      _stream_handle(stream)))


def relative_to_reference(q, ref, stream=None):
    """delta Q = (Q - Q_ref)/Q_ref of two device tensors (Sec. 6.2)."""
    import torch
    delta = torch.empty_like(q)
    rt_relative_deviation(q.contiguous(), ref.contiguous(), delta, stream)
    return delta


def image_diagnostics(img: dict, intensity, bin_width: float, n_bins: int, stream=None):
    """The diagnostics of a traced image as a dict of device scalars (DIAG_KEYS)
    plus the radial profile (device tensor [n_bins])."""
    import torch
    out = torch.empty(RT_DIAG_COUNT, dtype=torch.float64, device=intensity.device)
    prof = torch.empty(n_bins, dtype=torch.float64, device=intensity.device)
    rt_image_diagnostics(intensity.contiguous(), params_from(img), bin_width, n_bins, out, prof,
                         stream)
    d = dict(zip(DIAG_KEYS, out))
    d["profile"] = prof
    return d


def rt_trace_points(params: rt_image_params, xy, out: rt_image_out, stream=None) -> None:
    """Calls rt_trace_points on a device tensor xy [n][2] (f64 screen points)."""
    n = int(xy.shape[0])
    _check(_lib.rt_trace_points(C.byref(params), C.c_void_p(xy.data_ptr()), n, C.byref(out),
                                _stream_handle(stream)))


def alloc_point_outputs(n: int, device="cuda", emission: bool = True) -> dict:
    """Device tensors for every output of n screen points."""
    import torch
    d = dict(ncross=torch.empty(n, dtype=torch.uint8, device=device),
             status=torch.empty(n, dtype=torch.uint8, device=device),
             r_em=torch.empty((3, n), dtype=torch.float64, device=device),
             phi_em=torch.empty((3, n), dtype=torch.float64, device=device),
             t_em=torch.empty((3, n), dtype=torch.float64, device=device),
             attempts=torch.empty(n, dtype=torch.int32, device=device))
    if emission:
        d.update(g_em=torch.empty((3, n), dtype=torch.float64, device=device),
                 intensity=torch.empty(n, dtype=torch.float64, device=device),
                 intensity_n=torch.empty((3, n), dtype=torch.float64, device=device))
    return d


def trace_points(img: dict, xy, device="cuda", stream=None, emission: bool = True) -> dict:
    """Trace the screen points xy ([n][2] f64, a device tensor or array) of the
    observer of img; returns the outputs as device tensors indexed by point."""
    import torch
    xy = torch.as_tensor(xy, dtype=torch.float64, device=device).contiguous()
    outs = alloc_point_outputs(int(xy.shape[0]), device, emission)
    rt_trace_points(params_from(img), xy, out_from(outs), stream)
    return outs


def rt_refine_points(params: rt_image_params, ncross, status, sub: int, max_points: int, xy,
                     pix, n_marked, stream=None) -> None:
    """Calls rt_refine_points on device tensors: ncross, status [ny][nx] uint8,
    xy [max_points][2] f64 (or None), pix int64 (or None), n_marked [1] int64."""
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
    _check(_lib.rt_refine_points(C.byref(params), ptr(ncross), ptr(status), sub, max_points, ptr(xy),
                                 ptr(pix), ptr(n_marked), _stream_handle(stream)))


def refine_points(img: dict, ncross, status, sub: int, stream=None):
    """The band-edge pixels of a traced screen and their sub x sub subpixel
    centres: a counting call, then one that fills buffers of that size.
    Returns (xy [n sub^2][2], pix [n]) as device tensors."""
    import torch
    dev = ncross.device
    n_marked = torch.zeros(1, dtype=torch.int64, device=dev)
    p = params_from(img)
    nc, st = ncross.contiguous(), status.contiguous()
    rt_refine_points(p, nc, st, sub, 0, None, None, n_marked, stream)
    torch.cuda.synchronize()
    n = int(n_marked.item())
    xy = torch.empty((n * sub * sub, 2), dtype=torch.float64, device=dev)
    pix = torch.empty(n, dtype=torch.int64, device=dev)
    if n:
        rt_refine_points(p, nc, st, sub, n * sub * sub, xy, pix, n_marked, stream)
    return xy, pix


def rt_shadow_boundary(params: rt_image_params, dirs, b_lo: float, b_hi: float, b_tol: float,
                       out, status, attempts=None, stream=None, samples: int = 64) -> None:
    """Calls rt_shadow_boundary on device tensors: dirs [n][2] f64 (cos psi,
    sin psi), out [n][2] f64, status [n] int32 and optionally attempts [n]
    int64 (outputs)."""
    n = int(dirs.shape[0])
    _check(_lib.rt_shadow_boundary(C.byref(params), C.c_void_p(dirs.data_ptr()), n, samples, b_lo, b_hi,
                                   b_tol, C.c_void_p(out.data_ptr()),
                                   C.c_void_p(status.data_ptr()),
                                   None if attempts is None else C.c_void_p(attempts.data_ptr()),
                                   _stream_handle(stream)))


def rt_shadow_boundary_samples(n: int) -> int:
    """The library's sample count for n directions on the current device
    (16, 32 or 64, see rt.h)."""
    rc = _lib.rt_shadow_boundary_samples(n)
    _check(min(rc, 0))
    return rc


def shadow_boundary(img: dict, dirs, b_lo: float, b_hi: float, b_tol: float, stream=None,
                    samples: int = 64):
    """The shadow boundary of img's spacetime and observer along the screen
    directions dirs ([n][2] (cos psi, sin psi), numpy or tensor): returns device
    tensors (out [n][2] = the final bracket of b, status [n])."""
    import torch
    d = torch.as_tensor(dirs, dtype=torch.float64, device="cuda").reshape(-1, 2).contiguous()
    out = torch.empty(d.shape[0], 2, dtype=torch.float64, device=d.device)
    status = torch.empty(d.shape[0], dtype=torch.int32, device=d.device)
    rt_shadow_boundary(params_from(img), d, b_lo, b_hi, b_tol, out, status, stream=stream,
                       samples=samples)
    return out, status


def rt_set_launch_config(chunk: int = 0, tile_w: int = 0, tile_h: int = 0,
                         blocks_per_cu: int = 0, order: int = RT_ORDER_CENTRE,
                         reset: bool = False) -> None:
    """Work-distribution settings of later traces on this thread (see rt.h);
    reset=True restores the library defaults."""
    if reset:
        _check(_lib.rt_set_launch_config(None))
        return
    cfg = rt_launch_config(chunk, tile_w, tile_h, blocks_per_cu, order)
    _check(_lib.rt_set_launch_config(C.byref(cfg)))


def rt_get_launch_config() -> dict:
    cfg = rt_launch_config()
    _check(_lib.rt_get_launch_config(C.byref(cfg)))
    return dict(chunk=cfg.chunk, tile_w=cfg.tile_w, tile_h=cfg.tile_h,
                blocks_per_cu=cfg.blocks_per_cu, order=cfg.order)


def rt_image_vjp(params: rt_image_params, dl_dI, grad, grad_pix=None,
                 basis: int = RT_GRAD_NATIVE, stream=None) -> None:
    """Calls rt_image_vjp on device tensors: dl_dI [ny][nx] f64 (input),
    grad [4] f64 and optionally grad_pix [ny][nx][4] f64 (outputs)."""
    _check(_lib.rt_image_vjp(C.byref(params), C.c_void_p(dl_dI.data_ptr()), basis,
                             C.c_void_p(grad.data_ptr()),
                             None if grad_pix is None else C.c_void_p(grad_pix.data_ptr()),
                             _stream_handle(stream)))


def rt_mixed_stats() -> dict:
    """Counters of the last mixed-precision image traced on this thread."""
    buf = (C.c_int64 * 4)()
    _check(_lib.rt_mixed_stats(buf))
    return dict(binary64=buf[0], rerun=buf[1], handed_off=buf[0] - buf[1],
                attempts32=buf[2], attempts64=buf[3])


def rt_set_split_timing(event) -> None:
    """Record `event` (torch.cuda.Event, created) between the binary32 and the
    binary64 pass of each later mixed-precision image; None switches it off."""
    _check(_lib.rt_set_split_timing(None if event is None else C.c_void_p(event.cuda_event)))


def rt_set_checkpoint_budget(nbytes: int) -> None:
    _check(_lib.rt_set_checkpoint_budget(int(nbytes)))


def rt_vjp_stats() -> dict:
    """Statistics of the last gradient on this thread (synchronous)."""
    buf = (C.c_int64 * 5)()
    _check(_lib.rt_vjp_stats(buf))
    return dict(rays=buf[0], steps=buf[1], slots=buf[2], scratch_bytes=buf[3], diverged=buf[4])


def rt_version() -> int:
    return _lib.rt_version()


def rt_last_error() -> str:
    return _lib.rt_last_error().decode()


# --------------------------------------------------------------- conveniences
def alloc_outputs(img: dict, device="cuda", emission: bool = True, reduce: bool = True) -> dict:
    """Device tensors for every output of one image."""
    import torch
    ny, nx = int(img["ny"]), int(img["nx"])
    d = dict(
        ncross=torch.empty((ny, nx), dtype=torch.uint8, device=device),
        status=torch.empty((ny, nx), dtype=torch.uint8, device=device),
        r_em=torch.empty((3, ny, nx), dtype=torch.float64, device=device),
        phi_em=torch.empty((3, ny, nx), dtype=torch.float64, device=device),
        t_em=torch.empty((3, ny, nx), dtype=torch.float64, device=device),
        attempts=torch.empty((ny, nx), dtype=torch.int32, device=device),
    )
    if emission:
        d.update(g_em=torch.empty((3, ny, nx), dtype=torch.float64, device=device),
                 intensity=torch.empty((ny, nx), dtype=torch.float64, device=device),
                 intensity_n=torch.empty((3, ny, nx), dtype=torch.float64, device=device))
        if reduce:
            d["reduce"] = torch.empty(3, dtype=torch.float64, device=device)
    return d


def trace(img: dict, device="cuda", stream=None, emission: bool = True) -> dict:
    """Trace one image (workload dict) and return its outputs as device tensors."""
    outs = alloc_outputs(img, device, emission)
    f = rt_trace_image if emission else rt_transfer_maps
    f([params_from(img)], [out_from(outs)], stream)
    return outs


def trace_many(imgs: list, device="cuda", stream=None) -> list:
    outs = [alloc_outputs(i, device) for i in imgs]
    rt_trace_image([params_from(i) for i in imgs], [out_from(o) for o in outs], stream)
    return outs


def image_vjp(img: dict, dl_dI, basis: str = "native", per_pixel: bool = False, stream=None):
    """dL/dq for the image of `img` given the device tensor dl_dI [ny][nx]:
    returns a device tensor [4] (and [ny][nx][4] per-pixel terms if asked).
    basis "native": q = (spin, incl, halo0, halo1); "density" (cored NFW):
    q = (spin, incl, rho_s, r_s)."""
    import torch
    dev = dl_dI.device
    grad = torch.empty(4, dtype=torch.float64, device=dev)
    gp = (torch.empty((int(img["ny"]), int(img["nx"]), 4), dtype=torch.float64, device=dev)
          if per_pixel else None)
    rt_image_vjp(params_from(img), dl_dI.contiguous(), grad, gp,
                 RT_GRAD_DENSITY if basis == "density" else RT_GRAD_NATIVE, stream)
    return (grad, gp) if per_pixel else grad


__all__ = ["rt_mixed_stats", "rt_image_vjp", "rt_set_checkpoint_budget", "rt_vjp_stats", "image_vjp", "rt_trace_image", "rt_transfer_maps", "rt_image_setup", "rt_set_kernel_timing", "rt_set_split_timing",
           "rt_set_launch_config", "rt_get_launch_config", "rt_visibility_dft", "visibility",
           "rt_visibility_dft_batch", "rt_vis_image", "vis_image_from", "visibility_many",
           "rt_visibility_rings", "visibility_rings",
           "rt_shadow_boundary", "rt_shadow_boundary_samples", "shadow_boundary", "rt_image_diagnostics", "rt_image_diagnostics_noalloc", "image_diagnostics",
           "rt_relative_deviation", "relative_to_reference",
           "rt_parameter_scan", "parameter_scan", "rt_scan_point", "einasto_extremal_spin",
           "rt_trace_thick", "trace_thick", "rt_thick_disc",
           "rt_trace_points", "trace_points", "alloc_point_outputs", "rt_refine_points",
           "refine_points",
           "RT_DIAG_COUNT", "RT_DIAG_NOALLOC_MAX_BINS", "DIAG_KEYS",
           "rt_version",
           "rt_last_error", "trace", "trace_many", "params_from", "out_from", "alloc_outputs",
           "RTError"]
