"""Throughput benchmark of the backward geodesic ray tracer on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-<leg> ...]

One step = one full trace of the 1024x1024 cored-NFW screen (chi = 0.94,
(eta, lambda_c) = (0.02, 10), theta_o = 163 deg, R_o = 1000, +-10 M, FP64
Dormand-Prince at rtol = atol = 1e-8, up to three crossings, thin-disc
intensity, flux and centroid) through the C ABI, with the outputs resident in
HBM.  Prints one JSON line: whole-job rays/s, the trace kernel's algorithmic
FLOP rate against the FP64 vector peak, and the CPU oracle's rate on a
strided sample of the same screen.
"""
from __future__ import annotations

import argparse
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "geodesic rays/s at 1024² (FP64 vs mixed); adjoint image-gradient ms"
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X, packed binary32 (two FMAs per lane per cycle)
HOST_THREADS = 16                # host threads the CPU baseline uses at most (one GPU's share of the host)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel_hash: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when it is missing or was taken on different kernel code (comments and
    layout aside)."""
    path = os.path.join(ROOT, "profiles", "trace_kernel_cnfw_1024_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def host_cpu() -> dict:
    """The host this runs on: CPU model, logical CPUs of the machine and of
    this process's affinity mask."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count() or 1}


def oracle_threads() -> int:
    return max(1, min(HOST_THREADS, host_cpu()["nproc"]))


def cpu_baseline(img: dict, stride: int):
    """The oracle timed on the host's cores on the same screen (every
    `stride`-th pixel in x and y).  Returns the baseline object and the
    oracle's outputs with their pixel indices, from which the bench reports
    the GPU images' per-pixel error against the oracle."""
    from oracle import oracle as O
    from paper_2605_05635_amd import workloads as W
    threads = oracle_threads()
    idx = W.subsample_indices(img["nx"], img["ny"], stride)
    log(f"cpu baseline: oracle on {idx.size} pixels with {threads} threads")
    t0 = time.perf_counter()
    ref = O.trace_pixels(img, idx, threads=threads)
    dt = time.perf_counter() - t0
    res = {"value": idx.size / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
           "sample": (f"every {stride}th pixel in x and y of" if stride > 1 else "every pixel of")
                     + " the same screen "
                     f"({idx.size} rays, {dt:.1f} s)", **host_cpu()}
    return res, ref, idx


def error_vs_oracle(outs: dict, ref: dict, idx) -> dict:
    """Per-pixel difference of a GPU image from the oracle's trace of the same
    pixels: as image_error, plus the fraction of pixels whose intensity is
    within the binary64 parity bar (1e-6 relative, exact zeros)."""
    import numpy as np
    import torch
    ii = torch.as_tensor(np.asarray(idx), device=outs["ncross"].device)
    take = lambda t: t.reshape(-1)[ii] if t.dim() == 2 else t.reshape(3, -1)[:, ii]  # noqa: E731
    g = {k: take(outs[k]) for k in ("ncross", "status", "intensity", "r_em")}
    o = {"ncross": torch.as_tensor(ref["ncross"], device=ii.device),
         "status": torch.as_tensor(ref["status"], device=ii.device),
         "intensity": torch.as_tensor(ref["intensity"], device=ii.device),
         "r_em": torch.as_tensor(ref["r_em"], device=ii.device)}
    res = image_error(g, o)
    same = (g["ncross"].long() == o["ncross"].long()) & (g["status"].long() == o["status"].long())
    Io, Ig = o["intensity"], g["intensity"]
    ok = torch.where(Io != 0, (Ig - Io).abs() <= 1e-6 * Io.abs(), Ig == 0) & same
    res["pixels"] = int(ii.numel())
    res["intensity_within_1e-6_frac"] = float(ok.double().mean().item())
    return res


def batch_measurement(steps: int) -> dict:
    """64 images of mixed metric and resolution in one persistent launch, plus
    normalised visibility amplitudes at 2000 seeded (u, v) points per image."""
    import torch

    from paper_2605_05635_amd import autotune, rt, workloads as W
    imgs = W.batch_64(rt.einasto_extremal_spin)
    rays = sum(i["nx"] * i["ny"] for i in imgs)
    log(f"batch: 64 images, {rays} rays; autotuning the launch configuration")
    best = autotune.tune(imgs, log=log)
    outs = [rt.alloc_outputs(i) for i in imgs]
    params = [rt.params_from(i) for i in imgs]
    ouv = [rt.out_from(o) for o in outs]
    uvs = [torch.tensor(W.uv_points(1000 + j, 2000), device="cuda") for j in range(len(imgs))]
    amps = [torch.empty(2000, dtype=torch.float64, device="cuda") for _ in imgs]
    vdesc = [rt.vis_image_from(img, o["intensity"], uv, amp)
             for img, o, uv, amp in zip(imgs, outs, uvs, amps)]
    stream = torch.cuda.current_stream()

    def visibilities():
        rt.rt_visibility_dft_batch(vdesc, stream)

    def one_batch():
        rt.rt_trace_image(params, ouv, stream)
        visibilities()

    one_batch()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for _ in range(steps):
        rt.rt_trace_image(params, ouv, stream)
    ev[1].record(stream)
    for _ in range(steps):
        visibilities()
    ev[2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    trace_ms = ev[0].elapsed_time(ev[1]) / steps
    dft_ms = ev[1].elapsed_time(ev[2]) / steps
    rt.rt_set_launch_config(reset=True)
    attempts = sum(o["attempts"].double().sum().item() for o in outs)
    log(f"batch: trace {trace_ms:.2f} ms, visibilities {dft_ms:.2f} ms per batch")
    # the trace's algorithmic flops, as for the single-image trace kernel, per image's metric
    from paper_2605_05635_amd import census
    trace_flops = 0.0
    for img, o in zip(imgs, outs):
        m, n = img["metric"], img["nx"] * img["ny"]
        trace_flops += (o["attempts"].double().sum().item()
                        * (6 * census.flops_rhs(m) + census.flops_step_overhead())
                        + o["ncross"].double().sum().item() * census.flops_crossing()
                        + n * (20 + census.flops_rhs(m)))
    trace_tflops = trace_flops / (trace_ms * 1e-3) / 1e12
    # the visibility contraction: 2 K nx ny complex-by-real multiply-adds = 4 K nx ny flops
    vis_flops = sum(4.0 * 2000 * i["nx"] * i["ny"] for i in imgs)
    vis_tflops = vis_flops / (dft_ms * 1e-3) / 1e12
    return {"workload": "64 images, res in {128..768}^2, mixed metrics, one launch; "
                        "2000 (u,v) visibility amplitudes per image (one batched call)",
            "rays": rays, "steps": steps, "trace_ms": trace_ms, "visibility_ms": dft_ms,
            "trace_roofline": {"bound": "alu", "achieved": trace_tflops,
                               "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": trace_tflops / FP64_VECTOR_PEAK_TFLOPS,
                               "flops": trace_flops, "kernel": "trace_batch_kernel"},
            "visibility_roofline": {"bound": "alu", "achieved": vis_tflops,
                                    "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                    "frac": vis_tflops / FP64_VECTOR_PEAK_TFLOPS,
                                    "flops": vis_flops, "kernel": "vis_partial_kernel"},
            "ms_per_batch": wall * 1e3 / steps, "rays_per_s": rays / (trace_ms * 1e-3),
            "attempts_per_ray": attempts / rays,
            "launch_config": {k: best[k] for k in ("chunk", "tile_w", "tile_h", "blocks_per_cu")},
            "visibility_finite": bool(all(torch.isfinite(a).all().item() for a in amps))}


def image_error(outs: dict, ref: dict) -> dict:
    """Per-pixel difference of a traced image from a reference trace of the same
    screen: |dI|/max I over pixels with equal crossing count and status (50th,
    99th percentile, max), |dR_em| over their recorded crossings, and the
    numbers of pixels whose crossing count or status differ."""
    import torch
    nc, ncr = outs["ncross"].flatten().long(), ref["ncross"].flatten().long()
    st, str_ = outs["status"].flatten().long(), ref["status"].flatten().long()
    same = (nc == ncr) & (st == str_)
    I, Ir = outs["intensity"].flatten(), ref["intensity"].flatten()
    dI = ((I - Ir).abs() / Ir.abs().max())[same]
    r, rr = outs["r_em"].reshape(3, -1), ref["r_em"].reshape(3, -1)
    have = (torch.arange(3, device=r.device)[:, None] < ncr.clamp(max=3)[None, :]) & same[None, :]
    dR = (r - rr).abs()[have]
    q = lambda t, p: float(torch.quantile(t, p).item()) if t.numel() else 0.0  # noqa: E731
    return {"dI_rel_p50": q(dI, 0.5), "dI_rel_p99": q(dI, 0.99),
            "dI_rel_max": float(dI.max().item()) if dI.numel() else 0.0,
            "dR_em_p99": q(dR, 0.99), "dR_em_max": float(dR.max().item()) if dR.numel() else 0.0,
            "ncross_mismatch": int((nc != ncr).sum().item()),
            "status_mismatch": int((st != str_).sum().item())}


def timed_trace(img: dict, steps: int):
    """Trace `img` `steps` times (after one warm-up); returns (outputs, kernel ms)."""
    import numpy as np
    import torch

    from paper_2605_05635_amd import rt
    outs = rt.alloc_outputs(img)
    p, o = [rt.params_from(img)], [rt.out_from(outs)]
    stream = torch.cuda.current_stream()
    rt.rt_trace_image(p, o, stream)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    stops = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for ev in starts + stops:
        ev.record(stream)
    torch.cuda.synchronize()
    for k in range(steps):
        rt.rt_set_kernel_timing(starts[k], stops[k])
        rt.rt_trace_image(p, o, stream)
    rt.rt_set_kernel_timing(None, None)
    torch.cuda.synchronize()
    return outs, float(np.mean([a.elapsed_time(b) for a, b in zip(starts, stops)]))


def mixed_measurement(steps: int, ref64: dict) -> dict:
    """The same 1024x1024 cored-NFW screen in mixed precision (binary32 bulk at
    1e-6, binary64 from 1.5 R_+ inward, rays with two crossings traced again in
    binary64): rays/s, its difference from the FP64 run at 1e-8, and the
    accuracy-matched comparison -- the error of the mixed image and of FP64
    images at tolerances 1e-6 ... 1e-9 against an FP64 reference at 1e-11,
    with each one's rays/s."""
    import numpy as np
    import torch

    from paper_2605_05635_amd import census, rt, workloads as W
    img = W.cnfw_1024("mixed")
    n = img["nx"] * img["ny"]
    splits = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for ev in splits + starts:
        ev.record()
    outs = rt.alloc_outputs(img)
    p, o = [rt.params_from(img)], [rt.out_from(outs)]
    stream = torch.cuda.current_stream()
    rt.rt_trace_image(p, o, stream)
    stops = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for ev in stops:
        ev.record(stream)
    torch.cuda.synchronize()
    for k in range(steps):
        rt.rt_set_kernel_timing(starts[k], stops[k])
        rt.rt_set_split_timing(splits[k])
        rt.rt_trace_image(p, o, stream)
    rt.rt_set_kernel_timing(None, None)
    rt.rt_set_split_timing(None)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in zip(starts, stops)]))
    bulk_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(starts, splits)]))
    stats = rt.rt_mixed_stats()
    log(f"mixed: kernel {ms:.3f} ms (binary32 pass {bulk_ms:.3f} ms), {stats['binary64']} rays "
        f"finished in FP64 ({stats['rerun']} traced again)")
    # the binary32 pass's algorithmic flops (binary32 arithmetic; its crossings,
    # located in binary64, not counted) against the packed binary32 peak
    f32 = stats["attempts32"] * (6 * census.flops_rhs(img["metric"])
                                 + census.flops_step_overhead32())
    t32 = f32 / (bulk_ms * 1e-3) / 1e12
    res = {"rays_per_s": n / (ms * 1e-3), "kernel_ms": ms, "fp64_finished": stats["binary64"],
           "fp64_reruns": stats["rerun"],
           "attempts_per_ray": float(outs["attempts"].double().mean().item()),
           "binary32_pass": {"kernel": "trace32_kernel<CNFW_NEAR>", "kernel_ms": bulk_ms,
                             "attempts": stats["attempts32"],
                             "algorithmic_tflops": t32, "peak": FP32_VECTOR_PEAK_TFLOPS,
                             "frac_of_fp32_vector_peak": t32 / FP32_VECTOR_PEAK_TFLOPS,
                             "frac_of_unpacked_fp32_rate": t32 / FP64_VECTOR_PEAK_TFLOPS},
           "binary64_pass": {"kernel": "resume_kernel<CNFW_NEAR>", "kernel_ms": ms - bulk_ms,
                             "attempts": stats["attempts64"]},
           "error_vs_fp64_1e-8": image_error(outs, ref64)}
    tight = dict(W.cnfw_1024(), rtol=1e-11, atol=1e-11)
    ref, ref_ms = timed_trace(tight, 1)
    log(f"fp64 reference at 1e-11: {ref_ms:.1f} ms")
    res["error_vs_fp64_1e-11"] = image_error(outs, ref)
    sweep = []
    for tol in (1e-6, 1e-7, 1e-8, 1e-9):
        o, t_ms = timed_trace(dict(W.cnfw_1024(), rtol=tol, atol=tol), max(2, steps // 2))
        e = image_error(o, ref)
        sweep.append({"tol": tol, "rays_per_s": n / (t_ms * 1e-3), "kernel_ms": t_ms,
                      "dI_rel_p99": e["dI_rel_p99"], "dR_em_p99": e["dR_em_p99"],
                      "ncross_mismatch": e["ncross_mismatch"]})
        log(f"fp64 tol {tol:g}: {t_ms:.2f} ms, p99 dI/max I {e['dI_rel_p99']:.2e}")
    res["fp64_sweep_vs_1e-11"] = sweep
    p99 = res["error_vs_fp64_1e-11"]["dI_rel_p99"]
    ok = [s_ for s_ in sweep if s_["dI_rel_p99"] <= p99]
    match = max(ok, key=lambda s_: s_["rays_per_s"]) if ok else None
    res["fp64_at_matched_accuracy"] = match
    res["speedup_vs_fp64_1e-8"] = res["rays_per_s"] / next(
        s_["rays_per_s"] for s_ in sweep if s_["tol"] == 1e-8)
    res["speedup_vs_fp64_matched"] = res["rays_per_s"] / match["rays_per_s"] if match else None
    return res, outs


def adjoint_measurement(steps: int, cpu: bool) -> dict:
    """Image gradient of the cored-NFW 256x256 tapered-disc image (chi = 0.94,
    theta_o = 60 deg, (eta, lambda_c) = (0.02, 10)) for the loss
    L = sum (I - I_target)^2, I_target traced at a 1 % change of
    (chi, theta_o, rho_s, r_s): time of rt_image_vjp per call (all its
    passes, stream-ordered with no host synchronisation, HIP events on the
    stream), beside the forward trace of the same image.  The same gradient
    of the image at 1024x1024 is timed too, with the scratch it took."""
    import math

    import numpy as np
    import torch

    from paper_2605_05635_amd import rt, workloads as W
    img = W.cnfw_adjoint_256()
    eta, lc = img["halo"]
    q = np.array([img["spin"], img["incl"], eta / (4 * math.pi * lc * lc), lc])
    qt = q * (1 + 0.01 * W.adjoint_target_signs())
    tgt = dict(img, spin=float(qt[0]), incl=float(qt[1]),
               halo=(float(4 * math.pi * qt[2] * qt[3] ** 2), float(qt[3])))
    stream = torch.cuda.current_stream()
    outs = rt.alloc_outputs(img)
    p, o = [rt.params_from(img)], [rt.out_from(outs)]
    rt.rt_trace_image(p, o, stream)
    I_t = rt.trace(tgt)["intensity"]
    dl = 2.0 * (outs["intensity"] - I_t)
    grad = torch.empty(4, dtype=torch.float64, device="cuda")
    rt.rt_image_vjp(p[0], dl, grad, None, rt.RT_GRAD_DENSITY, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        rt.rt_image_vjp(p[0], dl, grad, None, rt.RT_GRAD_DENSITY, stream)
    b.record(stream)
    torch.cuda.synchronize()
    adj_ms = a.elapsed_time(b) / steps
    stats = rt.rt_vjp_stats()
    a.record(stream)
    for _ in range(steps):
        rt.rt_trace_image(p, o, stream)
    b.record(stream)
    torch.cuda.synchronize()
    fwd_ms = a.elapsed_time(b) / steps
    loss = float(((outs["intensity"] - I_t) ** 2).sum().item())
    log(f"adjoint: {adj_ms:.2f} ms per gradient, forward {fwd_ms:.2f} ms")
    res = {"workload": "cored-NFW 256x256, tapered disc, L2 loss vs a 1 % parameter change",
           "adjoint_ms": adj_ms, "forward_ms": fwd_ms, "ratio": adj_ms / fwd_ms,
           "steps": steps, "loss": loss, "grad_chi_theta_rho_rs": grad.cpu().tolist(),
           "reversed_rays": stats["rays"], "reversed_steps": stats["steps"],
           "checkpoint_slots": stats["slots"], "scratch_bytes": stats["scratch_bytes"]}
    big = dict(img, nx=1024, ny=1024)
    outs_b = rt.trace(big)
    tgt_b = rt.trace(dict(tgt, nx=1024, ny=1024))
    dl_b = 2.0 * (outs_b["intensity"] - tgt_b["intensity"])
    del outs_b, tgt_b
    rt.rt_image_vjp(rt.params_from(big), dl_b, grad, None, rt.RT_GRAD_DENSITY, stream)
    torch.cuda.synchronize()
    n_big = 2
    a.record(stream)
    for _ in range(n_big):
        rt.rt_image_vjp(rt.params_from(big), dl_b, grad, None, rt.RT_GRAD_DENSITY, stream)
    b.record(stream)
    torch.cuda.synchronize()
    st_b = rt.rt_vjp_stats()
    res["full_screen"] = {"workload": "the same image at 1024x1024",
                          "adjoint_ms": a.elapsed_time(b) / n_big, "calls": n_big,
                          "reversed_rays": st_b["rays"], "reversed_steps": st_b["steps"],
                          "checkpoint_slots": st_b["slots"],
                          "scratch_bytes": st_b["scratch_bytes"], "diverged": st_b["diverged"]}
    log(f"adjoint 1024^2: {res['full_screen']['adjoint_ms']:.1f} ms, "
        f"{st_b['scratch_bytes'] / 2**30:.2f} GiB scratch")
    if cpu:
        from oracle import oracle as O
        threads = oracle_threads()
        idx = W.subsample_indices(img["nx"], img["ny"], 8)
        t0 = time.perf_counter()
        O.trace_grad_pixels(img, idx, threads=threads)
        dt = time.perf_counter() - t0
        res["cpu_dual_gradient"] = {
            "ms_per_image": dt * 1e3 * img["nx"] * img["ny"] / idx.size, "cores": threads,
            "kind": "oracle", "sample": f"every 8th pixel in x and y ({idx.size} rays, "
                                        f"{dt:.1f} s), scaled to the image"}
    return res


def _diagnostics_graph(rt, I, p, bw, nb, out, prof, steps, nbytes) -> dict:
    """Ten calls of rt_image_diagnostics_noalloc captured in one HIP graph and
    replayed: time per call, and whether every replay (with eager work between
    them) equals the eager call bit for bit."""
    import torch
    stream = torch.cuda.current_stream()
    ref_out, ref_prof = out.clone(), prof.clone()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g_out = torch.empty_like(out)
    g_prof = torch.empty_like(prof)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        rt.rt_image_diagnostics_noalloc(I, p, bw, nb, g_out, g_prof, side)   # first call: set-up
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    per_graph = 10
    with torch.cuda.graph(graph, capture_error_mode="relaxed"):
        gs = torch.cuda.current_stream()
        for _ in range(per_graph):
            rt.rt_image_diagnostics_noalloc(I, p, bw, nb, g_out, g_prof, gs)
    same = True
    reps = max(3, steps // per_graph)
    a.record(stream)
    for _ in range(reps):
        graph.replay()
    b.record(stream)
    torch.cuda.synchronize()
    gms = a.elapsed_time(b) / (reps * per_graph)
    for _ in range(3):   # replays interleaved with eager work, each checked
        g_out.zero_()
        g_prof.zero_()
        graph.replay()
        torch.cuda.synchronize()
        same = same and torch.equal(g_out, ref_out) and bool(
            torch.equal(torch.nan_to_num(g_prof, nan=-1.0), torch.nan_to_num(ref_prof, nan=-1.0)))
    log(f"diagnostics in a graph: {gms * 1e3:.1f} us per image (replays equal: {same})")
    return {"graph_us": gms * 1e3, "graph_replays_equal_eager": same,
            "graph_image_reads_GBps": nbytes / (gms * 1e-3) / 1e9}


def diagnostics_measurement(steps: int, outs: dict, img: dict, cpu: bool) -> dict:
    """Image diagnostics (Sec. 6.2-6.3) of the bench's traced 1024x1024 image:
    wall time of rt_image_diagnostics per call (HIP events on the stream),
    300 radial bins of 0.05 M.  Back-to-back calls from Python leave the GPU
    waiting for the host between kernels, so the same work is also timed as
    a HIP graph of ten calls of rt_image_diagnostics_noalloc (which allocates
    nothing and can be captured), replayed; every replay's results must equal
    the eager call's bit for bit."""
    import torch

    from paper_2605_05635_amd import rt
    I = outs["intensity"]
    bw, nb = 0.05, 300
    out = torch.empty(rt.RT_DIAG_COUNT, dtype=torch.float64, device="cuda")
    prof = torch.empty(nb, dtype=torch.float64, device="cuda")
    p = rt.params_from(img)
    stream = torch.cuda.current_stream()
    rt.rt_image_diagnostics(I, p, bw, nb, out, prof, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        rt.rt_image_diagnostics(I, p, bw, nb, out, prof, stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    vals = dict(zip(rt.DIAG_KEYS, out.cpu().tolist()))
    # four full reads of the image (flux/centroid, the moments, the width, the
    # profile's visits: ~1.2 reads measured by the run lengths) as the traffic floor
    nbytes = 8 * I.numel() * 4
    log(f"diagnostics: {ms * 1e3:.1f} us per image")
    res = {"workload": "image diagnostics of the 1024x1024 cored-NFW image, 300 bins of 0.05 M",
           "us": ms * 1e3, "steps": steps, "values": vals,
           "image_reads_GBps": nbytes / (ms * 1e-3) / 1e9}
    # the same calls captured in a graph (no host work between the kernels)
    try:
        res.update(_diagnostics_graph(rt, I, p, bw, nb, out, prof, steps, nbytes))
    except Exception as exc:   # a capture the runtime refuses is reported, not fatal
        res["graph_error"] = f"{type(exc).__name__}: {exc}"
        log(f"diagnostics in a graph: {res['graph_error']}")

    if cpu:
        from oracle import oracle as O
        In = I.cpu().numpy()
        t0 = time.perf_counter()
        O.image_diagnostics(img, In, bw, nb)
        res["cpu_oracle_ms"] = (time.perf_counter() - t0) * 1e3
    return res


def adaptive_measurement(steps: int, outs: dict, img: dict, cpu: bool) -> dict:
    """Adaptive screen (Sec. 4: the screen refined where the image
    classification changes) of the bench's traced 1024x1024 image: its
    band-edge pixels (a 4-neighbour with another N_cross or status) each
    refined into 4 x 4 subpixels by rt_refine_points, and the subpixel rays
    traced by rt_trace_points with their emission; HIP-event time of each call
    on the stream."""
    import torch

    from paper_2605_05635_amd import census, rt
    sub = 4
    p = rt.params_from(img)
    stream = torch.cuda.current_stream()
    xy, pix = rt.refine_points(img, outs["ncross"], outs["status"], sub)
    n_pts = int(xy.shape[0])
    n_marked = torch.zeros(1, dtype=torch.int64, device="cuda")
    pts = rt.alloc_point_outputs(n_pts)
    o = rt.out_from(pts)
    rt.rt_trace_points(p, xy, o, stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    for _ in range(steps):
        rt.rt_refine_points(p, outs["ncross"], outs["status"], sub, n_pts, xy, pix, n_marked, stream)
    ev[1].record(stream)
    for _ in range(steps):
        rt.rt_trace_points(p, xy, o, stream)
    ev[2].record(stream)
    torch.cuda.synchronize()
    refine_ms = ev[0].elapsed_time(ev[1]) / steps
    trace_ms = ev[1].elapsed_time(ev[2]) / steps
    att = pts["attempts"].double().sum().item()
    crossings = pts["ncross"].double().sum().item()
    flops = (att * (6 * census.flops_rhs(img["metric"]) + census.flops_step_overhead())
             + crossings * census.flops_crossing()
             + n_pts * (20 + census.flops_rhs(img["metric"])))
    tflops = flops / (trace_ms * 1e-3) / 1e12
    n_pix = img["nx"] * img["ny"]
    log(f"adaptive screen: {n_pts // (sub * sub)} band-edge pixels, {n_pts} subpixel rays in "
        f"{trace_ms:.2f} ms (refinement {refine_ms * 1e3:.0f} us)")
    res = {"workload": "band-edge pixels of the 1024x1024 cored-NFW image, 4 x 4 subpixels each",
            "band_edge_pixels": n_pts // (sub * sub), "subpixel_rays": n_pts,
            "refine_us": refine_ms * 1e3, "trace_ms": trace_ms, "steps": steps,
            "rays_per_s": n_pts / trace_ms * 1e3, "attempts_per_ray": att / max(n_pts, 1),
            "refine_image_reads_GBps": 2.0 * n_pix / (refine_ms * 1e-3) / 1e9,
            "trace_roofline": {"bound": "alu", "achieved": tflops, "peak": FP64_VECTOR_PEAK_TFLOPS,
                               "unit": "TFLOP/s", "frac": tflops / FP64_VECTOR_PEAK_TFLOPS,
                               "kernel": "trace_points_kernel"},
            "higher_order_fraction": float((pts["ncross"] >= 2).double().mean().item())}
    if cpu:
        from oracle import oracle as O
        sample = xy[::64].cpu().numpy()
        threads = oracle_threads()
        t0 = time.perf_counter()
        O.trace_points(img, sample, threads=threads)
        dt = time.perf_counter() - t0
        res["cpu_oracle"] = {"rays_per_s": len(sample) / dt, "cores": threads, "kind": "oracle",
                             "sample": f"every 64th subpixel ray ({len(sample)} rays, {dt:.1f} s)"}
    return res


def thick_measurement(steps: int, cpu: bool) -> dict:
    """Thick-disc image (Sec. 5.1-5.2) of the 1024x1024 cored-NFW screen with
    (R_s, H_0, h) = (8, 0.2, 0.1), p = 2: kernel time per image (HIP events on
    the stream) against the thin-disc trace of the same screen."""
    import torch

    from paper_2605_05635_amd import rt, workloads as W
    img = dict(W.cnfw_1024(), emis_pow=2.0)
    thick = rt.rt_thick_disc(8.0, 0.2, 0.1)
    outs = rt.alloc_outputs(img, reduce=False)
    for k in ("g_em", "intensity_n"):
        outs.pop(k)
    o = rt.out_from(outs)
    p = rt.params_from(img)
    stream = torch.cuda.current_stream()
    rt.rt_trace_thick(p, thick, o, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        rt.rt_trace_thick(p, thick, o, stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    n = img["nx"] * img["ny"]
    att = outs["attempts"].double().mean().item()
    from paper_2605_05635_amd import census
    # algorithmic flops: the trace's per attempt (crossings not counted) plus
    # five source evaluations per attempt and one per ray start; seven error terms
    m = img["metric"]
    flops = n * (att * (6 * census.flops_rhs(m) + census.flops_step_overhead()
                        + 5 * census.flops_thick_source(m) + 2 * 7)
                 + 20 + census.flops_rhs(m) + census.flops_thick_source(m))
    tflops = flops / (ms * 1e-3) / 1e12
    log(f"thick disc: {ms:.2f} ms per image, {att:.1f} attempts per ray, {tflops:.1f} TFLOP/s")
    res = {"workload": "cored-NFW 1024x1024 screen, thick disc (R_s, H_0, h) = (8, 0.2, 0.1), p = 2",
           "ms": ms, "rays_per_s": n / ms * 1e3, "steps": steps, "attempts_per_ray": att,
           "algorithmic_tflops": tflops, "frac_of_fp64_vector_peak": tflops / FP64_VECTOR_PEAK_TFLOPS,
           "flux_sum": float(outs["intensity"].sum().item())}
    if cpu:
        from oracle import oracle as O
        idx = W.subsample_indices(img["nx"], img["ny"], 16)
        threads = oracle_threads()
        t0 = time.perf_counter()
        O.trace_thick_pixels(img, (8.0, 0.2, 0.1), idx, threads=threads)
        dt = time.perf_counter() - t0
        res["cpu_oracle"] = {"rays_per_s": len(idx) / dt, "cores": threads, "kind": "oracle",
                             "sample": f"every 16th pixel in x and y ({len(idx)} rays, {dt:.1f} s)"}
    return res


def scan_measurement(steps: int, cpu: bool) -> dict:
    """Parameter scan (Sec. 2) over a 64 x 64 grid of cored-NFW points, chi in
    [0, 1.05] x eta in [0, 0.3] at lambda_c = 10, theta = 60 deg: wall time of
    rt_parameter_scan per call (HIP events on the stream)."""
    import numpy as np
    import torch

    from paper_2605_05635_amd import rt
    chi, eta = np.meshgrid(np.linspace(0.0, 1.05, 64), np.linspace(0.0, 0.3, 64))
    n = chi.size
    stream = torch.cuda.current_stream()
    out = rt.parameter_scan(["cnfw"] * n, chi.ravel(), eta.ravel(), 10.0, math.radians(60.0))
    host = (rt.rt_scan_point * n)()
    for i, (c, e) in enumerate(zip(chi.ravel(), eta.ravel())):
        host[i].metric, host[i].spin, host[i].theta = rt.RT_CNFW, float(c), math.radians(60.0)
        host[i].halo[0], host[i].halo[1] = float(e), 10.0
    pts = torch.frombuffer(bytearray(bytes(host)), dtype=torch.uint8).to("cuda")
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        rt.rt_parameter_scan(pts, out, stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    o = out.cpu().numpy()
    log(f"parameter scan: {n} points in {ms:.2f} ms")
    res = {"workload": "cored-NFW 64 x 64 grid of (chi, eta), lambda_c = 10, ergosurface at 60 deg",
           "ms": ms, "points_per_s": n / ms * 1e3, "steps": steps,
           "with_horizon": int(np.isfinite(o[:, 0]).sum()),
           "chi_e_range": [float(np.nanmin(o[:, 2])), float(np.nanmax(o[:, 2]))]}
    if cpu:
        from oracle import oracle as O
        pick = list(range(0, n, n // 16))
        t0 = time.perf_counter()
        O.parameter_scan([("cnfw", float(chi.ravel()[i]), float(eta.ravel()[i]), 10.0,
                           math.radians(60.0)) for i in pick])
        dt = time.perf_counter() - t0
        res["cpu_oracle"] = {"points_per_s": len(pick) / dt, "cores": 1, "kind": "oracle",
                             "sample": f"every {n // 16}th point ({len(pick)} points, {dt:.1f} s)"}
    return res


def shadow_measurement(steps: int, cpu: bool) -> dict:
    """Shadow boundary (Sec. 4.1) of the benchmark spacetime and observer along
    4096 screen directions, b in [2, 9] M to a bracket of 1e-10 M, with the
    library's sample count for that many directions (16 per pass on 256 compute
    units: four directions per wavefront): wall time of rt_shadow_boundary per
    call (HIP events on the stream)."""
    import numpy as np
    import torch

    from paper_2605_05635_amd import rt, workloads as W
    img = W.cnfw_1024()
    n, b_lo, b_hi, b_tol = 4096, 2.0, 9.0, 1e-10
    S = rt.rt_shadow_boundary_samples(n)
    psi = (np.arange(n) + 0.5) * (2.0 * np.pi / n)
    dirs = np.stack([np.cos(psi), np.sin(psi)], axis=1)
    d = torch.tensor(dirs, device="cuda")
    stream = torch.cuda.current_stream()
    out = torch.empty(n, 2, dtype=torch.float64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    att = torch.empty(n, dtype=torch.int64, device="cuda")
    p = rt.params_from(img)
    rt.rt_shadow_boundary(p, d, b_lo, b_hi, b_tol, out, st, att, stream, samples=S)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        rt.rt_shadow_boundary(p, d, b_lo, b_hi, b_tol, out, st, att, stream, samples=S)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    bc = out.mean(dim=1).cpu().numpy()
    passes = int(np.ceil(np.log((b_hi - b_lo) / b_tol) / np.log(S + 1.0)))
    rays = n * S * passes + 2 * n
    attempts = float(att.sum().item())
    from paper_2605_05635_amd import census
    # algorithmic flops as for the trace kernel, without the crossings (not counted)
    flops = (attempts * (6 * census.flops_rhs(img["metric"]) + census.flops_step_overhead())
             + rays * (20 + census.flops_rhs(img["metric"])))
    tflops = flops / (ms * 1e-3) / 1e12
    log(f"shadow boundary: {n} directions in {ms:.2f} ms, {attempts / rays:.0f} attempts per ray")
    res = {"workload": "cored-NFW benchmark spacetime, 4096 directions, b in [2, 9], "
                       f"bracket 1e-10 ({S}-point multisection)", "samples": S,
           "ms": ms, "directions_per_s": n / ms * 1e3, "steps": steps,
           "passes": passes, "rays_traced": rays, "attempts_per_ray": attempts / rays,
           "algorithmic_tflops": tflops, "frac_of_fp64_vector_peak": tflops / FP64_VECTOR_PEAK_TFLOPS,
           "all_found": bool((st == 0).all().item()),
           "b_mean": float(bc.mean()), "b_min": float(bc.min()), "b_max": float(bc.max())}
    if cpu:
        from oracle import oracle as O
        threads = oracle_threads()
        pick = np.arange(0, n, n // 16)
        t0 = time.perf_counter()
        O.shadow_boundary(img, dirs[pick], b_lo, b_hi, b_tol, threads=threads)
        dt = time.perf_counter() - t0
        res["cpu_oracle"] = {"directions_per_s": len(pick) / dt, "cores": threads,
                             "kind": "oracle",
                             "sample": f"every {n // 16}th direction ({len(pick)} directions, "
                                       f"{dt:.1f} s)"}
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    # the GPU's clock settles over the first launches of a run (a cold first
    # trace ~2x, then ~10 % above the steady time for another four or five)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=1)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-image batched trace + visibility measurement")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision measurement")
    ap.add_argument("--no-thick", action="store_true",
                    help="skip the thick-disc measurement")
    ap.add_argument("--no-scan", action="store_true",
                    help="skip the parameter-scan measurement")
    ap.add_argument("--no-diagnostics", action="store_true",
                    help="skip the image-diagnostics measurement")
    ap.add_argument("--no-shadow", action="store_true",
                    help="skip the shadow-boundary measurement")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the image-gradient measurement")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the adaptive-screen (band-edge refinement) measurement")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after the timed steps, run one plain device-to-device copy of this "
                         "many MiB (the reference kernel for HBM byte counters) and report it")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the ray tracer runs on a single MI355X "
              "(rays are independent: across GPUs the screen's tiles would be split)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2605_05635_amd import census, rt, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    img = W.cnfw_1024("fp64")
    n_rays = img["nx"] * img["ny"]
    outs = rt.alloc_outputs(img)
    params, o = [rt.params_from(img)], [rt.out_from(outs)]
    stream = torch.cuda.current_stream()

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        rt.rt_trace_image(params, o, stream)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    stops = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for ev in starts + stops:      # torch creates the hipEvent_t at its first record
        ev.record(stream)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        rt.rt_set_kernel_timing(starts[k], stops[k])
        rt.rt_trace_image(params, o, stream)
    rt.rt_set_kernel_timing(None, None)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in zip(starts, stops)]
    ms_per_step = 1e3 * wall / args.steps
    value = n_rays * args.steps / wall
    log(f"{ms_per_step:.3f} ms/step, trace kernel {np.mean(kernel_ms):.3f} ms")

    attempts = outs["attempts"].double().sum().item()
    crossings = outs["ncross"].double().sum().item()
    flops = (attempts * (6 * census.flops_rhs(img["metric"]) + census.flops_step_overhead())
             + crossings * census.flops_crossing()
             + n_rays * (20 + census.flops_rhs(img["metric"])))
    k_s = float(np.mean(kernel_ms)) * 1e-3
    achieved = flops / k_s / 1e12
    from paper_2605_05635_amd.profiling import trace_source_hash
    khash = trace_source_hash()
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": measured_traffic(khash),
                "kernel": "trace_kernel<CNFW_NEAR> (cored NFW, 0 <= eta <= 0.34)",
                "kernel_ms": float(np.mean(kernel_ms)),
                "flops_per_launch": flops, "kernel_source_hash": khash}

    line = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "cored-NFW 1024x1024 screen, FP64 trace", "metric": img["metric"],
                   "spin": img["spin"], "eta": img["halo"][0], "lambda_c": img["halo"][1],
                   "incl_deg": 163.0, "r_obs": img["r_obs"], "screen": "+-10 M",
                   "rtol": img["rtol"], "atol": img["atol"], "rays": n_rays},
        "fp64_rays_per_s": value,
        "attempts_per_ray": attempts / n_rays,
        "roofline": roofline,
    }
    mixed_outs = None
    if not args.no_mixed:
        line["mixed"], mixed_outs = mixed_measurement(max(2, args.steps // 2), outs)
        line["mixed_rays_per_s"] = line["mixed"]["rays_per_s"]
    if not args.no_batch:
        line["batch_64"] = batch_measurement(max(2, args.steps // 4))
    if not args.no_adjoint:
        line["adjoint"] = adjoint_measurement(max(2, args.steps // 2), not args.no_cpu_baseline)
    if not args.no_diagnostics:
        line["diagnostics"] = diagnostics_measurement(args.steps, outs, img, not args.no_cpu_baseline)
    if not args.no_adaptive:
        line["adaptive_screen"] = adaptive_measurement(max(2, args.steps // 2), outs, img,
                                                       not args.no_cpu_baseline)
    if not args.no_thick:
        line["thick_disc"] = thick_measurement(max(2, args.steps // 2), not args.no_cpu_baseline)
    if not args.no_scan:
        line["parameter_scan"] = scan_measurement(max(2, args.steps // 2), not args.no_cpu_baseline)
    if not args.no_shadow:
        line["shadow_boundary"] = shadow_measurement(max(2, args.steps // 4), not args.no_cpu_baseline)
    if args.calibration_copy_mib > 0:
        nbytes = args.calibration_copy_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = nbytes
        log(f"calibration copy: {nbytes} bytes read and {nbytes} bytes written")
    if not args.no_cpu_baseline:
        line["cpu_baseline"], ref, idx = cpu_baseline(img, args.cpu_stride)
        # the oracle's trace of the same pixels, against the GPU images
        line["fp64_error_vs_oracle"] = error_vs_oracle(outs, ref, idx)
        if mixed_outs is not None:
            line["mixed"]["error_vs_oracle"] = error_vs_oracle(mixed_outs, ref, idx)
        log(f"error vs oracle: fp64 {line['fp64_error_vs_oracle']}")
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
