"""Autotuner of the trace kernels' work distribution.

Grid search over the launch configuration of include/rt.h (pixels per
work-queue claim, tile shape of the pixel enumeration, resident workgroups
per compute unit), timed with HIP events on the GPU, for one workload (a list
of images).  The best configuration is cached per device and workload
signature in a JSON file (default: ~/.cache/paper_2605_05635_amd/autotune.json,
override with RT_AUTOTUNE_CACHE) and applied with rt_set_launch_config.
The configuration never changes a traced value, only the speed.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import rt

CHUNKS = (32, 64, 128, 256)
TILES = ((0, 0), (8, 8), (16, 4))
BLOCKS_PER_CU = (0, 1)


def cache_path() -> str:
    return os.environ.get("RT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache",
                                       "paper_2605_05635_amd", "autotune.json"))


def signature(imgs: list[dict]) -> str:
    """Workload key: metric, screen size and spin of every image (the quantities
    that set the per-ray cost distribution)."""
    key = [(i["metric"], int(i["nx"]), int(i["ny"]), round(float(i["spin"]), 6),
            round(float(i["incl"]), 6)) for i in imgs]
    return hashlib.sha256(json.dumps(key).encode()).hexdigest()[:20]


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device())


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_config(imgs: list[dict], outs: list, cfg: tuple, repeats: int = 2) -> float:
    """Median milliseconds of one trace of `imgs` under `cfg`."""
    import torch
    chunk, (tw, th), bpc = cfg
    rt.rt_set_launch_config(chunk, tw, th, bpc)
    params = [rt.params_from(i) for i in imgs]
    ouv = [rt.out_from(o) for o in outs]
    stream = torch.cuda.current_stream()
    rt.rt_trace_image(params, ouv, stream)          # warm
    times = []
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        rt.rt_trace_image(params, ouv, stream)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return sorted(times)[len(times) // 2]


def tune(imgs: list[dict], force: bool = False, log=None) -> dict:
    """Best launch configuration for the workload, from the cache or by grid
    search; applies it and returns it (with its time in ms)."""
    key = f"{_device_name()}|{signature(imgs)}"
    cache = _load()
    if not force and key in cache:
        best = cache[key]
    else:
        outs = [rt.alloc_outputs(i) for i in imgs]
        results = []
        for chunk in CHUNKS:
            for tile in TILES:
                for bpc in BLOCKS_PER_CU:
                    ms = time_config(imgs, outs, (chunk, tile, bpc))
                    results.append((ms, chunk, tile, bpc))
                    if log:
                        log(f"autotune chunk={chunk} tile={tile} blocks/CU={bpc}: {ms:.3f} ms")
        ms, chunk, tile, bpc = min(results)
        best = dict(chunk=chunk, tile_w=tile[0], tile_h=tile[1], blocks_per_cu=bpc, ms=ms,
                    searched=len(results))
        cache[key] = best
        _store(cache)
    rt.rt_set_launch_config(best["chunk"], best["tile_w"], best["tile_h"],
                            best["blocks_per_cu"])
    return best
