"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2605_05635_amd.profiling stats KERNEL_STATS_CSV --command CMD --out TXT
        [--trace KERNEL_TRACE_CSV --skip N]
    python -m paper_2605_05635_amd.profiling counters COUNTER_CSV --kernel SUBSTRING
        --command CMD --out TXT
    python -m paper_2605_05635_amd.profiling traffic --fetch CSV --write CSV
        --kernel SUBSTRING --copy-bytes N --command CMD --out JSON

`stats` condenses a `rocprofv3 --kernel-trace --stats --output-format csv`
kernel_stats table (calls, total and average duration per kernel); with
`--trace KERNEL_TRACE_CSV --skip N` (the same run's kernel_trace table) it adds
each kernel's average over its dispatches after the first N, the untimed
warm-up launches of a bench run, while the GPU's clock settles, and each
kernel's launch resources.
`traffic` turns two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs
(KiB per dispatch) into HBM bytes per launch of one kernel, each counter
scaled by what it reads for a plain device-to-device copy of known size run
in the same process (the largest dispatch whose name contains "copy"), and
records the hash of the trace kernel's sources it was taken on.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
TRACE_SOURCES = ("rt_trace.hip", "rt_ray.h", "rt_device.h", "rt_math.h", "rt_dual.h",
                 "rt_kernels.h")


def code_tokens(text: str) -> str:
    """C++ source without its comments, its whitespace runs collapsed to one
    space: what the compiler sees, so that an edit of comments or layout
    keeps the hash (string and character literals are kept as written)."""
    out = []
    i, n = 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def trace_source_hash() -> str:
    """Hash of the code (comments and layout aside) of the sources the
    single-image trace kernel is compiled from."""
    h = hashlib.sha256()
    for name in TRACE_SOURCES:
        with open(os.path.join(PKG, "csrc", name), encoding="utf-8") as f:
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


def _rows(path: str) -> list[dict]:
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def kernel_stats(path: str) -> list[dict]:
    out = []
    for r in _rows(path):
        out.append(dict(name=r["Name"], calls=int(r["Calls"]),
                        total_ms=float(r["TotalDurationNs"]) * 1e-6,
                        avg_ms=float(r["AverageNs"]) * 1e-6,
                        min_ms=float(r["MinNs"]) * 1e-6, max_ms=float(r["MaxNs"]) * 1e-6,
                        pct=float(r["Percentage"])))
    return sorted(out, key=lambda d: -d["total_ms"])


def stats_text(path: str, command: str, top: int = 20) -> str:
    ks = kernel_stats(path)
    lines = [f"command: {command}", "",
             f"{'calls':>6} {'total ms':>10} {'avg ms':>10} {'min ms':>10} {'max ms':>10} "
             f"{'%':>6}  kernel"]
    for k in ks[:top]:
        name = k["name"] if len(k["name"]) <= 110 else k["name"][:107] + "..."
        lines.append(f"{k['calls']:>6} {k['total_ms']:>10.3f} {k['avg_ms']:>10.4f} "
                     f"{k['min_ms']:>10.4f} {k['max_ms']:>10.4f} {k['pct']:>6.2f}  {name}")
    return "\n".join(lines) + "\n"


def settled_text(trace_csv: str, skip: int, top: int = 8) -> str:
    """Per-kernel average duration over the dispatches after the first `skip`
    of each kernel (dispatch order), from a kernel_trace table."""
    runs: dict[str, list[tuple[int, float]]] = {}
    for r in _rows(trace_csv):
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
        runs.setdefault(r["Kernel_Name"], []).append((int(r["Dispatch_Id"]), d))
    rows = []
    for name, v in runs.items():
        v.sort()
        kept = [d for _, d in v[skip:]]
        if kept:
            rows.append((sum(kept), len(kept), min(kept), max(kept), name))
    rows.sort(key=lambda t: -t[0])
    lines = ["", f"after the first {skip} dispatches of each kernel (from the kernel trace):",
             f"{'calls':>6} {'avg ms':>10} {'min ms':>10} {'max ms':>10}  kernel"]
    for tot, n, lo, hi, name in rows[:top]:
        name = name if len(name) <= 110 else name[:107] + "..."
        lines.append(f"{n:>6} {tot / n:>10.4f} {lo:>10.4f} {hi:>10.4f}  {name}")
    return "\n".join(lines) + "\n"


def resources_text(trace_csv: str, top: int = 8) -> str:
    """Per-kernel launch resources as the kernel trace records them (register
    counts as rocprofv3 reports them, LDS and scratch bytes, workgroup and grid
    sizes) and the wavefronts per SIMD the grid puts on a 256-CU, 4-SIMD
    device when every workgroup is resident at once (the persistent kernels)."""
    seen: dict[str, dict] = {}
    for r in _rows(trace_csv):
        seen.setdefault(r["Kernel_Name"], r)
    lines = ["", "launch resources (from the kernel trace; waves/SIMD = grid wavefronts / 1024 SIMDs):",
             f"{'VGPR':>5} {'SGPR':>5} {'LDS B':>7} {'scratch':>8} {'wg':>5} {'grid':>9} "
             f"{'waves/SIMD':>10}  kernel"]
    for name, r in list(seen.items())[:top]:
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        name = name if len(name) <= 90 else name[:87] + "..."
        lines.append(f"{r['VGPR_Count']:>5} {r['SGPR_Count']:>5} {r['LDS_Block_Size']:>7} "
                     f"{r['Scratch_Size']:>8} {r['Workgroup_Size_X']:>5} {grid:>9} "
                     f"{grid / 64 / 1024:>10.2f}  {name}")
    return "\n".join(lines) + "\n"


def _counter(path: str, name: str) -> list[tuple[str, float]]:
    return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in _rows(path)
            if r["Counter_Name"] == name]


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int) -> dict:
    res = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"),
                               ("write", write_csv, "WRITE_SIZE")):
        rows = _counter(path, counter)
        kern = [v for n, v in rows if kernel in n]
        copies = [v for n, v in rows if "copy" in n.lower()]
        if not kern or not copies:
            raise SystemExit(f"{counter}: no dispatch of {kernel!r} or of a copy kernel")
        kib = sum(kern) / len(kern)
        copy_kib = max(copies)
        scale = copy_bytes / (copy_kib * 1024.0)
        res[key] = dict(counter_kib_per_launch=kib, launches=len(kern),
                        copy_counter_kib=copy_kib, scale=scale,
                        bytes_per_launch=kib * 1024.0 * scale)
    res["hbm_bytes_per_launch"] = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    return res


def counters_text(path: str, kernel: str, command: str) -> str:
    """Average of every counter over the dispatches of `kernel` (a substring
    of the kernel name) in a `rocprofv3 --pmc` counter_collection table."""
    acc: dict[str, list[float]] = {}
    name = None
    for r in _rows(path):
        if kernel in r["Kernel_Name"]:
            name = r["Kernel_Name"]
            acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if not acc:
        raise SystemExit(f"no dispatch of {kernel!r}")
    lines = [f"command: {command}", f"kernel: {name}", ""]
    for k in sorted(acc):
        v = acc[k]
        lines.append(f"{k:32s} {sum(v) / len(v):>22.1f}   (mean of {len(v)} dispatches)")
    return "\n".join(lines) + "\n"


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    a.add_argument("--out", required=True)
    a.add_argument("--trace")
    a.add_argument("--skip", type=int, default=0)
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--kernel", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--out", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--command", required=True)
    b.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        with open(args.out, "w") as f:
            f.write(stats_text(args.csv, args.command))
            if args.trace:
                f.write(settled_text(args.trace, args.skip))
                f.write(resources_text(args.trace))
        return 0
    if args.cmd == "counters":
        with open(args.out, "w") as f:
            f.write(counters_text(args.csv, args.kernel, args.command))
        return 0
    t = traffic(args.fetch, args.write, args.kernel, args.copy_bytes)
    t.update(kernel=args.kernel, command=args.command, kernel_source_hash=trace_source_hash(),
             copy_bytes=args.copy_bytes)
    with open(args.out, "w") as f:
        json.dump(t, f, indent=1)
        f.write("\n")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
