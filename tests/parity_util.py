"""Element-by-element comparison of the HIP path's outputs with the oracle's.

Tolerances (stated once, used by every parity test):
  * N_cross and status: identical (integer outputs are bit-exact).
  * crossing records n < min(N_cross, 3): R_em and phi_em within 1e-6 absolute,
    T_em within 1e-6 * max(1, |T_em|) (T grows to ~2 R_o), g_em within 1e-9
    relative; records n >= min(N_cross, 3) NaN on both sides.
  * intensity I and I_n: within 1e-6 relative where the oracle's value is
    non-zero, exactly 0 where it is 0.
The accuracy of both sides against the exact geodesic is a separate matter
(bounded by the integration tolerance, see test_oracle_geodesics.py); these
tolerances bound the difference of two implementations of the same discrete
method, which differ only by rounding.
"""
from __future__ import annotations

import numpy as np

R_ABS = 1e-6
PHI_ABS = 1e-6
T_REL = 1e-6
G_REL = 1e-9
I_REL = 1e-6


def gpu_to_numpy(outs: dict, idx: np.ndarray | None = None) -> dict:
    """Device outputs -> numpy, flattened to pixels (maps as (3, n)), optionally
    sampled at pixel indices idx."""
    res = {}
    for k, t in outs.items():
        if k == "reduce":
            res[k] = t.cpu().numpy()
            continue
        a = t.cpu().numpy()
        a = a.reshape(3, -1) if a.ndim == 3 else a.reshape(-1)
        if idx is not None:
            a = a[:, idx] if a.ndim == 2 else a[idx]
        res[k] = a
    return res


def compare(gpu: dict, orc: dict, emission: bool = True) -> list[str]:
    """Returns a list of human-readable mismatches (empty means parity)."""
    bad = []
    n = orc["ncross"].size
    nc_g = gpu["ncross"].astype(np.int64)
    nc_o = orc["ncross"].astype(np.int64)
    st_g, st_o = gpu["status"].astype(np.int64), orc["status"].astype(np.int64)
    for name, a, b in (("ncross", nc_g, nc_o), ("status", st_g, st_o)):
        w = np.nonzero(a != b)[0]
        if w.size:
            bad.append(f"{name}: {w.size}/{n} pixels differ, first at {w[:8].tolist()} "
                       f"gpu={a[w[:8]].tolist()} oracle={b[w[:8]].tolist()}")
    same = (nc_g == nc_o) & (st_g == st_o)
    rec = np.minimum(nc_o, 3)
    for j in range(3):
        have = same & (rec > j)
        none = same & (rec <= j)
        checks = [("r_em", R_ABS, 0.0), ("phi_em", PHI_ABS, 0.0), ("t_em", 0.0, T_REL)]
        if emission:
            checks += [("g_em", 1e-15, G_REL)]
        for key, aabs, rel in checks:
            if key not in gpu:
                continue
            g, o = gpu[key][j], orc[key][j]
            tol = aabs + rel * np.maximum(1.0 if key == "t_em" else np.abs(o), np.abs(o))
            diff = np.abs(g - o)
            w = np.nonzero(have & ~(diff <= tol))[0]
            if w.size:
                bad.append(f"{key}[{j}]: {w.size} pixels off, worst {np.nanmax(diff[w]):.3e} "
                           f"at {w[np.nanargmax(diff[w])]}")
            w = np.nonzero(none & ~(np.isnan(g) & np.isnan(o)))[0]
            if w.size:
                bad.append(f"{key}[{j}]: {w.size} pixels should be NaN")
    if emission:
        for key in ("intensity",):
            g, o = gpu[key], orc[key]
            nz = same & (o != 0)
            w = np.nonzero(nz & ~(np.abs(g - o) <= I_REL * np.abs(o)))[0]
            if w.size:
                rel = np.abs(g[w] - o[w]) / np.abs(o[w])
                bad.append(f"{key}: {w.size} pixels off, worst rel {rel.max():.3e}")
            w = np.nonzero(same & (o == 0) & (g != 0))[0]
            if w.size:
                bad.append(f"{key}: {w.size} pixels should be exactly 0")
        for j in range(3):
            g, o = gpu["intensity_n"][j], orc["i_n"][j]
            have = same & (rec > j)
            nz = have & (o != 0)
            w = np.nonzero(nz & ~(np.abs(g - o) <= I_REL * np.abs(o)))[0]
            if w.size:
                bad.append(f"intensity_n[{j}]: {w.size} pixels off")
            w = np.nonzero(have & (o == 0) & (g != 0))[0]
            if w.size:
                bad.append(f"intensity_n[{j}]: {w.size} pixels should be 0")
    return bad


def summary(gpu: dict, orc: dict) -> str:
    a_g, a_o = gpu["attempts"].astype(np.int64), orc["attempts"].astype(np.int64)
    same_att = float(np.mean(a_g == a_o))
    return (f"n={a_o.size} ncross hist={np.bincount(orc['ncross'].astype(np.int64)).tolist()} "
            f"attempts mean gpu={a_g.mean():.2f} oracle={a_o.mean():.2f} "
            f"identical step counts on {100 * same_att:.2f}% of rays")
