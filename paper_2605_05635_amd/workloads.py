"""Seeded synthetic workloads (screens and spacetime parameters).

This module only draws and lists parameters: it holds none of the ray
tracer's arithmetic, so both the HIP path and the CPU oracle can take their
inputs from it.  Every image is a plain ``dict`` with the keys below; each
side converts it to its own parameter struct.

Keys
    metric          "kerr" | "einasto" | "cnfw"
    spin            chi = a/M
    halo            (lambda_E, 0) for Einasto, (eta, lambda_c) for cored NFW
    incl            observer inclination theta_o [rad]
    r_obs           observer radius R_o
    nx, ny          pixels; pixel (ix, iy) sits at the centre
                    X = x_min + (ix + 1/2)(x_max - x_min)/nx, likewise Y
    x_min .. y_max  screen extent
    rtol, atol      Dormand-Prince tolerances
    r_stop_fac      capture radius factor (times R_+)
    r_esc_fac       escape radius factor (times R_o)
    r_in, r_out     disc window; r_in <= 0 means the outer horizon
    emis_pow        emissivity exponent p in R^-p
    sigma_in/out    tanh taper widths; 0 means hard edges
    max_attempts    step-attempt budget per ray
    h0              first trial step
    precision       "fp64" | "mixed"

The five workloads follow the paper's parameter choices where it states
them (chi, theta_o, observer radius, screen conventions) and seeded draws in
its representative ranges where it does not.
"""
from __future__ import annotations

import math

import numpy as np

METRICS = ("kerr", "einasto", "cnfw")

BASE = dict(
    metric="kerr", spin=0.5, halo=(0.0, 0.0), incl=math.radians(17.0), r_obs=1000.0,
    nx=64, ny=64, x_min=-12.0, x_max=12.0, y_min=-12.0, y_max=12.0,
    rtol=1e-8, atol=1e-8, r_stop_fac=1.01, r_esc_fac=1.1,
    r_in=0.0, r_out=20.0, emis_pow=3.0, sigma_in=0.0, sigma_out=0.0,
    max_attempts=20000, h0=1.0, precision="fp64",
)


def image(**kw) -> dict:
    """A parameter dict: BASE overridden by keyword arguments."""
    d = dict(BASE)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(f"unknown image parameter {k!r}")
        d[k] = v
    d["halo"] = tuple(float(h) for h in d["halo"])
    return d


def kerr_small() -> dict:
    """Kerr chi=0.5, theta_o=17 deg, R_o=1000, 64x64 over +-12 M, FP64 1e-8."""
    return image()


def einasto_512(seed: int = 2) -> dict:
    """Einasto-type chi=0.9, theta_o=60 deg, 512x512 over +-10 M.

    lambda_E ~ U[0.10, 0.18] (extremal spin above 0.93 on that range)."""
    rng = np.random.default_rng(seed)
    lam = float(rng.uniform(0.10, 0.18))
    return image(metric="einasto", spin=0.9, halo=(lam, 0.0), incl=math.radians(60.0),
                 nx=512, ny=512, x_min=-10.0, x_max=10.0, y_min=-10.0, y_max=10.0)


def cnfw_1024(precision: str = "fp64") -> dict:
    """Cored NFW (eta, lambda_c) = (0.02, 10), chi=0.94, theta_o=163 deg,
    1024x1024 over +-10 M."""
    return image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=math.radians(163.0),
                 nx=1024, ny=1024, x_min=-10.0, x_max=10.0, y_min=-10.0, y_max=10.0,
                 precision=precision)


def cnfw_adjoint_256() -> dict:
    """Cored NFW chi=0.94, theta_o=60 deg, 256x256 over +-10 M, tapered disc
    window sigma_in = sigma_out = 0.5 (the image-gradient workload)."""
    return image(metric="cnfw", spin=0.94, halo=(0.02, 10.0), incl=math.radians(60.0),
                 nx=256, ny=256, x_min=-10.0, x_max=10.0, y_min=-10.0, y_max=10.0,
                 sigma_in=0.5, sigma_out=0.5)


def adjoint_target_signs(seed: int = 4) -> np.ndarray:
    """Signs s_i in {-1, +1} of the 1 % perturbation of (chi, theta_o, rho_s, r_s)."""
    rng = np.random.default_rng(seed)
    return np.where(rng.integers(0, 2, size=4) == 0, -1.0, 1.0)


def batch_64(einasto_extremal_spin, seed: int = 5, n_images: int = 64) -> list[dict]:
    """64 images of mixed resolution and metric for one batched launch.

    res ~ U{128, 256, 512, 768}^2, chi ~ U[0, 0.99], theta_o ~ U[5, 85] deg,
    metric ~ U{Kerr, Einasto, cored NFW}; Einasto lambda_E drawn from
    U[0.05, 0.30] again until the spacetime keeps a horizon with a margin,
    einasto_extremal_spin(lambda_E) >= chi + 0.005 (the caller supplies the
    extremal spin of the Einasto seed: this module computes nothing of the
    spacetimes); cored NFW eta ~ U[0.005, 0.05], lambda_c ~ U[5, 20] (extremal
    spin above 1 there); screen +-12 M."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_images):
        res = int(rng.choice([128, 256, 512, 768]))
        chi = float(rng.uniform(0.0, 0.99))
        incl = math.radians(float(rng.uniform(5.0, 85.0)))
        metric = METRICS[int(rng.integers(0, 3))]
        if metric == "einasto":
            while True:
                lam = float(rng.uniform(0.05, 0.30))
                if einasto_extremal_spin(lam) >= chi + 0.005:
                    break
            halo = (lam, 0.0)
        elif metric == "cnfw":
            halo = (float(rng.uniform(0.005, 0.05)), float(rng.uniform(5.0, 20.0)))
        else:
            halo = (0.0, 0.0)
        out.append(image(metric=metric, spin=chi, halo=halo, incl=incl, nx=res, ny=res,
                         x_min=-12.0, x_max=12.0, y_min=-12.0, y_max=12.0))
    return out


def random_small_images(seed: int, n: int) -> list[dict]:
    """n small screens (5-14 x 4-12 pixels, possibly off-centre) with seeded
    draws over the parameter space: metric, spin in [-0.9, 0.9] (below every
    halo's extremal spin for these halo ranges), inclination in [3, 177] deg,
    observer radius in [300, 1000], tolerance 10^U[-10, -6], emission window,
    exponent and tapers; Einasto lambda_E in [0.10, 0.18], cored-NFW eta in
    [0, 0.3] and lambda_c in [3, 20]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        m = METRICS[int(rng.integers(3))]
        halo = ((float(rng.uniform(0.10, 0.18)), 0.0) if m == "einasto" else
                (float(rng.uniform(0.0, 0.3)), float(rng.uniform(3.0, 20.0))) if m == "cnfw" else
                (0.0, 0.0))
        half = float(rng.uniform(4.0, 15.0))
        cx, cy = rng.uniform(-3.0, 3.0, size=2)
        tol = float(10.0 ** rng.uniform(-10.0, -6.0))
        taper = bool(rng.integers(2))
        sig = float(rng.uniform(0.2, 1.0))
        out.append(image(
            metric=m, spin=float(rng.uniform(-0.9, 0.9)), halo=halo,
            incl=math.radians(float(rng.uniform(3.0, 177.0))), r_obs=float(rng.uniform(300.0, 1000.0)),
            nx=int(rng.integers(5, 15)), ny=int(rng.integers(4, 13)),
            x_min=float(cx - half), x_max=float(cx + half), y_min=float(cy - half), y_max=float(cy + half),
            rtol=tol, atol=tol, r_in=float(rng.uniform(2.0, 6.0)) if rng.integers(2) else 0.0,
            r_out=float(rng.uniform(12.0, 30.0)), emis_pow=float(rng.uniform(2.0, 3.5)),
            sigma_in=sig if taper else 0.0, sigma_out=sig if taper else 0.0))
    return out


def uv_points(seed: int, k: int = 2000) -> np.ndarray:
    """k seeded (u, v) baselines [cycles/M]: |q| ~ U[0, 0.5], angle ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    q = rng.uniform(0.0, 0.5, size=k)
    a = rng.uniform(0.0, 2.0 * math.pi, size=k)
    return np.stack([q * np.cos(a), q * np.sin(a)], axis=1)


def screen_points(seed: int, n: int, half_width: float = 10.0) -> np.ndarray:
    """n seeded screen points (X, Y) [M]: half uniform over the square
    [-half_width, half_width]^2, half in the annulus 4 <= sqrt(X^2 + Y^2) <= 6
    around the photon ring (where rays cross the equator more than once)."""
    rng = np.random.default_rng(seed)
    m = n // 2
    sq = rng.uniform(-half_width, half_width, size=(m, 2))
    r = np.sqrt(rng.uniform(16.0, 36.0, size=n - m))
    a = rng.uniform(0.0, 2.0 * math.pi, size=n - m)
    return np.concatenate([sq, np.stack([r * np.cos(a), r * np.sin(a)], axis=1)])


def band_maps(seed: int, nx: int, ny: int, block: int = 3) -> tuple[np.ndarray, np.ndarray]:
    """Seeded synthetic N_cross and status maps ([ny][nx] uint8) made of
    block x block runs of equal values, so that band edges and interiors both
    occur (inputs for the screen refinement)."""
    rng = np.random.default_rng(seed)
    by, bx = (ny + block - 1) // block, (nx + block - 1) // block
    nc = np.repeat(np.repeat(rng.integers(0, 4, (by, bx)), block, 0), block, 1)[:ny, :nx]
    st = np.repeat(np.repeat(rng.integers(1, 3, (by, bx)), block + 1, 0), block + 1, 1)[:ny, :nx]
    return nc.astype(np.uint8), st.astype(np.uint8)


def subsample_indices(nx: int, ny: int, stride: int, offset: int = 0) -> np.ndarray:
    """Row-major pixel indices of a strided sub-grid (every `stride`-th pixel in
    x and y), used to sample a large screen."""
    iy, ix = np.meshgrid(np.arange(offset % stride, ny, stride),
                         np.arange(offset % stride, nx, stride), indexing="ij")
    return (iy * nx + ix).reshape(-1).astype(np.int64)


def random_pixels(nx: int, ny: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct seeded pixel indices of an nx x ny screen."""
    rng = np.random.default_rng(seed)
    count = min(count, nx * ny)
    return np.sort(rng.choice(nx * ny, size=count, replace=False)).astype(np.int64)
