"""Seeded synthetic inputs for the footprint and patch-transfer workloads:
a flight's GNSS/IMU poses over a digital surface model (DSM) raster, and the
image's patch grid.  Inputs only: no footprint, overlap or transfer
arithmetic lives here.

The DSM samples the flight's terrain (a sum of Gaussian hills, as in the
cluster scenes) on a square grid of `cell` metres (12 m: the TanDEM-X
posting named in Sec. 3.1) and stores heights as float32."""
from __future__ import annotations

import math

import numpy as np

from synth import aerial as A


def make_geo_flight(seed: int = 21, n_strips: int = 4, imgs_per_strip: int = 40, cell: float = 12.0,
                    n_hills: int = 8, pos_noise_m: float = 0.5, att_noise_deg: float = 0.05,
                    jitter_deg: float = 1.0) -> dict:
    """Poses (R camera->world, T centre) of a boustrophedon flight with
    GNSS/IMU noise, and the DSM raster covering the flight with one footprint
    of margin.  Raster node (i, j) sits at (x0 + i cell, y0 + j cell); h is
    [ny][nx] (row j = y)."""
    spec = A.SceneSpec(n_strips=n_strips, imgs_per_strip=imgs_per_strip, n_hills=n_hills, jitter_deg=jitter_deg)
    rng = np.random.Generator(np.random.PCG64(seed))
    R_t, T_t, strip = A.flight_poses(spec, rng)
    lo = T_t[:, :2].min(0) - np.array([A.FOOT_ACROSS, A.FOOT_ALONG])
    hi = T_t[:, :2].max(0) + np.array([A.FOOT_ACROSS, A.FOOT_ALONG])
    terrain = A.Terrain(rng, lo, hi, n_hills)
    nx = int(math.ceil((hi[0] - lo[0]) / cell)) + 1
    ny = int(math.ceil((hi[1] - lo[1]) / cell)) + 1
    gx, gy = np.meshgrid(lo[0] + cell * np.arange(nx), lo[1] + cell * np.arange(ny))
    h = terrain.height(np.stack([gx.ravel(), gy.ravel()], 1)).reshape(ny, nx).astype(np.float32)
    C = R_t.shape[0]
    T = T_t + rng.normal(0.0, pos_noise_m, (C, 3))
    R = np.stack([R_t[k] @ A.rotvec_to_matrix(rng.normal(0.0, att_noise_deg * A.DEG, 3)) for k in range(C)])
    return {"n_images": C, "R": np.ascontiguousarray(R), "T": np.ascontiguousarray(T), "strip": strip,
            "dsm": {"nx": nx, "ny": ny, "x0": float(lo[0]), "y0": float(lo[1]), "cell": float(cell),
                    "h": np.ascontiguousarray(h)},
            "f": A.F_PX, "cx": A.CX, "cy": A.CY, "width": A.IMG_W, "height": A.IMG_H}


def flight_dsm(fl: dict, cell: float = 12.0) -> dict:
    """The DSM raster of a generated flight's own terrain (fl["truth"]
    ["terrain"], the hills its tie points lie on), covering its cameras with
    one footprint of margin, heights as float32."""
    T = np.asarray(fl["truth"]["T"])
    lo = T[:, :2].min(0) - np.array([A.FOOT_ACROSS, A.FOOT_ALONG])
    hi = T[:, :2].max(0) + np.array([A.FOOT_ACROSS, A.FOOT_ALONG])
    terrain = A.Terrain.__new__(A.Terrain)
    terrain.a, terrain.s, terrain.c = (np.asarray(fl["truth"]["terrain"][k]) for k in ("a", "s", "c"))
    nx = int(math.ceil((hi[0] - lo[0]) / cell)) + 1
    ny = int(math.ceil((hi[1] - lo[1]) / cell)) + 1
    gx, gy = np.meshgrid(lo[0] + cell * np.arange(nx), lo[1] + cell * np.arange(ny))
    h = terrain.height(np.stack([gx.ravel(), gy.ravel()], 1)).reshape(ny, nx).astype(np.float32)
    return {"nx": nx, "ny": ny, "x0": float(lo[0]), "y0": float(lo[1]), "cell": float(cell),
            "h": np.ascontiguousarray(h)}


def patch_grid(width: int = A.IMG_W, height: int = A.IMG_H, size: int = A.CELL_PX) -> np.ndarray:
    """Centres (u, v) of the whole size x size px cells of the image, row by
    row: 53 x 40 = 2120 patches for 8000 x 6000 px at 150 px."""
    nu, nv = width // size, height // size
    u = (np.arange(nu) + 0.5) * size
    v = (np.arange(nv) + 0.5) * size
    uu, vv = np.meshgrid(u, v)
    return np.ascontiguousarray(np.stack([uu.ravel(), vv.ravel()], 1))


def plane_dsm(nx: int, ny: int, x0: float, y0: float, cell: float, a: float, b: float, c: float) -> dict:
    """A raster sampling the plane h = a x + b y + c (bilinear interpolation
    reproduces it exactly between the nodes)."""
    gx, gy = np.meshgrid(x0 + cell * np.arange(nx), y0 + cell * np.arange(ny))
    h = (a * gx + b * gy + c).astype(np.float32)
    return {"nx": nx, "ny": ny, "x0": x0, "y0": y0, "cell": cell, "h": np.ascontiguousarray(h)}
