"""Seeded synthetic aerial bundle-adjustment scenes.

This is the input generator shared by the tests, the benchmark and the smoke
check.  It flies a block of nadir images over Gaussian-hill terrain, spawns tie
points in 150x150 px image cells (the patch grid of Sec. 3.1), observes them in
the overlapping images of the cluster (including images of the adjacent strip,
Sec. 3.1 / 3.2), adds pixel noise and wrong-match outliers, and perturbs the
poses into a GNSS/IMU-like initialisation that also serves as pose prior
(Sec. 3.2: initial T_k^(0), R_k^(0) from navigation data).

It holds only the data-generating process: a forward camera model to synthesise
measurements and a ray/terrain intersection to place points.  Nothing here
evaluates residuals, Jacobians or any part of the adjustment.

Conventions (shared by every consumer of a scene):
  * R[k] is camera->world (columns are the camera x, y, z axes in the world
    frame), T[k] is the projection centre, so a world point X is seen at
    X_c = R[k]^T (X - T[k]), with z forward and the image y axis down.
  * obs_uv are pixel coordinates with the origin at the image corner; the
    principal point is (cx, cy).
  * World frame: local ENU metres.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Camera of the workload: 50 MP, 8000 x 6000 px, 3.76 um pixels, f = 50 mm.
IMG_W = 8000
IMG_H = 6000
PIXEL_M = 3.76e-6
FOCAL_M = 0.050
F_PX = FOCAL_M / PIXEL_M            # 13297.87 px
CX = IMG_W / 2.0
CY = IMG_H / 2.0
ALTITUDE = 300.0
CELL_PX = 150                       # patch cell size used to spawn tie points
FWD_OVERLAP = 0.80
SIDE_OVERLAP = 0.60
DEG = math.pi / 180.0

GSD = ALTITUDE / F_PX
FOOT_ALONG = IMG_H * GSD            # image y axis is the along-track axis
FOOT_ACROSS = IMG_W * GSD
BASE = (1.0 - FWD_OVERLAP) * FOOT_ALONG
STRIP_SPACING = (1.0 - SIDE_OVERLAP) * FOOT_ACROSS

R_NADIR = np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, -1.0]])


@dataclasses.dataclass
class SceneSpec:
    n_strips: int = 2
    imgs_per_strip: int = 3
    n_points: int = 2000
    # observations per point: ("geom", mean) = 1 + geometric extra observers
    # with the given mean total; ("tgeom", p, lo, hi) = truncated geometric.
    obs_model: tuple = ("geom", 3.0)
    noise_px: float = 0.5
    outlier_frac: float = 0.03
    outlier_px: float = 75.0
    k_true: tuple = (0.0, 0.0)
    k_init: tuple = (0.0, 0.0)
    intr_mask: int = 0
    pos_noise_m: float = 0.5
    att_noise_deg: float = 0.05
    point_noise_m: float = 1.0
    prior_sigma_T: float = 0.5
    prior_sigma_w_deg: float = 0.05
    priors: bool = True
    priors_at_truth: bool = False
    n_fixed: int = 0
    sigma_px: float = 0.5
    huber_delta_px: float = 1.0
    jitter_deg: float = 1.0
    n_hills: int = 8
    first_strip: int = 0
    # Whole-flight blocks: test visibility only against the cameras whose
    # footprint can overlap the spawning image's, in chunks of candidate points
    # (bounded memory for hundreds of cameras and ~1M points).
    neighbour_vis: bool = False


def rotvec_to_matrix(w: np.ndarray) -> np.ndarray:
    """Rotation matrices for rotation vectors w[..., 3] (Rodrigues)."""
    w = np.asarray(w, dtype=np.float64)
    th = np.linalg.norm(w, axis=-1, keepdims=True)
    small = th < 1e-12
    k = np.where(small, 0.0, w / np.where(small, 1.0, th))
    K = np.zeros(w.shape[:-1] + (3, 3))
    K[..., 0, 1], K[..., 0, 2] = -k[..., 2], k[..., 1]
    K[..., 1, 0], K[..., 1, 2] = k[..., 2], -k[..., 0]
    K[..., 2, 0], K[..., 2, 1] = -k[..., 1], k[..., 0]
    th = th[..., None]
    eye = np.broadcast_to(np.eye(3), K.shape)
    return eye + np.sin(th) * K + (1.0 - np.cos(th)) * (K @ K)


def heading_matrix(psi: float) -> np.ndarray:
    c, s = math.cos(psi), math.sin(psi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


class Terrain:
    """Sum of Gaussian hills: z = sum_i a_i exp(-|xy - c_i|^2 / (2 s_i^2))."""

    def __init__(self, rng: np.random.Generator, lo: np.ndarray, hi: np.ndarray, n: int):
        self.a = rng.uniform(0.0, 50.0, n)
        self.s = rng.uniform(50.0, 250.0, n)
        self.c = rng.uniform(lo, hi, (n, 2))

    def height(self, xy: np.ndarray) -> np.ndarray:
        d2 = ((xy[:, None, :] - self.c[None, :, :]) ** 2).sum(-1)
        return (self.a[None, :] * np.exp(-d2 / (2.0 * self.s[None, :] ** 2))).sum(-1)

    def intersect(self, origin: np.ndarray, direction: np.ndarray) -> np.ndarray:
        """Ray/terrain intersection by fixed-point iteration on the height."""
        z = np.zeros(origin.shape[0])
        for _ in range(200):
            t = (z - origin[:, 2]) / direction[:, 2]
            p = origin + t[:, None] * direction
            z_new = self.height(p[:, :2])
            if np.max(np.abs(z_new - z)) < 1e-9:
                z = z_new
                break
            z = z_new
        t = (z - origin[:, 2]) / direction[:, 2]
        return origin + t[:, None] * direction


def _distort(a, b, k1, k2):
    r2 = a * a + b * b
    d = 1.0 + k1 * r2 + k2 * r2 * r2
    return a * d, b * d


def synth_project(R, T, X, k1, k2):
    """Data-generating camera: pixel coordinates of X (N,3) in cameras (R,T).

    R: (C,3,3), T: (C,3); returns uv (N,C,2) and depth z (N,C).
    """
    d = X[:, None, :] - T[None, :, :]
    xc = np.einsum("cji,ncj->nci", R, d)
    z = xc[..., 2]
    zs = np.where(np.abs(z) < 1e-9, 1e-9, z)
    a, b = xc[..., 0] / zs, xc[..., 1] / zs
    ad, bd = _distort(a, b, k1, k2)
    uv = np.stack([F_PX * ad + CX, F_PX * bd + CY], axis=-1)
    return uv, z


def project_obs(R, T, X, k, obs_cam, obs_pt):
    """Data-generating camera applied per observation: pixel (O,2) of point
    obs_pt[o] in camera obs_cam[o]."""
    R, T, X = np.asarray(R).reshape(-1, 3, 3), np.asarray(T).reshape(-1, 3), np.asarray(X).reshape(-1, 3)
    d = X[obs_pt] - T[obs_cam]
    xc = np.einsum("nji,nj->ni", R[obs_cam], d)
    a, b = _distort(xc[:, 0] / xc[:, 2], xc[:, 1] / xc[:, 2], k[0], k[1])
    return np.stack([F_PX * a + CX, F_PX * b + CY], -1)


def _undistort(ad, bd, k1, k2):
    a, b = ad.copy(), bd.copy()
    for _ in range(20):
        r2 = a * a + b * b
        d = 1.0 + k1 * r2 + k2 * r2 * r2
        a, b = ad / d, bd / d
    return a, b


def flight_poses(spec: SceneSpec, rng: np.random.Generator):
    """Truth poses of a boustrophedon block, in flight order (strip-major)."""
    R, T, strip = [], [], []
    for s in range(spec.n_strips):
        gs = spec.first_strip + s
        north = gs % 2 == 0
        psi = 0.0 if north else math.pi
        for i in range(spec.imgs_per_strip):
            y = i * BASE if north else (spec.imgs_per_strip - 1 - i) * BASE
            T.append([gs * STRIP_SPACING, y, ALTITUDE])
            jit = rng.normal(0.0, spec.jitter_deg * DEG, 3)
            R.append(heading_matrix(psi) @ R_NADIR @ rotvec_to_matrix(jit))
            strip.append(gs)
    return np.array(R), np.array(T), np.array(strip, dtype=np.int32)


def _n_observers(spec: SceneSpec, rng: np.random.Generator, n: int) -> np.ndarray:
    kind = spec.obs_model[0]
    if kind == "geom":
        mean_total = spec.obs_model[1]
        p = 1.0 / max(mean_total - 1.0, 1e-9)
        return 1 + rng.geometric(min(p, 1.0), n)
    if kind == "tgeom":
        p, lo, hi = spec.obs_model[1], spec.obs_model[2], spec.obs_model[3]
        ks = np.arange(lo, hi + 1)
        pk = p * (1.0 - p) ** (ks - lo)
        pk /= pk.sum()
        return rng.choice(ks, size=n, p=pk)
    if kind == "all":
        return np.full(n, 1 << 30)
    raise ValueError(kind)


def make_scene(spec: SceneSpec, seed: int) -> dict:
    """Generate one cluster.  Returns a dict of C-contiguous numpy arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R_t, T_t, strip = flight_poses(spec, rng)
    C = R_t.shape[0]
    lo = T_t[:, :2].min(0) - np.array([FOOT_ACROSS, FOOT_ALONG])
    hi = T_t[:, :2].max(0) + np.array([FOOT_ACROSS, FOOT_ALONG])
    terrain = Terrain(rng, lo, hi, spec.n_hills)
    k1t, k2t = spec.k_true
    ncx, ncy = IMG_W // CELL_PX, IMG_H // CELL_PX

    if spec.neighbour_vis:
        X_true, obs_cam, obs_pt, uv_true = _spawn_points_blocked(spec, rng, R_t, T_t, terrain)
    else:
        X_true, obs_cam, obs_pt, uv_true = _spawn_points(spec, rng, R_t, T_t, terrain)
    sc = _finish_scene(spec, rng, R_t, T_t, strip, X_true, obs_cam, obs_pt, uv_true)
    sc["truth"]["terrain"] = {"a": terrain.a.copy(), "s": terrain.s.copy(), "c": terrain.c.copy()}
    return sc


def _spawn_points(spec, rng, R_t, T_t, terrain):
    """Tie points and their true observations, testing every camera."""
    C = R_t.shape[0]
    k1t, k2t = spec.k_true
    ncx, ncy = IMG_W // CELL_PX, IMG_H // CELL_PX
    X_list, obs_list = [], []
    have = 0
    guard = 0
    while have < spec.n_points:
        guard += 1
        if guard > 200:
            raise RuntimeError("scene generator could not place enough points")
        B = max(1024, int(1.6 * (spec.n_points - have)))
        img = rng.integers(0, C, B)
        cu = rng.integers(0, ncx, B)
        cv = rng.integers(0, ncy, B)
        u = (cu + rng.uniform(0, 1, B)) * CELL_PX
        v = (cv + rng.uniform(0, 1, B)) * CELL_PX
        a, b = _undistort((u - CX) / F_PX, (v - CY) / F_PX, k1t, k2t)
        dirc = np.stack([a, b, np.ones(B)], -1)
        dirw = np.einsum("nij,nj->ni", R_t[img], dirc)
        X = terrain.intersect(T_t[img], dirw)
        uv, z = synth_project(R_t, T_t, X, k1t, k2t)
        vis = (z > 1.0) & (uv[..., 0] >= 0) & (uv[..., 0] < IMG_W) & (uv[..., 1] >= 0) & (uv[..., 1] < IMG_H)
        vis[np.arange(B), img] = False
        want = _n_observers(spec, rng, B) - 1
        score = rng.uniform(0, 1, (B, C))
        score[~vis] = np.inf
        order = np.argsort(score, axis=1)
        n_extra = np.minimum(want, vis.sum(1))
        keep = np.nonzero(n_extra >= 1)[0][: spec.n_points - have]
        if keep.size == 0:
            continue
        # observers of each kept point: its spawning image and its n_extra
        # chosen images, in camera order
        ne = n_extra[keep]
        w = int(ne.max()) + 1
        cams = np.full((keep.size, w), C, np.int64)
        cams[:, 0] = img[keep]
        cols = np.arange(1, w)[None, :]
        cams[:, 1:] = np.where(cols <= ne[:, None], order[keep, : w - 1], C)
        cams.sort(axis=1)
        sel = np.arange(w)[None, :] <= ne[:, None]
        rows = np.repeat(np.arange(keep.size), ne + 1)
        cam_flat = cams[sel]
        X_list.append(X[keep])
        obs_list.append((rows + have, cam_flat, uv[keep[rows], cam_flat]))
        have += keep.size

    X_true = np.concatenate(X_list)
    obs_cam = np.concatenate([o[1] for o in obs_list]).astype(np.int32)
    obs_pt = np.concatenate([o[0] for o in obs_list]).astype(np.int32)
    uv_true = np.concatenate([o[2] for o in obs_list])
    return X_true, obs_cam, obs_pt, uv_true


def _spawn_points_blocked(spec, rng, R_t, T_t, terrain, chunk=32768):
    """Tie points and their true observations for large blocks: each candidate
    is tested against the cameras whose centre lies within one footprint of
    the spawning camera's (with margin), so memory is chunk x neighbours."""
    C = R_t.shape[0]
    k1t, k2t = spec.k_true
    ncx, ncy = IMG_W // CELL_PX, IMG_H // CELL_PX
    dxy = np.abs(T_t[:, None, :2] - T_t[None, :, :2])
    near = (dxy[..., 0] < 1.25 * FOOT_ACROSS) & (dxy[..., 1] < 1.25 * FOOT_ALONG)
    np.fill_diagonal(near, False)
    K = int(near.sum(1).max()) if C > 1 else 0
    nbr = np.full((C, max(K, 1)), -1, np.int64)
    for k in range(C):
        idx = np.nonzero(near[k])[0]
        nbr[k, : idx.size] = idx
    Xs, cams_s, pts_s, uvs_s = [], [], [], []
    have = 0
    guard = 0
    while have < spec.n_points:
        guard += 1
        if guard > 100000:
            raise RuntimeError("scene generator could not place enough points")
        B = int(min(chunk, max(1024, 1.6 * (spec.n_points - have))))
        img = rng.integers(0, C, B)
        cu = rng.integers(0, ncx, B)
        cv = rng.integers(0, ncy, B)
        u = (cu + rng.uniform(0, 1, B)) * CELL_PX
        v = (cv + rng.uniform(0, 1, B)) * CELL_PX
        a, b = _undistort((u - CX) / F_PX, (v - CY) / F_PX, k1t, k2t)
        dirc = np.stack([a, b, np.ones(B)], -1)
        dirw = np.einsum("nij,nj->ni", R_t[img], dirc)
        X = terrain.intersect(T_t[img], dirw)
        cand = nbr[img]                                   # (B, K), -1 padded
        cs = np.where(cand < 0, 0, cand)
        d = X[:, None, :] - T_t[cs]
        xc = np.einsum("nkji,nkj->nki", R_t[cs], d)
        z = xc[..., 2]
        zs = np.where(np.abs(z) < 1e-9, 1e-9, z)
        ad, bd = _distort(xc[..., 0] / zs, xc[..., 1] / zs, k1t, k2t)
        uv = np.stack([F_PX * ad + CX, F_PX * bd + CY], -1)
        vis = (cand >= 0) & (z > 1.0) & (uv[..., 0] >= 0) & (uv[..., 0] < IMG_W) & (uv[..., 1] >= 0) & \
            (uv[..., 1] < IMG_H)
        want = _n_observers(spec, rng, B) - 1
        score = rng.uniform(0, 1, vis.shape)
        score[~vis] = np.inf
        order = np.argsort(score, axis=1)
        n_extra = np.minimum(want, vis.sum(1))
        keep = np.nonzero(n_extra >= 1)[0][: spec.n_points - have]
        if keep.size == 0:
            continue
        ne = n_extra[keep]
        col = np.arange(order.shape[1])[None, :]
        sel = col < ne[:, None]                           # (n, K) chosen extra observers
        rows = np.repeat(np.arange(keep.size), ne)
        extra = cand[keep[:, None], order[keep]][sel]     # camera ids, row-major
        extra_uv = uv[keep[:, None], order[keep]][sel]
        # the spawning camera sees the point where its ray was cast
        all_cam = np.concatenate([img[keep], extra])
        all_row = np.concatenate([np.arange(keep.size), rows])
        all_uv = np.concatenate([synth_pixel(R_t[img[keep]], T_t[img[keep]], X[keep], k1t, k2t), extra_uv])
        srt = np.lexsort((all_cam, all_row))
        Xs.append(X[keep])
        cams_s.append(all_cam[srt])
        pts_s.append(all_row[srt] + have)
        uvs_s.append(all_uv[srt])
        have += keep.size
    return (np.concatenate(Xs), np.concatenate(cams_s).astype(np.int32), np.concatenate(pts_s).astype(np.int32),
            np.concatenate(uvs_s))


def synth_pixel(R, T, X, k1, k2):
    """Data-generating camera per row: pixel (N,2) of X[n] in camera (R[n], T[n])."""
    xc = np.einsum("nji,nj->ni", R, X - T)
    a, b = _distort(xc[:, 0] / xc[:, 2], xc[:, 1] / xc[:, 2], k1, k2)
    return np.stack([F_PX * a + CX, F_PX * b + CY], -1)


def _finish_scene(spec, rng, R_t, T_t, strip, X_true, obs_cam, obs_pt, uv_true):
    """Noise, outliers, observation shuffle, perturbed initial poses and priors."""
    C = R_t.shape[0]
    O = obs_cam.shape[0]

    uv = uv_true + rng.normal(0.0, spec.noise_px, (O, 2))
    n_out = int(round(spec.outlier_frac * O))
    out_idx = rng.choice(O, n_out, replace=False) if n_out > 0 else np.zeros(0, np.int64)
    uv[out_idx] = uv_true[out_idx] + rng.uniform(-spec.outlier_px, spec.outlier_px, (n_out, 2))

    perm = rng.permutation(O)
    obs_cam, obs_pt, uv = obs_cam[perm], obs_pt[perm], uv[perm]
    is_outlier = np.zeros(O, dtype=bool)
    is_outlier[out_idx] = True
    is_outlier = is_outlier[perm]

    R0 = np.einsum("cij,cjk->cik", R_t, rotvec_to_matrix(rng.normal(0.0, spec.att_noise_deg * DEG, (C, 3))))
    T0 = T_t + rng.normal(0.0, spec.pos_noise_m, (C, 3))
    X0 = X_true + rng.normal(0.0, spec.point_noise_m, X_true.shape)

    if spec.priors_at_truth:
        pR, pT = R_t.copy(), T_t.copy()
    else:
        pR, pT = R0.copy(), T0.copy()
    sig = np.zeros((C, 6))
    if spec.priors:
        sig[:, :3] = spec.prior_sigma_w_deg * DEG
        sig[:, 3:] = spec.prior_sigma_T
    fixed = np.zeros(C, dtype=np.uint8)
    fixed[: spec.n_fixed] = 1

    c = lambda x, dt=np.float64: np.ascontiguousarray(x, dtype=dt)
    return {
        "n_cams": C,
        "n_points": int(X0.shape[0]),
        "n_obs": int(O),
        "R": c(R0),
        "T": c(T0),
        "X": c(X0),
        "k": c(spec.k_init),
        "prior_R": c(pR),
        "prior_T": c(pT),
        "prior_sigma": c(sig),
        "fixed": c(fixed, np.uint8),
        "obs_cam": c(obs_cam, np.int32),
        "obs_pt": c(obs_pt, np.int32),
        "obs_uv": c(uv),
        "f": F_PX,
        "cx": CX,
        "cy": CY,
        "intr_mask": int(spec.intr_mask),
        "sigma_px": float(spec.sigma_px),
        "huber_delta": float(spec.huber_delta_px),
        "truth": {
            "R": c(R_t),
            "T": c(T_t),
            "X": c(X_true),
            "k": c(spec.k_true),
            "strip": strip,
            "outlier": is_outlier,
        },
    }


# ---------------------------------------------------------------------------
# Workload presets.  Sizes follow the workloads the method is evaluated on.

def spec_tiny() -> SceneSpec:
    """6 cameras (2 strips x 3), 2,000 points, every image that sees a point
    observes it (~3.1 observations per point, ~6,200 observations)."""
    return SceneSpec(n_strips=2, imgs_per_strip=3, n_points=2000, obs_model=("all",))


def spec_cluster12() -> SceneSpec:
    """Paper-scale local cluster: 12 cameras (2 strips x 6), ~20k points,
    ~85k observations (every image that sees a point observes it), k1/k2
    radial distortion estimated (truth -0.05, 0.02)."""
    return SceneSpec(n_strips=2, imgs_per_strip=6, n_points=20000, obs_model=("all",),
                     k_true=(-0.05, 0.02), k_init=(0.0, 0.0), intr_mask=3)


def spec_batched(seed: int) -> SceneSpec:
    """One cluster of the uneven batch: 6-24 cameras in 2-3 strips, points
    log-uniform in [5k, 60k], 2-6 observations per point (geometric, p=0.5),
    5% outliers, pinhole."""
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5EED))
    C = int(rng.integers(6, 25))
    n_strips = 2 if C < 12 else 3
    per = int(math.ceil(C / n_strips))
    P = int(round(math.exp(rng.uniform(math.log(5000), math.log(60000)))))
    return SceneSpec(n_strips=n_strips, imgs_per_strip=per, n_points=P,
                     obs_model=("tgeom", 0.5, 2, 6), outlier_frac=0.05)


def spec_micro(n_strips=2, imgs_per_strip=2, n_points=40, **kw) -> SceneSpec:
    """Small scenes for brute-force checks."""
    kw.setdefault("obs_model", ("geom", 3.0))
    return SceneSpec(n_strips=n_strips, imgs_per_strip=imgs_per_strip, n_points=n_points, **kw)


def scene_tiny(seed: int = 1) -> dict:
    return make_scene(spec_tiny(), seed)


def scene_cluster12(seed: int = 2) -> dict:
    return make_scene(spec_cluster12(), seed)


def scene_batched(index: int) -> dict:
    seed = 4_000_000 + index
    return make_scene(spec_batched(seed), seed)


def spec_global(n_strips: int = 10, imgs_per_strip: int = 40, n_points: int = 800_000) -> SceneSpec:
    """Whole-flight block for the global adjustment: 400 cameras (10 strips x
    40), 800k tie points, 1 + geometric extra observers with mean 4.8 total,
    truncated by visibility (~4.39 per point, ~3.5M observations), 3% outliers,
    pinhole."""
    return SceneSpec(n_strips=n_strips, imgs_per_strip=imgs_per_strip, n_points=n_points,
                     obs_model=("geom", 4.8), neighbour_vis=True)


def scene_global(seed: int = 5, **kw) -> dict:
    return make_scene(spec_global(**kw), seed)


def _flight(seed, n_strips, imgs_per_strip, pts_per_image, obs_mean):
    """A flight with one global tie-point pool, and its observations grouped
    by camera (order, starts)."""
    spec = SceneSpec(n_strips=n_strips, imgs_per_strip=imgs_per_strip,
                     n_points=pts_per_image * n_strips * imgs_per_strip,
                     obs_model=("geom", obs_mean), neighbour_vis=True)
    fl = make_scene(spec, seed)
    order = np.argsort(fl["obs_cam"], kind="stable")
    starts = np.searchsorted(fl["obs_cam"][order], np.arange(fl["n_cams"] + 1))
    return fl, order, starts


def _overlapping_prev_strip(fl, i):
    """Images of the previous strip whose footprint overlaps image i's, nearest first."""
    strip = fl["truth"]["strip"]
    Txy = fl["truth"]["T"][:, :2]
    prev = np.nonzero(strip == strip[i] - 1)[0]
    d = np.abs(Txy[prev] - Txy[i])
    prev = prev[(d[:, 0] < FOOT_ACROSS) & (d[:, 1] < FOOT_ALONG)]
    return prev[np.argsort(np.hypot(*(Txy[prev] - Txy[i]).T))]


def _cut_cluster(fl, order, starts, cams, fixed, image):
    """The cluster scene of the given flight images: pool points with at least
    two observations among them, IDs = flight indices."""
    C = fl["n_cams"]
    obs = np.concatenate([order[starts[k]:starts[k + 1]] for k in cams])
    cnt = np.bincount(fl["obs_pt"][obs], minlength=fl["n_points"])
    pts = np.nonzero(cnt >= 2)[0]
    obs = obs[cnt[fl["obs_pt"][obs]] >= 2]
    obs = np.sort(obs)
    cam_loc = np.full(C, -1, np.int64)
    cam_loc[cams] = np.arange(cams.size)
    pt_loc = np.full(fl["n_points"], -1, np.int64)
    pt_loc[pts] = np.arange(pts.size)
    c = lambda x, dt=np.float64: np.ascontiguousarray(x, dtype=dt)
    return {
        "image": image, "n_cams": int(cams.size), "n_points": int(pts.size), "n_obs": int(obs.size),
        "R": c(fl["R"][cams]), "T": c(fl["T"][cams]), "X": c(fl["X"][pts]), "k": c(fl["k"]),
        "prior_R": c(fl["prior_R"][cams]), "prior_T": c(fl["prior_T"][cams]),
        "prior_sigma": c(fl["prior_sigma"][cams]), "fixed": np.asarray(fixed, np.uint8),
        "obs_cam": c(cam_loc[fl["obs_cam"][obs]], np.int32), "obs_pt": c(pt_loc[fl["obs_pt"][obs]], np.int32),
        "obs_uv": c(fl["obs_uv"][obs]), "f": fl["f"], "cx": fl["cx"], "cy": fl["cy"], "intr_mask": 0,
        "sigma_px": fl["sigma_px"], "huber_delta": fl["huber_delta"],
        "cam_ids": c(cams, np.int64), "point_ids": c(pts, np.int64),
    }


def stream_flight(seed: int = 3, n_strips: int = 4, imgs_per_strip: int = 40, pts_per_image: int = 2000,
                  obs_mean: float = 4.8) -> dict:
    """The serving stream's flight: n_strips x imgs_per_strip images in flight
    order over one global tie-point pool (~pts_per_image spawned per image).
    Returns {"flight": scene of the whole block (truth["strip"], the strip of
    each image; truth["terrain"], its hills), "order", "starts": the
    observations grouped by camera}."""
    fl, order, starts = _flight(seed, n_strips, imgs_per_strip, pts_per_image, obs_mean)
    return {"flight": fl, "order": order, "starts": starts}


def cut_clusters(sf: dict, membership) -> list:
    """Cluster scenes of a stream flight for a given membership: membership[i]
    is None (image i triggers no cluster) or (cameras, fixed flags), the
    cameras as flight indices.  Scenes as make_stream's, "image" = i."""
    fl, order, starts = sf["flight"], sf["order"], sf["starts"]
    out = []
    for i, m in enumerate(membership):
        if m is None:
            continue
        cams = np.asarray(m[0], np.int64)
        out.append(_cut_cluster(fl, order, starts, cams, np.asarray(m[1], np.uint8), i))
    return out


def make_stream(seed: int = 3, n_strips: int = 4, imgs_per_strip: int = 40, pts_per_image: int = 2000,
                max_cams: int = 20, min_cams: int = 8, back: int = 7, free_back: int = 3,
                obs_mean: float = 4.8) -> dict:
    """A flight of n_strips x imgs_per_strip images in flight order with one
    global tie-point pool (~pts_per_image spawned per image), cut into the
    sliding clusters that each arriving image triggers (Sec. 3.2): image i,
    its up to `back` in-strip predecessors and the previous strip's images
    whose footprint overlaps it (nearest first), capped at max_cams; a cluster
    is emitted once it has min_cams images.  Points are the pool points with
    at least two observations inside the cluster.  Images older than
    `free_back` in-strip steps and previous-strip images are fixed (they were
    adjusted by earlier clusters); the rest are free.

    Returns {"flight": scene of the whole block, "clusters": [scene, ...]} where
    each cluster scene carries cam_ids / point_ids (indices into the flight)
    and "image": the triggering image."""
    fl, order, starts = _flight(seed, n_strips, imgs_per_strip, pts_per_image, obs_mean)
    strip = fl["truth"]["strip"]
    clusters = []
    for i in range(fl["n_cams"]):
        s, pos = int(strip[i]), i % imgs_per_strip
        own = [i - b for b in range(1, back + 1) if pos - b >= 0]
        prev = _overlapping_prev_strip(fl, i)
        cams = ([i] + own + [int(k) for k in prev])[:max_cams]
        if len(cams) < min_cams:
            continue
        cams = np.array(sorted(cams), np.int64)
        fixed = np.array([0 if (k == i or (strip[k] == s and i - k <= free_back)) else 1 for k in cams], np.uint8)
        clusters.append(_cut_cluster(fl, order, starts, cams, fixed, i))
    return {"flight": fl, "clusters": clusters}


def chain_membership(n_images: int, cluster_size: int = 12, n_ref: int = 3):
    """The paper's chaining of clusters (Sec. 3.2, Sec. 4): images in flight
    order are cut into clusters of cluster_size; each cluster after the first
    starts with the last n_ref images of its predecessor as references, the
    first half of them (n_ref // 2) fixed and the rest free (their poses are
    then fused by Eq. 8), followed by new images.  A shorter last cluster
    takes the images left over.  Returns [(own, refs, fixed_refs)]: the
    cluster's images in flight order, its references, and the fixed ones."""
    if not 0 <= n_ref < cluster_size:
        raise ValueError("need 0 <= n_ref < cluster_size")
    out, prev, start = [], [], 0
    while start < n_images:
        refs = prev[len(prev) - n_ref:] if (prev and n_ref) else []
        new = list(range(start, min(n_images, start + cluster_size - len(refs))))
        own = refs + new
        out.append((own, refs, refs[: len(refs) // 2]))
        prev, start = own, new[-1] + 1
    return out


def make_chain(seed: int = 9, n_strips: int = 2, imgs_per_strip: int = 30, pts_per_image: int = 2000,
               cluster_size: int = 12, n_ref: int = 3, max_neighbours: int = 8, obs_mean: float = 4.8) -> dict:
    """The paper's evaluation flight shape (Sec. 4: 60 images in two strips,
    clusters of 12 reusing the last 3 images) cut by `chain_membership`.  Each
    cluster also holds up to max_neighbours images of the previous strip
    whose footprints overlap its own images (nearest first per image, fixed:
    adjusted by earlier clusters).  Cluster scenes as in make_stream, with
    "image" the cluster's last image, "refs" its reference IDs and
    "refs_fixed" the fixed ones."""
    fl, order, starts = _flight(seed, n_strips, imgs_per_strip, pts_per_image, obs_mean)
    clusters = []
    for own, refs, fixed_refs in chain_membership(fl["n_cams"], cluster_size, n_ref):
        nb = []
        for i in own:
            for k in _overlapping_prev_strip(fl, i):
                if int(k) not in own and int(k) not in nb:
                    nb.append(int(k))
        nb = nb[:max_neighbours]
        cams = np.array(sorted(own + nb), np.int64)
        fixed = np.array([1 if (k in fixed_refs or k in nb) else 0 for k in cams], np.uint8)
        sc = _cut_cluster(fl, order, starts, cams, fixed, own[-1])
        sc["refs"] = np.array(refs, np.int64)
        sc["refs_fixed"] = np.array(fixed_refs, np.int64)
        clusters.append(sc)
    return {"flight": fl, "clusters": clusters}
