"""ctypes binding of libba.so (include/ba.h), with the same names.

Argument marshalling only: every step of the adjustment runs in the HIP
kernels of libba.so.  Loading fails loudly when the library has not been
built (paper_2511_06152_amd/build.py) or no GPU is present.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libba.so")

BA_OK, BA_E_ARG, BA_E_NOMEM, BA_E_AGAIN, BA_E_STATE, BA_E_DEVICE, BA_E_TIMEOUT = 0, -1, -2, -3, -4, -5, -7
BA_FP64, BA_MIXED = 0, 1
BA_SOLVER_AUTO, BA_SOLVER_DENSE, BA_SOLVER_PCG = 0, 1, 2
BA_ST_QUEUED, BA_ST_RUNNING, BA_ST_MAXITER, BA_ST_CONVERGED, BA_ST_STALLED, BA_ST_BAD_INIT = range(6)
BA_MAX_FREE_CAMS = 24
BA_MAX_CAMS = 512
BA_MAX_OBS_PER_POINT = 64

EXPORTED = ["ba_create", "ba_destroy", "ba_submit_cluster", "ba_submit_clusters", "ba_step", "ba_solve_batch", "ba_solve", "ba_wait",
            "ba_fetch", "ba_release", "ba_footprint", "ba_profile_enable", "ba_profile_read", "ba_strerror",
            "ba_last_error", "ba_resident_poses", "ba_geo_create", "ba_geo_destroy", "ba_footprints",
            "ba_footprint_overlaps", "ba_cluster_membership", "ba_patch_transfer", "ba_patch_transfer_noalloc",
            "ba_geo_last_ms", "ba_geo_last_error"]
# Kernel slots of ba_profile_enable / ba_profile_read.  "blocks" is the Schur
# block launch: camera and pair tasks together in BA_MIXED, camera tasks
# alone in BA_FP64 (whose pair tasks are "pairblk").
BA_PROF_KERNELS = ["point", "blocks", "pairblk", "reduce", "solve", "backsub", "lm", "pcg"]
BA_PROF_ALL = (1 << len(BA_PROF_KERNELS)) - 1


DEV_ALLOC = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_void_p)
DEV_FREE = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p)


class ba_options(ct.Structure):
    _fields_ = [("device", ct.c_int32), ("stream", ct.c_void_p), ("hbm_budget_bytes", ct.c_size_t),
                ("max_slots", ct.c_int32), ("max_queue", ct.c_int32), ("precision", ct.c_int32),
                ("serve", ct.c_int32), ("iters_per_tick", ct.c_int32), ("chunks_per_wg", ct.c_int32),
                ("chunks_per_task", ct.c_int32), ("solver", ct.c_int32), ("pcg_max_iters", ct.c_int32),
                ("pcg_tol", ct.c_double), ("resident_cams", ct.c_int32), ("resident_points", ct.c_int32),
                ("batch_streams", ct.c_int32), ("dev_alloc", DEV_ALLOC), ("dev_free", DEV_FREE),
                ("alloc_user", ct.c_void_p), ("stage_threads", ct.c_int32)]


class TorchAllocator:
    """Device memory for a context from PyTorch's caching allocator (the
    ba_options.dev_alloc / dev_free hooks): each block is a uint8 tensor kept
    alive until the library frees it."""

    def __init__(self, device: int):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}
        self.c_alloc = DEV_ALLOC(self._alloc)
        self.c_free = DEV_FREE(self._free)

    def _alloc(self, nbytes, user):
        try:
            t = self._torch.empty(max(int(nbytes), 1), dtype=self._torch.uint8, device=f"cuda:{self.device}")
        except RuntimeError:
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, user):
        self.live.pop(ptr, None)


class ba_cluster(ct.Structure):
    _fields_ = [("n_cams", ct.c_int32), ("n_points", ct.c_int32), ("n_obs", ct.c_int32), ("intr_mask", ct.c_int32),
                ("R", ct.c_void_p), ("T", ct.c_void_p), ("X", ct.c_void_p), ("k", ct.c_void_p),
                ("prior_R", ct.c_void_p), ("prior_T", ct.c_void_p), ("prior_sigma", ct.c_void_p),
                ("fixed", ct.c_void_p), ("obs_cam", ct.c_void_p), ("obs_pt", ct.c_void_p), ("obs_uv", ct.c_void_p),
                ("f", ct.c_double), ("cx", ct.c_double), ("cy", ct.c_double),
                ("sigma_px", ct.c_double), ("huber_delta", ct.c_double),
                ("max_iters", ct.c_int32), ("stop_on_ftol", ct.c_int32),
                ("lambda0", ct.c_double), ("ftol", ct.c_double),
                ("cam_ids", ct.c_void_p), ("point_ids", ct.c_void_p), ("use_resident", ct.c_int32),
                ("fuse_resident", ct.c_int32)]


class ba_dsm(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("x0", ct.c_double), ("y0", ct.c_double),
                ("cell", ct.c_double), ("h", ct.c_void_p)]


class ba_pinhole(ct.Structure):
    _fields_ = [("f", ct.c_double), ("cx", ct.c_double), ("cy", ct.c_double), ("width", ct.c_int32),
                ("height", ct.c_int32)]


class ba_cluster_rule(ct.Structure):
    _fields_ = [("max_back", ct.c_int32), ("free_back", ct.c_int32), ("max_cams", ct.c_int32),
                ("min_cams", ct.c_int32), ("min_overlap", ct.c_double)]


class ba_result(ct.Structure):
    _fields_ = [("R", ct.c_void_p), ("T", ct.c_void_p), ("X", ct.c_void_p), ("k", ct.c_void_p),
                ("cost_log", ct.c_void_p), ("status", ct.c_int32), ("iterations", ct.c_int32),
                ("accepted", ct.c_int32), ("rejected", ct.c_int32), ("lambda_", ct.c_double),
                ("initial_cost", ct.c_double), ("final_cost", ct.c_double),
                ("t_submit", ct.c_double), ("t_admit", ct.c_double), ("t_done", ct.c_double),
                ("cg_iters", ct.c_int64), ("intr", ct.c_void_p), ("lambda_log", ct.c_void_p),
                ("accepted_log", ct.c_void_p), ("nu", ct.c_double), ("n_reproj", ct.c_int64),
                ("n_inliers", ct.c_int64), ("reproj_rms", ct.c_double), ("reproj_mean", ct.c_double),
                ("reproj_std", ct.c_double), ("inlier_mean", ct.c_double), ("inlier_std", ct.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libba.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libba.so not built ({path}); run paper_2511_06152_amd/build.py")
    L = ct.CDLL(path)
    P = ct.c_void_p
    L.ba_create.argtypes = [ct.POINTER(ba_options), ct.POINTER(P)]
    L.ba_destroy.argtypes = [P]
    L.ba_submit_cluster.argtypes = [P, ct.POINTER(ba_cluster), ct.POINTER(ct.c_int64)]
    L.ba_submit_clusters.argtypes = [P, ct.c_int32, ct.POINTER(ba_cluster), ct.POINTER(ct.c_int64)]
    L.ba_step.argtypes = [P, ct.c_int64, ct.c_int32]
    L.ba_solve_batch.argtypes = [P, ct.POINTER(ct.c_int64), ct.c_int32]
    L.ba_solve.argtypes = [P, ct.c_int64]
    L.ba_wait.argtypes = [P, ct.c_int64, ct.c_double]
    L.ba_fetch.argtypes = [P, ct.c_int64, ct.POINTER(ba_result)]
    L.ba_release.argtypes = [P, ct.c_int64]
    L.ba_footprint.argtypes = [P, ct.POINTER(ba_cluster)]
    L.ba_footprint.restype = ct.c_size_t
    L.ba_profile_enable.argtypes = [P, ct.c_int32]
    L.ba_profile_read.argtypes = [P, P, P]
    L.ba_resident_poses.argtypes = [P, ct.c_int32, P, P, P, P]
    L.ba_geo_create.argtypes = [ct.c_int32, ct.POINTER(ba_dsm), ct.POINTER(P)]
    L.ba_geo_destroy.argtypes = [P]
    L.ba_footprints.argtypes = [P, ct.c_int32, P, P, ct.POINTER(ba_pinhole), P, P]
    L.ba_footprint_overlaps.argtypes = [P, ct.c_int32, P, P]
    L.ba_cluster_membership.argtypes = [P, ct.c_int32, P, P, ct.POINTER(ba_cluster_rule), P, P, P]
    L.ba_patch_transfer.argtypes = [P, ct.c_int32, P, P, ct.c_int32, P, ct.c_int32, P, ct.POINTER(ba_pinhole),
                                    P, P, P]
    L.ba_patch_transfer_noalloc.argtypes = [P, ct.c_int32, P, P, ct.c_int32, P, ct.c_int32, P,
                                            ct.POINTER(ba_pinhole), P, P]
    L.ba_geo_last_ms.argtypes = [P, P, P]
    L.ba_geo_last_error.argtypes = [P]
    L.ba_geo_last_error.restype = ct.c_char_p
    L.ba_strerror.argtypes = [ct.c_int]
    L.ba_strerror.restype = ct.c_char_p
    L.ba_last_error.argtypes = [P]
    L.ba_last_error.restype = ct.c_char_p
    for name in EXPORTED:
        if name not in ("ba_footprint", "ba_strerror", "ba_last_error", "ba_geo_last_error"):
            getattr(L, name).restype = ct.c_int
    _lib = L
    return L


class BAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


class Cluster:
    """Marshals a scene dict into a ba_cluster, keeping the arrays alive."""

    def __init__(self, sc: dict, max_iters: int = 10, lambda0: float = 1e-4, ftol: float = 1e-10,
                 stop_on_ftol: bool = False, use_resident: bool = False, fuse_resident: bool = False):
        C, P, O = int(sc["n_cams"]), int(sc["n_points"]), int(sc["n_obs"])
        f64 = lambda x: np.ascontiguousarray(np.asarray(x, np.float64).reshape(-1))
        self.arrays = {
            "R": f64(sc["R"]), "T": f64(sc["T"]), "X": f64(sc["X"]) if P else np.zeros(3),
            "k": f64(sc["k"]), "prior_R": f64(sc["prior_R"]), "prior_T": f64(sc["prior_T"]),
            "prior_sigma": f64(sc["prior_sigma"]),
            "fixed": np.ascontiguousarray(np.asarray(sc["fixed"], np.uint8).reshape(-1)),
            "obs_cam": np.ascontiguousarray(np.asarray(sc["obs_cam"], np.int32).reshape(-1)),
            "obs_pt": np.ascontiguousarray(np.asarray(sc["obs_pt"], np.int32).reshape(-1)),
            "obs_uv": f64(sc["obs_uv"]) if O else np.zeros(2),
        }
        for key in ("cam_ids", "point_ids"):
            if sc.get(key) is not None:
                self.arrays[key] = np.ascontiguousarray(np.asarray(sc[key], np.int64).reshape(-1))
        a = self.arrays
        self.C, self.P, self.O, self.max_iters = C, P, O, max_iters
        self.c = ba_cluster(C, P, O, int(sc["intr_mask"]),
                            _p(a["R"]), _p(a["T"]), _p(a["X"]), _p(a["k"]), _p(a["prior_R"]), _p(a["prior_T"]),
                            _p(a["prior_sigma"]), _p(a["fixed"]), _p(a["obs_cam"]), _p(a["obs_pt"]), _p(a["obs_uv"]),
                            float(sc["f"]), float(sc["cx"]), float(sc["cy"]), float(sc["sigma_px"]),
                            float(sc["huber_delta"]), int(max_iters), 1 if stop_on_ftol else 0,
                            float(lambda0), float(ftol), _p(a.get("cam_ids")), _p(a.get("point_ids")),
                            1 if use_resident else 0, 1 if fuse_resident else 0)


class Context:
    """Owns a ba_ctx.  Methods mirror the C ABI and raise BAError on failure."""

    def __init__(self, device: int = 0, stream=None, hbm_budget_bytes: int = 1 << 30, max_slots: int = 256,
                 max_queue: int = 4096, precision: int = BA_FP64, serve: bool = False, iters_per_tick: int = 10,
                 chunks_per_wg: int = 16, chunks_per_task: int = 4, solver: int = BA_SOLVER_AUTO,
                 pcg_max_iters: int = 500, pcg_tol: float = 0.1, resident_cams: int = 0,
                 resident_points: int = 0, batch_streams: int = 0, allocator=None, stage_threads: int = 0):
        """allocator: None (hipMalloc) or "torch" (PyTorch's caching allocator)."""
        self.lib = load()
        opt = ba_options(device, stream, hbm_budget_bytes, max_slots, max_queue, precision, 1 if serve else 0,
                         iters_per_tick, chunks_per_wg, chunks_per_task, solver, pcg_max_iters, pcg_tol,
                         resident_cams, resident_points, batch_streams)
        opt.stage_threads = int(stage_threads)
        self.allocator = None
        if allocator == "torch":
            self.allocator = TorchAllocator(device)
            opt.dev_alloc, opt.dev_free = self.allocator.c_alloc, self.allocator.c_free
        elif allocator is not None:
            raise ValueError("allocator must be None or 'torch'")
        h = ct.c_void_p()
        rc = self.lib.ba_create(ct.byref(opt), ct.byref(h))
        if rc != BA_OK:
            raise BAError(rc, "ba_create failed: " + self.lib.ba_strerror(rc).decode())
        self.h = h
        self.meta = {}

    def _chk(self, rc, what):
        if rc != BA_OK:
            raise BAError(rc, f"{what}: {self.lib.ba_strerror(rc).decode()}: {self.lib.ba_last_error(self.h).decode()}")
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.ba_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def ba_submit_cluster(self, cl: Cluster) -> int:
        t = ct.c_int64()
        self._chk(self.lib.ba_submit_cluster(self.h, ct.byref(cl.c), ct.byref(t)), "ba_submit_cluster")
        self.meta[t.value] = (cl.C, cl.P, cl.max_iters)
        return t.value

    def submit(self, sc: dict, **kw) -> int:
        return self.ba_submit_cluster(Cluster(sc, **kw))

    def ba_submit_clusters(self, cls) -> list:
        """Submit clusters that arrive together (laid out on host threads, queued in order)."""
        n = len(cls)
        arr = (ba_cluster * max(n, 1))(*[c.c for c in cls])
        t = (ct.c_int64 * max(n, 1))()
        try:
            self._chk(self.lib.ba_submit_clusters(self.h, n, arr, t), "ba_submit_clusters")
        finally:
            for i, c in enumerate(cls):
                if t[i]:
                    self.meta[t[i]] = (c.C, c.P, c.max_iters)
        return [t[i] for i in range(n)]

    def submit_many(self, scenes, **kw) -> list:
        return self.ba_submit_clusters([Cluster(sc, **kw) for sc in scenes])

    def ba_footprint(self, cl: Cluster) -> int:
        return int(self.lib.ba_footprint(self.h, ct.byref(cl.c)))

    def ba_step(self, t: int, n_iters: int):
        return self._chk(self.lib.ba_step(self.h, t, n_iters), "ba_step")

    def ba_solve_batch(self, tickets):
        arr = (ct.c_int64 * len(tickets))(*tickets)
        return self._chk(self.lib.ba_solve_batch(self.h, arr, len(tickets)), "ba_solve_batch")

    def ba_solve(self, t: int):
        return self._chk(self.lib.ba_solve(self.h, t), "ba_solve")

    def ba_wait(self, t: int, timeout_s: float = -1.0):
        return self._chk(self.lib.ba_wait(self.h, t, timeout_s), "ba_wait")

    def ba_release(self, t: int):
        self.meta.pop(t, None)
        return self._chk(self.lib.ba_release(self.h, t), "ba_release")

    def ba_profile_enable(self, kernels=True):
        """kernels: True (every kernel), False (off), or a bitmask of 1 << index in BA_PROF_KERNELS."""
        mask = BA_PROF_ALL if kernels is True else (0 if kernels is False else int(kernels))
        return self._chk(self.lib.ba_profile_enable(self.h, mask), "ba_profile_enable")

    def ba_profile_read(self) -> dict:
        ms = np.zeros(len(BA_PROF_KERNELS))
        n = np.zeros(len(BA_PROF_KERNELS), np.int64)
        self._chk(self.lib.ba_profile_read(self.h, _p(ms), _p(n)), "ba_profile_read")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(BA_PROF_KERNELS)}

    def ba_resident_poses(self, cam_ids):
        """(R [n,3,3], T [n,3], w [n]) held on the device for the given camera IDs."""
        ids = np.ascontiguousarray(np.asarray(cam_ids, np.int64).reshape(-1))
        n = ids.size
        R, T, w = np.zeros((n, 3, 3)), np.zeros((n, 3)), np.zeros(n)
        self._chk(self.lib.ba_resident_poses(self.h, n, _p(ids), _p(R), _p(T), _p(w)), "ba_resident_poses")
        return R, T, w

    def ba_fetch(self, t: int) -> dict:
        C, P, it = self.meta[t]
        out = {"R": np.zeros((C, 3, 3)), "T": np.zeros((C, 3)), "X": np.zeros((max(P, 1), 3)), "k": np.zeros(2),
               "cost_log": np.zeros(it + 1), "intr": np.zeros(3), "lambda_log": np.zeros(max(it, 1)),
               "accepted_log": np.zeros(max(it, 1), np.int32)}
        r = ba_result(_p(out["R"]), _p(out["T"]), _p(out["X"]), _p(out["k"]), _p(out["cost_log"]))
        r.intr = _p(out["intr"])
        r.lambda_log = _p(out["lambda_log"])
        r.accepted_log = _p(out["accepted_log"])
        self._chk(self.lib.ba_fetch(self.h, t, ct.byref(r)), "ba_fetch")
        out["X"] = out["X"][:P]
        n = r.iterations
        out.update(status=r.status, iterations=n, accepted=r.accepted, rejected=r.rejected, lambda_=r.lambda_,
                   nu=r.nu, initial_cost=r.initial_cost, final_cost=r.final_cost, t_submit=r.t_submit,
                   t_admit=r.t_admit, t_done=r.t_done, cg_iters=r.cg_iters, n_reproj=r.n_reproj,
                   n_inliers=r.n_inliers, reproj_rms=r.reproj_rms, reproj_mean=r.reproj_mean,
                   reproj_std=r.reproj_std, inlier_mean=r.inlier_mean, inlier_std=r.inlier_std)
        out["cost_log"] = out["cost_log"][: n + 1]
        out["lambda_log"] = out["lambda_log"][:n]
        out["accepted_log"] = out["accepted_log"][:n]
        out["state"] = (out["R"], out["T"], out["X"], out["k"])
        return out


GEO_OK, GEO_MISS, GEO_REINIT = 0, 1, 2


class Geo:
    """Owns a ba_geo (include/ba_geo.h): footprints, footprint overlaps and
    the Eq. (3) patch transfer over a DSM.  dsm: dict with nx, ny, x0, y0,
    cell, h ([ny][nx] float32)."""

    def __init__(self, dsm: dict, device: int = 0):
        self.lib = load()
        self._h = np.ascontiguousarray(np.asarray(dsm["h"], np.float32))
        d = ba_dsm(int(dsm["nx"]), int(dsm["ny"]), float(dsm["x0"]), float(dsm["y0"]), float(dsm["cell"]),
                   _p(self._h))
        h = ct.c_void_p()
        rc = self.lib.ba_geo_create(device, ct.byref(d), ct.byref(h))
        if rc != BA_OK:
            raise BAError(rc, "ba_geo_create failed: " + self.lib.ba_strerror(rc).decode())
        self.h = h

    def _chk(self, rc, what):
        if rc != BA_OK:
            raise BAError(rc, f"{what}: {self.lib.ba_strerror(rc).decode()}: {self.lib.ba_geo_last_error(self.h).decode()}")
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.ba_geo_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @staticmethod
    def _cam(cam: dict):
        return ba_pinhole(float(cam["f"]), float(cam["cx"]), float(cam["cy"]), int(cam["width"]), int(cam["height"]))

    def ba_footprints(self, R, T, cam: dict):
        """(ground [n,5,3], status [n]) for poses R [n,3,3], T [n,3]."""
        R = np.ascontiguousarray(np.asarray(R, np.float64))
        T = np.ascontiguousarray(np.asarray(T, np.float64))
        n = T.shape[0]
        ground, status = np.zeros((n, 5, 3)), np.zeros(n, np.int32)
        c = self._cam(cam)
        self._chk(self.lib.ba_footprints(self.h, n, _p(R), _p(T), ct.byref(c), _p(ground), _p(status)),
                  "ba_footprints")
        return ground, status

    def ba_footprint_overlaps(self, ground):
        """Packed upper triangle of the pairwise overlap areas."""
        ground = np.ascontiguousarray(np.asarray(ground, np.float64))
        n = ground.shape[0]
        area = np.zeros(max(n * (n - 1) // 2, 1))
        self._chk(self.lib.ba_footprint_overlaps(self.h, n, _p(ground), _p(area)), "ba_footprint_overlaps")
        return area[: n * (n - 1) // 2]

    def ba_cluster_membership(self, ground, strip, max_back=7, free_back=3, max_cams=20, min_cams=8,
                              min_overlap=0.05):
        """Per image i: None (no cluster) or (members ascending, fixed flags)."""
        ground = np.ascontiguousarray(np.asarray(ground, np.float64))
        strip = np.ascontiguousarray(np.asarray(strip, np.int32).reshape(-1))
        n = ground.shape[0]
        rule = ba_cluster_rule(int(max_back), int(free_back), int(max_cams), int(min_cams), float(min_overlap))
        mem = np.full((max(n, 1), max_cams), -1, np.int32)
        fix = np.zeros((max(n, 1), max_cams), np.uint8)
        cnt = np.zeros(max(n, 1), np.int32)
        self._chk(self.lib.ba_cluster_membership(self.h, n, _p(ground), _p(strip), ct.byref(rule), _p(mem), _p(fix),
                                                 _p(cnt)), "ba_cluster_membership")
        return [None if cnt[i] == 0 else (mem[i, :cnt[i]].copy(), fix[i, :cnt[i]].copy()) for i in range(n)]

    def ba_patch_transfer(self, R, T, uv0, pairs, cam: dict, want_lam: bool = False):
        """(uv [n_pairs, n_patch, 2], flags [n_pairs, n_patch], lam [n_img, n_patch] or None)."""
        R = np.ascontiguousarray(np.asarray(R, np.float64))
        T = np.ascontiguousarray(np.asarray(T, np.float64))
        uv0 = np.ascontiguousarray(np.asarray(uv0, np.float64))
        pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
        n_img, n_patch, n_pairs = T.shape[0], uv0.shape[0], pairs.shape[0]
        uv = np.zeros((n_pairs, n_patch, 2))
        flags = np.zeros((n_pairs, n_patch), np.int32)
        lam = np.zeros((n_img, n_patch)) if want_lam else None
        c = self._cam(cam)
        self._chk(self.lib.ba_patch_transfer(self.h, n_img, _p(R), _p(T), n_patch, _p(uv0), n_pairs, _p(pairs),
                                             ct.byref(c), _p(uv), _p(flags), _p(lam)), "ba_patch_transfer")
        return uv, flags, lam

    def ba_patch_transfer_noalloc(self, n_img: int, R_dev: int, T_dev: int, n_patch: int, uv0_dev: int, pairs,
                                  cam: dict, uv_dev: int, flags_dev: int):
        """The allocation-free transfer.  R_dev [n_img][9], T_dev [n_img][3],
        uv0_dev [n_patch][2] (float64) and the outputs uv_dev
        [n_pairs][n_patch][2] (float64), flags_dev [n_pairs][n_patch] (int32)
        are device addresses (ints) on the context's device; pairs is host
        data [n_pairs][2]."""
        pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
        c = self._cam(cam)
        self._chk(self.lib.ba_patch_transfer_noalloc(self.h, int(n_img), R_dev, T_dev, int(n_patch), uv0_dev,
                                                     pairs.shape[0], _p(pairs), ct.byref(c), uv_dev, flags_dev),
                  "ba_patch_transfer_noalloc")

    def ba_geo_last_ms(self, last_kernel: bool = False) -> float:
        """Device ms of the last call's kernels (or of its last kernel alone)."""
        tot, last = ct.c_double(), ct.c_double()
        self._chk(self.lib.ba_geo_last_ms(self.h, ct.byref(tot), ct.byref(last)), "ba_geo_last_ms")
        return last.value if last_kernel else tot.value
