"""FP64 CPU oracle for cluster bundle adjustment (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``ba_oracle.cpp`` (built into
``libba_oracle.so`` by :func:`build`) with ctypes and shares nothing with the
HIP library.

A scene is the dict produced by ``synth.aerial.make_scene``; a state is the
tuple (R[C,3,3], T[C,3], X[P,3], k[2]).

The pose fusion between successive clusters (:func:`fuse_pose`, Sec. 3.2,
Eq. (8)) is plain numpy in this module.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ba_oracle.cpp")
LIB = os.path.join(HERE, "libba_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with the host C++ compiler (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Scene(ct.Structure):
    _fields_ = [
        ("n_cams", ct.c_int32), ("n_points", ct.c_int32), ("n_obs", ct.c_int32),
        ("intr_mask", ct.c_int32),
        ("obs_cam", ct.c_void_p), ("obs_pt", ct.c_void_p), ("obs_uv", ct.c_void_p),
        ("prior_R", ct.c_void_p), ("prior_T", ct.c_void_p), ("prior_sigma", ct.c_void_p),
        ("fixed", ct.c_void_p),
        ("f", ct.c_double), ("cx", ct.c_double), ("cy", ct.c_double),
        ("sigma_px", ct.c_double), ("huber_delta", ct.c_double),
    ]


class _Options(ct.Structure):
    _fields_ = [("max_iters", ct.c_int32), ("stop_on_ftol", ct.c_int32),
                ("lambda0", ct.c_double), ("ftol", ct.c_double)]


class _Stats(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("accepted", ct.c_int32), ("rejected", ct.c_int32),
                ("status", ct.c_int32), ("lambda_", ct.c_double), ("nu", ct.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ct.CDLL(LIB)
        P = ct.c_void_p
        L.or_residuals.restype = ct.c_int
        L.or_residuals.argtypes = [P] * 11
        L.or_jacobians.restype = None
        L.or_jacobians.argtypes = [P] * 10
        L.or_prior.restype = None
        L.or_prior.argtypes = [P] * 5
        L.or_cost.restype = ct.c_double
        L.or_cost.argtypes = [P] * 5
        L.or_dims.restype = None
        L.or_dims.argtypes = [P, P, P]
        L.or_step.restype = ct.c_int
        L.or_step.argtypes = [P, P, P, P, P, ct.c_double, P, P]
        L.or_apply.restype = None
        L.or_apply.argtypes = [P] * 10
        L.or_solve.restype = ct.c_int
        L.or_solve.argtypes = [P] * 11
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


class Scene:
    """Keeps the scene's arrays alive and exposes the packed C struct."""

    def __init__(self, sc: dict):
        self.sc = sc
        C = sc["n_cams"]
        self.keep = dict(
            obs_cam=np.ascontiguousarray(sc["obs_cam"], np.int32),
            obs_pt=np.ascontiguousarray(sc["obs_pt"], np.int32),
            obs_uv=np.ascontiguousarray(sc["obs_uv"], np.float64).reshape(-1),
            prior_R=np.ascontiguousarray(sc["prior_R"], np.float64).reshape(C, 9),
            prior_T=np.ascontiguousarray(sc["prior_T"], np.float64).reshape(C, 3),
            prior_sigma=np.ascontiguousarray(sc["prior_sigma"], np.float64).reshape(C, 6),
            fixed=np.ascontiguousarray(sc["fixed"], np.uint8),
        )
        k = self.keep
        self.s = _Scene(sc["n_cams"], sc["n_points"], sc["n_obs"], int(sc["intr_mask"]),
                        _p(k["obs_cam"]), _p(k["obs_pt"]), _p(k["obs_uv"]),
                        _p(k["prior_R"]), _p(k["prior_T"]), _p(k["prior_sigma"]), _p(k["fixed"]),
                        float(sc["f"]), float(sc["cx"]), float(sc["cy"]),
                        float(sc["sigma_px"]), float(sc["huber_delta"]))

    @property
    def ptr(self):
        return ct.byref(self.s)


def _scene(sc) -> Scene:
    return sc if isinstance(sc, Scene) else Scene(sc)


SELF_CAL = 0b11100    # intr_mask bits of f, cx, cy


def initial_state(sc: dict):
    """(R, T, X, k); k = (k1, k2), or (k1, k2, f, cx, cy) when the scene
    estimates any of f, cx, cy (intr_mask bits 2, 3, 4)."""
    k = np.array(sc["k"], np.float64).reshape(2)
    if int(sc["intr_mask"]) & SELF_CAL:
        k = np.array([k[0], k[1], sc["f"], sc["cx"], sc["cy"]], np.float64)
    return (np.array(sc["R"], np.float64).reshape(-1, 3, 3).copy(),
            np.array(sc["T"], np.float64).reshape(-1, 3).copy(),
            np.array(sc["X"], np.float64).reshape(-1, 3).copy(),
            k.copy())


def _state(state, sc):
    """Contiguous arrays; the intrinsic state widened to (k1, k2, f, cx, cy)
    with the scene's f, cx, cy when only (k1, k2) is given."""
    R, T, X, k = state
    k = np.asarray(k, np.float64).reshape(-1)
    if k.size == 2:
        k = np.array([k[0], k[1], sc["f"], sc["cx"], sc["cy"]], np.float64)
    return (np.ascontiguousarray(R, np.float64), np.ascontiguousarray(T, np.float64),
            np.ascontiguousarray(X, np.float64), np.ascontiguousarray(k, np.float64))


def _k_out(k5, like):
    """The intrinsic state in the length the caller used (2 or 5)."""
    return k5.copy() if np.asarray(like).size == 5 else k5[:2].copy()


def residuals(sc, state) -> dict:
    S = _scene(sc)
    R, T, X, k = _state(state, S.sc)
    O = S.sc["n_obs"]
    out = {n: np.zeros(O * (2 if n in ("uv", "e") else 1)) for n in ("uv", "z", "e", "s", "rho", "w")}
    bad = lib().or_residuals(S.ptr, _p(R), _p(T), _p(X), _p(k), *(_p(out[n]) for n in ("uv", "z", "e", "s", "rho", "w")))
    out["uv"] = out["uv"].reshape(O, 2)
    out["e"] = out["e"].reshape(O, 2)
    out["bad"] = bad
    return out


def jacobians(sc, state) -> dict:
    S = _scene(sc)
    R, T, X, k = _state(state, S.sc)
    O = S.sc["n_obs"]
    Jw, JT, JX, Jk, Ji = (np.zeros((O, 2, 3)), np.zeros((O, 2, 3)), np.zeros((O, 2, 3)), np.zeros((O, 2, 2)),
                          np.zeros((O, 2, 3)))
    lib().or_jacobians(S.ptr, _p(R), _p(T), _p(X), _p(k), _p(Jw), _p(JT), _p(JX), _p(Jk), _p(Ji))
    return {"Jw": Jw, "JT": JT, "JX": JX, "Jk": Jk, "Ji": Ji}


def prior(sc, state):
    S = _scene(sc)
    R, T, X, k = _state(state, S.sc)
    C = S.sc["n_cams"]
    e, Jw = np.zeros((C, 6)), np.zeros((C, 3, 3))
    lib().or_prior(S.ptr, _p(R), _p(T), _p(e), _p(Jw))
    return e, Jw


def cost(sc, state) -> float:
    S = _scene(sc)
    R, T, X, k = _state(state, S.sc)
    return float(lib().or_cost(S.ptr, _p(R), _p(T), _p(X), _p(k)))


def dims(sc):
    S = _scene(sc)
    N, m = ct.c_int64(), ct.c_int32()
    lib().or_dims(S.ptr, ct.byref(N), ct.byref(m))
    return int(N.value), int(m.value)


def step(sc, state, lam: float):
    """Damped step delta[N] at the state; returns (status, delta, pred)."""
    S = _scene(sc)
    R, T, X, k = _state(state, S.sc)
    N, _ = dims(S)
    delta = np.zeros(N)
    pred = ct.c_double()
    rc = lib().or_step(S.ptr, _p(R), _p(T), _p(X), _p(k), ct.c_double(lam), _p(delta), ct.byref(pred))
    return rc, delta, pred.value


def apply(sc, state, delta):
    S = _scene(sc)
    R, T, X, k = _state(state, S.sc)
    out = (np.zeros_like(R), np.zeros_like(T), np.zeros_like(X), np.zeros_like(k))
    lib().or_apply(S.ptr, _p(R), _p(T), _p(X), _p(k), _p(np.ascontiguousarray(delta, np.float64)), *(_p(a) for a in out))
    return out[0], out[1], out[2], _k_out(out[3], state[3])


def solve(sc, state=None, max_iters: int = 10, lambda0: float = 1e-4, ftol: float = 1e-10,
          stop_on_ftol: bool = False) -> dict:
    """Run Levenberg-Marquardt; returns the final state and the per-iteration logs."""
    S = _scene(sc)
    if state is None:
        state = initial_state(S.sc)
    R, T, X, k = (a.copy() for a in _state(state, S.sc))
    opt = _Options(max_iters, 1 if stop_on_ftol else 0, lambda0, ftol)
    cost_log = np.full(max_iters + 1, np.nan)
    lam_log = np.full(max_iters, np.nan)
    rho_log = np.full(max_iters, np.nan)
    acc_log = np.zeros(max_iters, np.int32)
    st = _Stats()
    lib().or_solve(S.ptr, _p(R), _p(T), _p(X), _p(k), ct.byref(opt), _p(cost_log), _p(lam_log),
                   _p(rho_log), _p(acc_log), ct.byref(st))
    n = st.iterations
    k_ret = k.copy() if (np.asarray(state[3]).size == 5 or int(S.sc["intr_mask"]) & SELF_CAL) else k[:2].copy()
    return {"state": (R, T, X, k_ret), "intr": k[2:].copy(), "cost_log": cost_log[: n + 1], "lambda_log": lam_log[:n],
            "rho_log": rho_log[:n], "accepted_log": acc_log[:n], "iterations": n,
            "accepted": st.accepted, "rejected": st.rejected, "status": st.status,
            "lambda": st.lambda_, "nu": st.nu}


# --- Pose fusion between successive clusters (Sec. 3.2, Eq. (8)) -----------
# Eq. (8) averages the overlapping image's pose from the previous and the new
# cluster with match-count weights.  Positions are averaged as written; a
# weighted mean of two rotations is taken on SO(3), i.e. the point at fraction
# w_new / (w_old + w_new) along the geodesic from the old to the new rotation
# (a linear mean of rotation matrices is not a rotation).

def so3_log(R) -> np.ndarray:
    """Rotation vector (unit axis times angle in [0, pi]) of a rotation matrix."""
    R = np.asarray(R, np.float64)
    c = np.clip(0.5 * (np.trace(R) - 1.0), -1.0, 1.0)      # cos(theta)
    v = 0.5 * np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])  # sin(theta) * axis
    s = np.linalg.norm(v)
    theta = np.arctan2(s, c)
    if theta < 1e-8:
        return v * (1.0 + theta * theta / 6.0)
    if np.pi - theta < 1e-6:
        # The symmetric part of R is cos(theta) I + (1 - cos(theta)) a a^T:
        # the axis from the column of (R + R^T) / 2 - cos(theta) I with the
        # largest diagonal entry, its sign from the skew part.
        B = 0.5 * (R + R.T) - c * np.eye(3)
        j = int(np.argmax(np.diag(B)))
        a = B[:, j] / np.linalg.norm(B[:, j])
        if a @ v < 0:
            a = -a
        return theta * a
    return theta * v / s


def so3_exp(w) -> np.ndarray:
    """Rotation matrix of a rotation vector (Rodrigues' formula)."""
    w = np.asarray(w, np.float64)
    theta = np.linalg.norm(w)
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if theta < 1e-12:
        return np.eye(3) + K
    K /= theta
    return np.eye(3) + np.sin(theta) * K + (1.0 - np.cos(theta)) * (K @ K)


def fuse_pose(R_old, T_old, w_old, R_new, T_new, w_new):
    """Eq. (8) for one camera: the match-count weighted mean of the pose left
    by the earlier cluster (weight w_old) and the new cluster's (w_new).
    Returns (R, T, w_old + w_new); with w_old <= 0 there is nothing to average
    and the new pose is returned with weight w_new."""
    R_old, R_new = np.asarray(R_old, np.float64), np.asarray(R_new, np.float64)
    T_old, T_new = np.asarray(T_old, np.float64), np.asarray(T_new, np.float64)
    if w_old <= 0:
        return R_new.copy(), T_new.copy(), float(w_new)
    wsum = float(w_old) + float(w_new)
    a = float(w_new) / wsum
    R = R_old @ so3_exp(a * so3_log(R_old.T @ R_new))
    T = (w_old * T_old + w_new * T_new) / wsum
    return R, T, wsum
