"""Brute-force helpers for pinning the oracle: finite differences through an
independent rotation implementation (scipy), dense normal equations, and a
flat parameter vector for generic minimisers.

State convention: (R[C,3,3], T[C,3], X[P,3], k) with k = (k1, k2), or
(k1, k2, f, cx, cy) when the scene estimates f, cx or cy; unknown ordering:
free cameras (omega[3], T[3]), estimated intrinsics (k1, k2, f, cx, cy per
mask bits 0-4), points.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation

import oracle


def rot(w):
    return Rotation.from_rotvec(np.asarray(w, dtype=np.float64)).as_matrix()


def layout(sc):
    free = [c for c in range(sc["n_cams"]) if not sc["fixed"][c]]
    cam_col = {c: 6 * i for i, c in enumerate(free)}
    kcols = []
    col = 6 * len(free)
    for b in range(5):
        if sc["intr_mask"] & (1 << b):
            kcols.append((b, col))
            col += 1
    m = col
    N = m + 3 * sc["n_points"]
    return cam_col, kcols, m, N


def boxplus(sc, state, delta):
    """x (+) delta using scipy rotations (independent of the oracle's Exp)."""
    R, T, X, k = (a.copy() for a in state)
    cam_col, kcols, m, N = layout(sc)
    for c, c0 in cam_col.items():
        R[c] = R[c] @ rot(delta[c0:c0 + 3])
        T[c] = T[c] + delta[c0 + 3:c0 + 6]
    for b, col in kcols:
        k[b] = k[b] + delta[col]
    X = X + delta[m:].reshape(-1, 3)
    return R, T, X, k


def dense_system(sc, state):
    """Stacked whitened residual r, Jacobian J (rows: 2 per observation, then
    6 prior rows per free camera) and IRLS weights per row."""
    cam_col, kcols, m, N = layout(sc)
    O, C = sc["n_obs"], sc["n_cams"]
    res = oracle.residuals(sc, state)
    jac = oracle.jacobians(sc, state)
    e_pr, Jw_pr = oracle.prior(sc, state)
    sig = float(sc["sigma_px"])
    free = sorted(cam_col)
    rows = 2 * O + 6 * len(free)
    J = np.zeros((rows, N))
    r = np.zeros(rows)
    wrow = np.ones(rows)
    for o in range(O):
        c, j = sc["obs_cam"][o], sc["obs_pt"][o]
        sl = slice(2 * o, 2 * o + 2)
        r[sl] = res["e"][o]
        wrow[sl] = res["w"][o]
        if c in cam_col:
            c0 = cam_col[c]
            J[sl, c0:c0 + 3] = jac["Jw"][o] / sig
            J[sl, c0 + 3:c0 + 6] = jac["JT"][o] / sig
        for b, col in kcols:
            J[sl, col] = (jac["Jk"][o][:, b] if b < 2 else jac["Ji"][o][:, b - 2]) / sig
        J[sl, m + 3 * j:m + 3 * j + 3] = jac["JX"][o] / sig
    for i, c in enumerate(free):
        base = 2 * O + 6 * i
        c0 = cam_col[c]
        r[base:base + 6] = e_pr[c]
        J[base:base + 3, c0:c0 + 3] = Jw_pr[c]
        sT = sc["prior_sigma"][c, 3:]
        inv = np.where((sT > 0) & np.isfinite(sT), 1.0 / np.where(sT > 0, sT, 1.0), 0.0)
        J[base + 3:base + 6, c0 + 3:c0 + 6] = np.diag(inv)
    return r, J, wrow


def dense_normal(sc, state):
    r, J, w = dense_system(sc, state)
    H = J.T @ (w[:, None] * J)
    g = J.T @ (w * r)
    return H, g


def fd_gradient(sc, state, h=1e-6):
    _, _, m, N = layout(sc)
    g = np.zeros(N)
    for i in range(N):
        d = np.zeros(N)
        d[i] = h
        ep = oracle.cost(sc, boxplus(sc, state, d))
        d[i] = -h
        em = oracle.cost(sc, boxplus(sc, state, d))
        g[i] = (ep - em) / (2 * h)
    return g
