"""Pins of the oracle's Levenberg-Marquardt control away from the quadratic
case: the gain ratio of a non-quadratic step, Nielsen's damping update at a
gain ratio other than 1 (including a ratio below 1/2, where the damping
grows), and the reject branch (a trial at non-positive depth, and a trial
whose cost rises).

The problem: one tie point seen by two fixed cameras (the reduced system is
empty, the unknowns are the point's three coordinates), noise-free
observations of its true position, the Huber threshold so large that every
residual stays on the quadratic branch (E = 1/2 sum |e / sigma|^2), and the
point started on the ray of the first camera at 1.8 or 4 times its true
depth.  Started that deep, the Gauss-Newton depth step overshoots past the
cameras (a depth error scales like z^2, so the linear model predicts a step
of about z0 (1 - z0 / z*)).

The test replays the iteration with code of its own: residuals from the
scene generator's projection (not the oracle's), the Jacobian by central
differences, the damped normal equations solved by numpy, and the damping
rules written out below.  The oracle must take the same decisions, with the
same gain ratios and damping, iteration by iteration.

Damping rules (Marquardt scaling, Nielsen's update): D = clamp(diag H, 1e-6,
1e32), step (H + lam D) d = -g, predicted reduction L = d^T (lam D d - g) / 2,
gain ratio rho = (E - E') / L; accept iff rho > 1e-3 and E' is finite, then
lam <- lam max(1/3, 1 - (2 rho - 1)^3) and nu <- 2; otherwise lam <- lam nu
and nu <- 2 nu.  A trial with a point at non-positive depth is rejected.
"""
import numpy as np
import pytest

import oracle
from synth import aerial as A


def one_point_scene(depth_factor):
    base = A.make_scene(A.spec_micro(n_strips=1, imgs_per_strip=2, n_points=30, noise_px=0.0, outlier_frac=0.0), 501)
    op = base["obs_pt"]
    j = int(np.argmax(np.bincount(op) == 2))
    sel = np.where(op == j)[0]
    Xt = base["truth"]["X"][j]
    sc = dict(base)
    sc.update(n_points=1, n_obs=2, obs_cam=base["obs_cam"][sel].astype(np.int32), obs_pt=np.zeros(2, np.int32),
              fixed=np.ones(base["n_cams"], np.uint8), huber_delta=1e9, R=base["truth"]["R"], T=base["truth"]["T"],
              intr_mask=0, k=np.zeros(2))
    sc["obs_uv"] = A.project_obs(sc["R"], sc["T"], Xt[None], (0.0, 0.0), sc["obs_cam"], sc["obs_pt"])
    c0 = int(sc["obs_cam"][0])
    sc["X"] = (sc["T"][c0] + depth_factor * (Xt - sc["T"][c0]))[None].copy()
    return sc


def replay(sc, lam, n_iters):
    """The LM iteration on the point alone, written out with numpy."""
    R, T = sc["R"], sc["T"]
    cams, uv, sig = sc["obs_cam"], sc["obs_uv"], sc["sigma_px"]

    def depths(X):
        return np.array([(R[c].T @ (X - T[c]))[2] for c in cams])

    def resid(X):
        return ((A.project_obs(R, T, X[None], (0.0, 0.0), cams, np.zeros(len(cams), np.int32)) - uv) / sig).ravel()

    def cost(X):
        return np.inf if np.any(depths(X) <= 0) else 0.5 * float(resid(X) @ resid(X))

    X, nu, E = sc["X"][0].copy(), 2.0, cost(sc["X"][0])
    log = []
    for _ in range(n_iters):
        h = 1e-4
        J = np.column_stack([(resid(X + h * e) - resid(X - h * e)) / (2 * h) for e in np.eye(3)])
        r = resid(X)
        H, g = J.T @ J, J.T @ r
        D = np.clip(np.diag(H), 1e-6, 1e32)
        d = np.linalg.solve(H + lam * np.diag(D), -g)
        pred = 0.5 * d @ (lam * D * d - g)
        E2 = cost(X + d)
        rho = (E - E2) / pred if np.isfinite(E2) else -np.inf
        acc = bool(np.isfinite(E2) and rho > 1e-3)
        log.append((lam, rho, acc))
        if acc:
            X, E = X + d, E2
            lam *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
            nu = 2.0
        else:
            lam *= nu
            nu *= 2.0
    return log, lam, nu


@pytest.mark.parametrize("depth_factor,lam0,expect", [
    # two trials behind the cameras, then an accepted step at rho ~ 0.56
    (4.0, 0.0215, [0, 0, 1, 1, 1]),
    # two trials whose cost rises (rho ~ -7.5, -4.0), then an accepted step
    # at rho ~ 0.35, where Nielsen's update raises the damping
    (1.8, 0.01, [0, 0, 1, 1, 1]),
])
def test_lm_control_matches_written_out_iteration(depth_factor, lam0, expect):
    sc = one_point_scene(depth_factor)
    n = len(expect)
    mine, lam_end, nu_end = replay(sc, lam0, n)
    ref = oracle.solve(sc, max_iters=n, lambda0=lam0)
    print("replay lam", [f"{l:.6g}" for l, _, _ in mine], "rho", [f"{r:.6g}" for _, r, _ in mine])
    print("oracle lam", ref["lambda_log"], "rho", ref["rho_log"])
    assert [int(a) for _, _, a in mine] == expect
    assert ref["accepted_log"].tolist() == expect
    assert ref["rejected"] == expect.count(0)
    for i, (lam, rho, acc) in enumerate(mine):
        assert ref["lambda_log"][i] == pytest.approx(lam, rel=1e-9)
        if np.isfinite(rho):
            assert ref["rho_log"][i] == pytest.approx(rho, rel=1e-6)
        else:
            assert ref["rho_log"][i] == -np.inf
    assert ref["lambda"] == pytest.approx(lam_end, rel=1e-6)
    assert ref["nu"] == nu_end
    # the accepted steps' gain ratios are away from 1 (the update is not the
    # clamped 1/3), and for the second case below 1/2 (the damping grows)
    first_acc = expect.index(1)
    rho = mine[first_acc][1]
    assert 0.2 < rho < 0.8
    if depth_factor == 1.8:
        assert rho < 0.5 and ref["lambda_log"][first_acc + 1] > ref["lambda_log"][first_acc]
        assert all(np.isfinite(r) and r < 0 for _, r, _ in mine[:first_acc])
    else:
        assert all(r == -np.inf for _, r, _ in mine[:first_acc])
