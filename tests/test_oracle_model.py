"""Pins of the oracle's camera model, robust cost, priors and Jacobians against
the paper's closed forms and against independent mathematics."""
import dataclasses

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from bruteforce import boxplus, dense_system, layout, rot
from synth import aerial as A

F, CX, CY = A.F_PX, A.CX, A.CY


def mini_scene(R, T, X, obs_cam, obs_pt, uv=None, k=(0.0, 0.0), intr_mask=0, sigma=0.5,
               delta=1.0, prior_sigma=None, prior_R=None, prior_T=None, fixed=None):
    R = np.ascontiguousarray(R, np.float64).reshape(-1, 3, 3)
    T = np.ascontiguousarray(T, np.float64).reshape(-1, 3)
    X = np.ascontiguousarray(X, np.float64).reshape(-1, 3)
    C, P, O = R.shape[0], X.shape[0], len(obs_cam)
    return {
        "n_cams": C, "n_points": P, "n_obs": O,
        "R": R, "T": T, "X": X, "k": np.array(k, np.float64),
        "prior_R": R.copy() if prior_R is None else np.asarray(prior_R, np.float64),
        "prior_T": T.copy() if prior_T is None else np.asarray(prior_T, np.float64),
        "prior_sigma": np.zeros((C, 6)) if prior_sigma is None else np.asarray(prior_sigma, np.float64),
        "fixed": np.zeros(C, np.uint8) if fixed is None else np.asarray(fixed, np.uint8),
        "obs_cam": np.asarray(obs_cam, np.int32), "obs_pt": np.asarray(obs_pt, np.int32),
        "obs_uv": np.zeros((O, 2)) if uv is None else np.asarray(uv, np.float64),
        "f": F, "cx": CX, "cy": CY, "intr_mask": intr_mask,
        "sigma_px": sigma, "huber_delta": delta,
    }


def predicted(sc, state=None):
    if state is None:
        state = oracle.initial_state(sc)
    return oracle.residuals(sc, state)["uv"]


def test_eq3_transfer_round_trip():
    """Eq. (3): a patch centre back-projected from I_0 with depth lambda along
    R_0 K^-1 p~ and re-projected by pi(K R_k^T (. - T_k)) lands on the same
    pixel for k = 0, and on the Eq. (3) prediction for any other image."""
    rng = np.random.default_rng(3)
    K = np.array([[F, 0, CX], [0, F, CY], [0, 0, 1.0]])
    R = np.stack([A.heading_matrix(a) @ A.R_NADIR @ rot(rng.normal(0, 0.05, 3)) for a in (0.3, 2.0)])
    T = np.array([[10.0, -4.0, 300.0], [40.0, 25.0, 310.0]])
    for _ in range(20):
        p = np.array([rng.uniform(0, 8000), rng.uniform(0, 6000), 1.0])
        lam = rng.uniform(250, 320)
        X = T[0] + lam * R[0] @ np.linalg.solve(K, p)
        sc = mini_scene(R, T, X[None], [0, 1], [0, 0])
        uv = predicted(sc)
        np.testing.assert_allclose(uv[0], p[:2], rtol=0, atol=1e-7)
        q = K @ R[1].T @ (X - T[1])
        np.testing.assert_allclose(uv[1], q[:2] / q[2], rtol=0, atol=1e-7)


def test_nadir_point_below_projects_to_principal_point():
    R = A.R_NADIR[None]
    T = np.array([[12.0, 34.0, 300.0]])
    sc = mini_scene(R, T, np.array([[12.0, 34.0, 17.0]]), [0], [0])
    np.testing.assert_allclose(predicted(sc)[0], [CX, CY], atol=1e-9)


def test_nadir_axes_image_y_down_points_south():
    """With R columns = camera axes in ENU, a point east of a nadir camera
    heading north appears right of the centre, a point north appears above."""
    R = A.R_NADIR[None]
    T = np.array([[0.0, 0.0, 300.0]])
    sc = mini_scene(R, T, np.array([[10.0, 0, 0], [0, 10.0, 0]]), [0, 0], [0, 1])
    uv = predicted(sc)
    assert uv[0, 0] > CX and abs(uv[0, 1] - CY) < 1e-9
    assert uv[1, 1] < CY and abs(uv[1, 0] - CX) < 1e-9


@pytest.mark.parametrize("k1,k2", [(-0.05, 0.02), (0.1, -0.03), (0.0, 0.0)])
def test_radial_distortion_closed_form(k1, k2):
    """A point at normalised radius r images at radius f r (1 + k1 r^2 + k2 r^4)
    along the same azimuth."""
    R = A.R_NADIR[None]
    T = np.array([[0.0, 0.0, 300.0]])
    rng = np.random.default_rng(5)
    pts, want = [], []
    for _ in range(10):
        r = rng.uniform(0.0, 0.4)
        phi = rng.uniform(0, 2 * np.pi)
        z = 280.0
        xc = np.array([r * np.cos(phi) * z, r * np.sin(phi) * z, z])
        pts.append(T[0] + R[0] @ xc)
        rad = F * r * (1 + k1 * r**2 + k2 * r**4)
        want.append([CX + rad * np.cos(phi), CY + rad * np.sin(phi)])
    sc = mini_scene(R, T, np.array(pts), [0] * 10, list(range(10)), k=(k1, k2))
    np.testing.assert_allclose(predicted(sc), np.array(want), atol=1e-8)


def test_huber_cost_is_textbook_huber_on_residual_norm():
    """Per observation the cost is 1/2 Huber_d(|e|/sigma) with the textbook
    Huber function (quadratic inside d, linear outside), d = delta/sigma."""
    R = A.R_NADIR[None]
    T = np.array([[0.0, 0.0, 300.0]])
    X = np.array([[1.0, 2.0, 0.0]])
    sigma, delta = 0.5, 1.0
    base = mini_scene(R, T, X, [0], [0], sigma=sigma, delta=delta)
    uv0 = predicted(base)[0]
    d = delta / sigma
    for off in [0.0, 0.3, 0.99, 1.0, 1.01, 3.0, 75.0]:
        ang = 0.7
        uv = uv0 + off * np.array([np.cos(ang), np.sin(ang)])
        sc = mini_scene(R, T, X, [0], [0], uv=uv[None], sigma=sigma, delta=delta)
        r = off / sigma
        huber = r * r if r <= d else 2 * d * r - d * d
        assert oracle.cost(sc, oracle.initial_state(sc)) == pytest.approx(0.5 * huber, rel=1e-12, abs=1e-15)
        res = oracle.residuals(sc, oracle.initial_state(sc))
        # IRLS weight = d rho / d s
        s = r * r
        hs = 1e-6 * max(s, 1.0)
        rho = lambda t: t if t <= d * d else 2 * d * np.sqrt(t) - d * d
        if abs(s - d * d) > 1e-3:
            assert res["w"][0] == pytest.approx((rho(s + hs) - rho(max(s - hs, 0))) / (s + hs - max(s - hs, 0)), rel=1e-6)


def test_huber_large_delta_is_least_squares():
    sc = A.make_scene(A.spec_micro(n_points=30, huber_delta_px=1e9, outlier_frac=0.0, priors=False), 11)
    st = oracle.initial_state(sc)
    res = oracle.residuals(sc, st)
    assert oracle.cost(sc, st) == pytest.approx(0.5 * (res["e"] ** 2).sum(), rel=1e-13)


def test_prior_residual_matches_scipy_log():
    rng = np.random.default_rng(7)
    C = 5
    Rp = np.stack([rot(rng.normal(0, 1, 3)) for _ in range(C)])
    angles = [1e-9, 1e-5, 0.3, 2.0, 3.1]
    R = np.stack([Rp[c] @ rot(angles[c] * rng.normal(0, 1, 3) / np.sqrt(3)) for c in range(C)])
    T = rng.normal(0, 5, (C, 3))
    Tp = T + rng.normal(0, 1, (C, 3))
    sig = np.column_stack([np.full((C, 3), 1e-3), np.full((C, 3), 0.5)])
    sc = mini_scene(R, T, np.zeros((0, 3)), [], [], prior_R=Rp, prior_T=Tp, prior_sigma=sig)
    e, _ = oracle.prior(sc, oracle.initial_state(sc))
    for c in range(C):
        want_w = Rotation.from_matrix(Rp[c].T @ R[c]).as_rotvec() / 1e-3
        np.testing.assert_allclose(e[c, :3], want_w, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(e[c, 3:], (T[c] - Tp[c]) / 0.5, rtol=1e-14)


def test_prior_jacobian_finite_difference():
    rng = np.random.default_rng(8)
    C = 4
    Rp = np.stack([rot(rng.normal(0, 1, 3)) for _ in range(C)])
    R = np.stack([Rp[c] @ rot(a * rng.normal(0, 1, 3)) for c, a in enumerate([1e-6, 0.01, 0.5, 1.5])])
    sc = mini_scene(R, np.zeros((C, 3)), np.zeros((0, 3)), [], [], prior_R=Rp,
                    prior_sigma=np.column_stack([np.full((C, 3), 2e-3), np.ones((C, 3))]))
    _, Jw = oracle.prior(sc, oracle.initial_state(sc))
    h = 1e-6
    for c in range(C):
        fd = np.zeros((3, 3))
        for i in range(3):
            d = np.zeros(3)
            d[i] = h
            ep = Rotation.from_matrix(Rp[c].T @ R[c] @ rot(d)).as_rotvec() / 2e-3
            em = Rotation.from_matrix(Rp[c].T @ R[c] @ rot(-d)).as_rotvec() / 2e-3
            fd[:, i] = (ep - em) / (2 * h)
        assert np.linalg.norm(Jw[c] - fd) <= 1e-6 * np.linalg.norm(fd)


def _fd_obs_jacobians(sc, state):
    """Central differences of the predicted pixels through scipy rotations."""
    R, T, X, k = state
    O = sc["n_obs"]
    out = {"Jw": np.zeros((O, 2, 3)), "JT": np.zeros((O, 2, 3)), "JX": np.zeros((O, 2, 3)), "Jk": np.zeros((O, 2, 2))}
    hw, ht, hk = 1e-6, 1e-4, 1e-2   # the pixel is linear in k1, k2
    cam, pt = sc["obs_cam"], sc["obs_pt"]
    for i in range(3):
        for sgn in (1, -1):
            d = np.zeros(3)
            d[i] = sgn * hw
            Rp = np.stack([R[c] @ rot(d) for c in range(len(R))])
            uv = predicted(sc, (Rp, T, X, k))
            out["Jw"][:, :, i] += sgn * uv / (2 * hw)
            d = np.zeros(3)
            d[i] = sgn * ht
            uv = predicted(sc, (R, T + d, X, k))
            out["JT"][:, :, i] += sgn * uv / (2 * ht)
            uv = predicted(sc, (R, T, X + d, k))
            out["JX"][:, :, i] += sgn * uv / (2 * ht)
    for b in range(2):
        for sgn in (1, -1):
            kk = k.copy()
            kk[b] += sgn * hk
            out["Jk"][:, :, b] += sgn * predicted(sc, (R, T, X, kk)) / (2 * hk)
    return out


def test_observation_jacobians_finite_difference():
    """Analytic Jacobians vs central differences (relative Frobenius error per
    block <= 1e-6), with radial distortion active."""
    spec = A.spec_micro(n_strips=2, imgs_per_strip=3, n_points=60, k_true=(-0.05, 0.02), k_init=(-0.04, 0.01))
    sc = A.make_scene(spec, 21)
    state = oracle.initial_state(sc)
    J = oracle.jacobians(sc, state)
    fd = _fd_obs_jacobians(sc, state)
    for name in ("Jw", "JT", "JX", "Jk"):
        for o in range(sc["n_obs"]):
            err = np.linalg.norm(J[name][o] - fd[name][o])
            assert err <= 1e-6 * np.linalg.norm(fd[name][o]), (name, o, err)


def test_gauge_null_space_without_priors():
    """With priors off and intrinsics fixed, the 7 similarity generators lie in
    the null space of the observation Jacobian."""
    spec = A.spec_micro(n_strips=2, imgs_per_strip=2, n_points=50, priors=False, k_true=(-0.05, 0.02),
                        k_init=(-0.05, 0.02))
    sc = A.make_scene(spec, 31)
    state = oracle.initial_state(sc)
    R, T, X, k = state
    r, J, w = dense_system(sc, state)
    Jo = J[: 2 * sc["n_obs"]]
    cam_col, kcols, m, N = layout(sc)
    gens = []
    for i in range(3):
        t = np.zeros(3)
        t[i] = 1.0
        n = np.zeros(N)
        for c, c0 in cam_col.items():
            n[c0 + 3:c0 + 6] = t
        n[m:] = np.tile(t, sc["n_points"])
        gens.append(n)
        th = np.zeros(3)
        th[i] = 1.0
        n = np.zeros(N)
        for c, c0 in cam_col.items():
            n[c0:c0 + 3] = R[c].T @ th
            n[c0 + 3:c0 + 6] = np.cross(th, T[c])
        n[m:] = np.cross(th, X).reshape(-1)
        gens.append(n)
    n = np.zeros(N)
    for c, c0 in cam_col.items():
        n[c0 + 3:c0 + 6] = T[c]
    n[m:] = X.reshape(-1)
    gens.append(n)
    for n in gens:
        Jn = Jo @ n
        assert np.linalg.norm(Jn) <= 1e-9 * np.linalg.norm(np.abs(Jo) @ np.abs(n))


def test_cost_invariant_under_similarity():
    spec = A.spec_micro(n_points=40, priors=False)
    sc = A.make_scene(spec, 41)
    R, T, X, k = oracle.initial_state(sc)
    E0 = oracle.cost(sc, (R, T, X, k))
    Q = rot([0.3, -0.2, 0.5])
    s, t = 1.7, np.array([100.0, -50.0, 20.0])
    R2 = np.einsum("ij,cjk->cik", Q, R)
    T2 = s * T @ Q.T + t
    X2 = s * X @ Q.T + t
    assert oracle.cost(sc, (R2, T2, X2, k)) == pytest.approx(E0, rel=1e-11)


def test_depth_nonpositive_gives_infinite_cost():
    R = A.R_NADIR[None]
    T = np.array([[0.0, 0.0, 300.0]])
    sc = mini_scene(R, T, np.array([[0.0, 0.0, 301.0]]), [0], [0])
    assert np.isinf(oracle.cost(sc, oracle.initial_state(sc)))
    assert oracle.residuals(sc, oracle.initial_state(sc))["bad"] == 1
