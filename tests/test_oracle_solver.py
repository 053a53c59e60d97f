"""Pins of the oracle's Levenberg-Marquardt solve: the Schur-complement step
against a dense solve of the damped normal equations, the gradient against
finite differences of the cost, the optimum against generic minimisers, and
closed-form special cases (noise-free convergence, prior-only problems,
triangulation with fixed cameras)."""
import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

import oracle
from bruteforce import boxplus, dense_normal, dense_system, fd_gradient, layout, rot
from synth import aerial as A


def micro(seed, **kw):
    return A.make_scene(A.spec_micro(**kw), seed)


SCENES = [
    dict(seed=101, n_strips=2, imgs_per_strip=1, n_points=12),
    dict(seed=102, n_strips=2, imgs_per_strip=2, n_points=60, k_true=(-0.05, 0.02), intr_mask=3),
    dict(seed=103, n_strips=2, imgs_per_strip=3, n_points=200, n_fixed=2, intr_mask=1, k_true=(-0.05, 0.0)),
    dict(seed=104, n_strips=3, imgs_per_strip=2, n_points=120, intr_mask=2, k_true=(0.0, 0.02),
         outlier_frac=0.1),
    # self-calibration: f, cx, cy in the intrinsic border (bits 2, 3, 4)
    dict(seed=105, n_strips=2, imgs_per_strip=2, n_points=80, k_true=(-0.05, 0.02), intr_mask=0b11111),
    dict(seed=106, n_strips=2, imgs_per_strip=3, n_points=150, n_fixed=1, intr_mask=0b11100),
    dict(seed=107, n_strips=3, imgs_per_strip=2, n_points=120, intr_mask=0b01101, k_true=(-0.05, 0.0),
         outlier_frac=0.1),
]


@pytest.mark.parametrize("cfg", SCENES, ids=lambda c: str(c["seed"]))
def test_gradient_matches_finite_difference_of_cost(cfg):
    cfg = dict(cfg)
    sc = micro(cfg.pop("seed"), **cfg)
    state = oracle.initial_state(sc)
    H, g = dense_normal(sc, state)
    gfd = fd_gradient(sc, state, h=1e-6)
    assert np.linalg.norm(g - gfd) <= 1e-5 * np.linalg.norm(gfd)


@pytest.mark.parametrize("cfg", SCENES, ids=lambda c: str(c["seed"]))
@pytest.mark.parametrize("lam", [1e-4, 1e-1, 10.0])
def test_schur_step_equals_dense_damped_solve(cfg, lam):
    """(H + lambda D) delta = -g with D = clamp(diag H, 1e-6, 1e32), solved
    densely by scipy Cholesky, equals the oracle's Schur-complement step to
    1e-10 (compared in Jacobi-scaled variables)."""
    cfg = dict(cfg)
    sc = micro(cfg.pop("seed"), **cfg)
    state = oracle.initial_state(sc)
    H, g = dense_normal(sc, state)
    D = np.clip(np.diag(H), 1e-6, 1e32)
    Hl = H + lam * np.diag(D)
    want = scipy.linalg.cho_solve(scipy.linalg.cho_factor(Hl), -g)
    rc, got, pred = oracle.step(sc, state, lam)
    assert rc == 0
    s = np.sqrt(np.diag(Hl))
    assert np.linalg.norm(s * (got - want)) <= 1e-10 * np.linalg.norm(s * want)
    assert pred == pytest.approx(0.5 * want @ (lam * D * want - g), rel=1e-9)


def test_pred_reduction_equals_model_decrease():
    """pred = E - m(delta) for the local quadratic model m."""
    sc = micro(105, n_points=50)
    state = oracle.initial_state(sc)
    H, g = dense_normal(sc, state)
    rc, d, pred = oracle.step(sc, state, 1e-2)
    assert pred == pytest.approx(-(g @ d) - 0.5 * d @ H @ d, rel=1e-9)


def test_noise_free_converges_to_truth():
    """No pixel noise, no outliers, priors at the truth: E -> ~0 and the truth
    is recovered from a perturbed start."""
    sc = micro(106, n_strips=2, imgs_per_strip=3, n_points=150, noise_px=0.0, outlier_frac=0.0,
               priors_at_truth=True, k_true=(-0.05, 0.02), intr_mask=3)
    r = oracle.solve(sc, max_iters=40)
    E0, E = r["cost_log"][0], r["cost_log"][-1]
    assert E < 1e-20 * E0 or E < 1e-16
    R, T, X, k = r["state"]
    tr = sc["truth"]
    assert np.abs(T - tr["T"]).max() < 1e-7
    assert np.abs(X - tr["X"]).max() < 1e-6
    assert np.abs(k - tr["k"]).max() < 1e-10


def test_truth_is_stationary():
    """State = priors = truth with noise-free observations: g = 0 and the step
    is zero."""
    sc = micro(107, n_points=80, noise_px=0.0, outlier_frac=0.0, priors_at_truth=True)
    tr = sc["truth"]
    state = (tr["R"].copy(), tr["T"].copy(), tr["X"].copy(), tr["k"].copy())
    H, g = dense_normal(sc, state)
    assert np.abs(g).max() < 1e-9
    rc, d, pred = oracle.step(sc, state, 1e-4)
    assert np.abs(d).max() < 1e-12


def _prior_only(T_off, R_off=None, C=3):
    R = np.stack([A.R_NADIR @ rot([0.01 * c, 0.0, 0.02]) for c in range(C)])
    T = np.array([[10.0 * c, 5.0, 300.0] for c in range(C)])
    Rp = R.copy() if R_off is None else np.stack([R[c] @ rot(R_off[c]) for c in range(C)])
    Tp = T + T_off
    return {
        "n_cams": C, "n_points": 0, "n_obs": 0, "R": R, "T": T, "X": np.zeros((0, 3)), "k": np.zeros(2),
        "prior_R": Rp, "prior_T": Tp,
        "prior_sigma": np.column_stack([np.full((C, 3), 8.7e-4), np.full((C, 3), 0.5)]),
        "fixed": np.zeros(C, np.uint8), "obs_cam": np.zeros(0, np.int32), "obs_pt": np.zeros(0, np.int32),
        "obs_uv": np.zeros((0, 2)), "f": A.F_PX, "cx": A.CX, "cy": A.CY, "intr_mask": 0,
        "sigma_px": 0.5, "huber_delta": 1.0,
    }


def test_prior_only_translation_is_one_quadratic_step():
    """A translation-only prior problem is quadratic: the step lands at
    1/(1+lambda) of the way, the gain ratio is exactly 1 and Nielsen's update
    divides lambda by 3."""
    off = np.array([[0.3, -0.2, 0.1], [1.0, 0.0, -0.5], [0.0, 0.4, 0.0]])
    sc = _prior_only(off)
    lam0 = 1e-2
    r = oracle.solve(sc, max_iters=1, lambda0=lam0)
    R, T, X, k = r["state"]
    np.testing.assert_allclose(T - sc["T"], off / (1 + lam0), rtol=1e-12, atol=1e-14)
    assert r["rho_log"][0] == pytest.approx(1.0, abs=1e-9)
    assert r["lambda"] == pytest.approx(lam0 / 3.0, rel=1e-12)
    E0 = 0.5 * ((off / 0.5) ** 2).sum()
    assert r["cost_log"][1] == pytest.approx(E0 * (lam0 / (1 + lam0)) ** 2, rel=1e-9)


def test_prior_only_rotation_reaches_prior():
    rng = np.random.default_rng(9)
    sc = _prior_only(np.zeros((3, 3)), R_off=rng.normal(0, 0.02, (3, 3)))
    r = oracle.solve(sc, max_iters=3, lambda0=1e-12)
    R = r["state"][0]
    for c in range(3):
        d = np.linalg.norm(scipy.spatial.transform.Rotation.from_matrix(sc["prior_R"][c].T @ R[c]).as_rotvec())
        assert d < 1e-12


def test_fixed_cameras_reduce_to_triangulation():
    """All cameras fixed, noise-free observations: the adjustment reduces to
    independent multi-view triangulations, whose linear (DLT) solution is
    exact; LM must reach it."""
    sc = micro(108, n_strips=2, imgs_per_strip=3, n_points=60, noise_px=0.0, outlier_frac=0.0,
               n_fixed=6, point_noise_m=3.0)
    tr = sc["truth"]
    sc["R"], sc["T"] = tr["R"].copy(), tr["T"].copy()
    r = oracle.solve(sc, max_iters=30)
    X = r["state"][2]
    K = np.array([[A.F_PX, 0, A.CX], [0, A.F_PX, A.CY], [0, 0, 1.0]])
    for j in range(sc["n_points"]):
        rows = []
        for o in np.nonzero(sc["obs_pt"] == j)[0]:
            c = sc["obs_cam"][o]
            Pm = K @ np.hstack([tr["R"][c].T, (-tr["R"][c].T @ tr["T"][c])[:, None]])
            u, v = sc["obs_uv"][o]
            rows += [u * Pm[2] - Pm[0], v * Pm[2] - Pm[1]]
        _, _, Vt = np.linalg.svd(np.array(rows))
        Xh = Vt[-1, :3] / Vt[-1, 3]
        np.testing.assert_allclose(X[j], Xh, atol=1e-6)


def _flat_cost(sc, state0):
    _, _, m, N = layout(sc)

    def f(x):
        return oracle.cost(sc, boxplus(sc, state0, x))

    def grad(x):
        st = boxplus(sc, state0, x)
        H, g = dense_normal(sc, st)
        # g is the gradient w.r.t. a right perturbation at st; the chain rule
        # to x goes through the right Jacobian of the rotation, so use finite
        # differences in x for the rotation columns only.
        cam_col, kcols, m_, N_ = layout(sc)
        gx = g.copy()
        h = 1e-7
        for c, c0 in cam_col.items():
            for i in range(3):
                d = np.zeros(N)
                d[c0 + i] = h
                gx[c0 + i] = (f(x + d) - f(x - d)) / (2 * h)
        return gx

    return f, grad, N


def test_optimum_matches_lbfgs_with_huber():
    """With Huber active the IRLS Gauss-Newton iteration converges linearly;
    run it until the damping stalls and check that an independent quasi-Newton
    minimiser started there finds no lower cost, and that the gradient vanished."""
    sc = micro(109, n_strips=2, imgs_per_strip=2, n_points=25, outlier_frac=0.08)
    r = oracle.solve(sc, max_iters=20000)
    E_lm = r["cost_log"][-1]
    f, grad, N = _flat_cost(sc, r["state"])
    res = scipy.optimize.minimize(f, np.zeros(N), jac=grad, method="L-BFGS-B",
                                  options={"gtol": 1e-12, "ftol": 1e-16, "maxiter": 3000})
    assert res.fun >= E_lm * (1 - 1e-10)
    H, g = dense_normal(sc, r["state"])
    H0, g0 = dense_normal(sc, oracle.initial_state(sc))
    assert np.abs(g).max() < 1e-6 * np.abs(g0).max()


def test_optimum_matches_scipy_lm_without_huber():
    """Without Huber the cost is a plain sum of squares: MINPACK's LM (scipy)
    reaches the same minimum from the start, and cannot lower the oracle's."""
    sc = micro(110, n_strips=2, imgs_per_strip=2, n_points=30, outlier_frac=0.0, huber_delta_px=1e9)
    r = oracle.solve(sc, max_iters=200, stop_on_ftol=True, ftol=1e-15)
    E_or = r["cost_log"][-1]
    _, _, m, N = layout(sc)

    for start in (oracle.initial_state(sc), r["state"]):
        def resid(x, start=start):
            rr, J, w = dense_system(sc, boxplus(sc, start, x))
            return rr

        sol = scipy.optimize.least_squares(resid, np.zeros(N), method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15)
        E_sp = 0.5 * (sol.fun ** 2).sum()
        assert E_sp >= E_or * (1 - 1e-12)
        assert E_sp == pytest.approx(E_or, rel=1e-6)


def test_lm_accepts_only_decreasing_steps_and_follows_nielsen():
    sc = micro(111, n_strips=2, imgs_per_strip=3, n_points=150, outlier_frac=0.05, k_true=(-0.05, 0.02),
               intr_mask=3)
    r = oracle.solve(sc, max_iters=25, lambda0=1e-8)
    cl = r["cost_log"]
    assert np.all(np.diff(cl) <= 0)
    lam = r["lambda_log"]
    for i in range(len(lam) - 1):
        if r["accepted_log"][i]:
            t = 2 * r["rho_log"][i] - 1
            assert lam[i + 1] == pytest.approx(max(lam[i] * max(1 / 3, 1 - t ** 3), 1e-16), rel=1e-12)
            assert r["rho_log"][i] > 1e-3
        else:
            assert lam[i + 1] > lam[i]


def test_self_calibration_noise_free_recovers_f_cx_cy():
    """Self-calibration (Sec. 5 names it as a variant): noise-free
    observations, priors at the truth, f, cx, cy started 0.3 %, +4 px and
    -3 px off the truth with k1, k2 also estimated: E -> ~0 and the truth,
    intrinsics included, is recovered."""
    sc = micro(121, n_strips=2, imgs_per_strip=3, n_points=200, noise_px=0.0, outlier_frac=0.0,
               priors_at_truth=True, k_true=(-0.05, 0.02), intr_mask=0b11111)
    f0, cx0, cy0 = sc["f"], sc["cx"], sc["cy"]
    sc = dict(sc, f=f0 * 1.003, cx=cx0 + 4.0, cy=cy0 - 3.0)
    r = oracle.solve(sc, max_iters=60)
    E0, E = r["cost_log"][0], r["cost_log"][-1]
    assert E < 1e-18 * E0 or E < 1e-16
    R, T, X, k = r["state"]
    tr = sc["truth"]
    assert k.size == 5
    assert np.abs(k[:2] - tr["k"]).max() < 1e-9
    assert abs(k[2] - f0) < 1e-6 * f0 and abs(k[3] - cx0) < 1e-6 and abs(k[4] - cy0) < 1e-6
    assert np.abs(r["intr"] - k[2:]).max() == 0.0
    assert np.abs(T - tr["T"]).max() < 1e-6


def test_self_calibration_jacobian_columns_closed_form():
    """d(u, v)/d(f, cx, cy) = [[D a, 1, 0], [D b, 0, 1]] with D the radial
    factor, from the predicted pixel: (u - cx) / f = D a."""
    sc = micro(122, n_strips=2, imgs_per_strip=2, n_points=30, k_true=(-0.05, 0.02), intr_mask=0b11111)
    st = oracle.initial_state(sc)
    jac = oracle.jacobians(sc, st)
    uv = oracle.residuals(sc, st)["uv"]
    Da = (uv[:, 0] - sc["cx"]) / sc["f"]
    Db = (uv[:, 1] - sc["cy"]) / sc["f"]
    Ji = jac["Ji"]
    assert np.abs(Ji[:, 0, 0] - Da).max() < 1e-12 and np.abs(Ji[:, 1, 0] - Db).max() < 1e-12
    assert np.all(Ji[:, 0, 1] == 1) and np.all(Ji[:, 1, 2] == 1) and np.all(Ji[:, 0, 2] == 0) and np.all(Ji[:, 1, 1] == 0)


def test_self_calibration_optimum_matches_scipy_lm():
    """f, cx, cy estimated, no Huber: MINPACK's LM from the start reaches the
    oracle's minimum and cannot lower it."""
    sc = micro(123, n_strips=2, imgs_per_strip=2, n_points=40, outlier_frac=0.0, huber_delta_px=1e9,
               intr_mask=0b11100)
    sc = dict(sc, f=sc["f"] * 1.002, cx=sc["cx"] + 2.0)
    r = oracle.solve(sc, max_iters=300, stop_on_ftol=True, ftol=1e-15)
    E_or = r["cost_log"][-1]
    _, _, m, N = layout(sc)
    for start in (oracle.initial_state(sc), r["state"]):
        def resid(x, start=start):
            rr, J, w = dense_system(sc, boxplus(sc, start, x))
            return rr

        sol = scipy.optimize.least_squares(resid, np.zeros(N), method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15)
        E_sp = 0.5 * (sol.fun ** 2).sum()
        assert E_sp >= E_or * (1 - 1e-12)
        assert E_sp == pytest.approx(E_or, rel=1e-6)
