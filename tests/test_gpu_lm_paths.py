"""GPU parity of the Levenberg-Marquardt control on its reject and failure
paths (Sec. 3.2 minimises Eq. (7); the damping rules are the readings the
oracle follows: accept iff the gain ratio exceeds 1e-3 and the trial cost is
finite, Nielsen's update on acceptance, lam <- lam nu and nu <- 2 nu on
rejection, a failed factorisation or a point at non-positive depth in the
trial counted as a rejection, status "stalled" once lam exceeds 1e32).

Each scene makes the oracle reject steps, and the GPU must take the same
decisions: the accepted flag and the damping of every iteration, the cost
after every iteration (FP64 path within 1e-8 relative), the rejected count,
the final damping and growth factor, and the status.

  * a micro scene with one tie point started at 4 times its depth below the
    first camera that sees it: the first Gauss-Newton steps carry it behind
    the cameras (non-positive depth), then a trial whose cost rises, then an
    accepted step with a gain ratio near 0.66;
  * the one-point scenes of the oracle's own control pins (every camera
    fixed, the reduced system empty): trials behind the cameras, trials
    whose cost rises, accepted steps at gain ratios 0.34 and 0.55;
  * a camera whose attitude prior has sigma 1e-160 rad at an attitude equal
    to its prior: the prior's information overflows to infinity in H, so
    every factorisation of the reduced system fails, every step is rejected
    and the damping doubles its growth until it passes 1e32 (stalled after
    15 iterations).
"""
import numpy as np
import pytest

import oracle
from synth import aerial as A
from test_oracle_lm_control import one_point_scene

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1


def gpu_run(sc, iters, precision=FP64, **kw):
    from paper_2511_06152_amd import Context
    with Context(precision=precision) as ctx:
        t = ctx.submit(sc, max_iters=iters, **kw)
        ctx.ba_step(t, iters)
        return ctx.ba_fetch(t)


def deep_point_scene():
    sc = dict(A.make_scene(A.spec_micro(n_strips=2, imgs_per_strip=3, n_points=300), 401))
    cnt = np.bincount(sc["obs_pt"], minlength=sc["n_points"])
    j = next(j for j in range(sc["n_points"]) if cnt[j] == 2 and 0 in sc["obs_cam"][sc["obs_pt"] == j])
    sc["X"] = sc["X"].copy()
    sc["X"][j] = sc["T"][0] + 4.0 * (sc["truth"]["X"][j] - sc["T"][0])
    return sc


def stall_scene():
    sc = dict(A.make_scene(A.spec_micro(n_strips=2, imgs_per_strip=3, n_points=300), 402))
    for key in ("R", "prior_R", "prior_sigma"):
        sc[key] = sc[key].copy()
    sc["R"][0] = A.R_NADIR          # exactly representable: R_prior^T R = I exactly, a zero prior residual
    sc["prior_R"][0] = A.R_NADIR
    sc["prior_sigma"][0, :3] = 1e-160
    return sc


def check_control(got, ref, cost_tol=1e-8, lam_rtol=1e-6):
    """Same decisions, iteration by iteration; the damping within lam_rtol
    (after an accepted step it carries the gain ratio, which the FP32
    assembly of the mixed path moves by ~1e-5 relative)."""
    print("oracle acc", ref["accepted_log"].tolist(), "lam", ref["lambda_log"].tolist())
    print("gpu    acc", got["accepted_log"].tolist(), "lam", got["lambda_log"].tolist())
    print("oracle cost", ref["cost_log"].tolist())
    print("gpu    cost", got["cost_log"].tolist(), flush=True)
    assert got["iterations"] == ref["iterations"]
    assert got["accepted_log"].tolist() == ref["accepted_log"].tolist()
    assert got["rejected"] == ref["rejected"] and got["accepted"] == ref["accepted"]
    assert np.allclose(got["lambda_log"], ref["lambda_log"], rtol=lam_rtol, atol=0)
    assert got["lambda_"] == pytest.approx(ref["lambda"], rel=lam_rtol)
    assert got["nu"] == ref["nu"]
    a, b = np.asarray(got["cost_log"]), np.asarray(ref["cost_log"])
    if cost_tol is not None:
        assert np.all(np.abs(a - b) <= cost_tol * np.abs(b)), np.max(np.abs(a - b) / np.abs(b))


# oracle status codes: 0 max-iters, 1 converged, 2 stalled; library: 2, 3, 4
ORACLE_STATUS = {0: 2, 1: 3, 2: 4}


def test_deep_point_rejections_fp64():
    sc = deep_point_scene()
    ref = oracle.solve(sc, max_iters=14, lambda0=1e-4)
    assert ref["rejected"] >= 3
    rho = ref["rho_log"]
    assert np.any(rho == -np.inf) and np.any(np.isfinite(rho) & (rho < 0))          # both kinds of rejection
    assert np.any(ref["accepted_log"].astype(bool) & (rho < 0.8))                     # Nielsen below the clamp
    got = gpu_run(sc, 14, lambda0=1e-4)
    check_control(got, ref)
    assert got["status"] == ORACLE_STATUS[ref["status"]]


def test_deep_point_rejections_mixed():
    """The FP32 assembly takes the same decisions; its final state is held to
    the mixed-precision bars after 40 iterations."""
    sc = deep_point_scene()
    ref = oracle.solve(sc, max_iters=40, lambda0=1e-4)
    got = gpu_run(sc, 40, precision=MIXED, lambda0=1e-4)
    check_control(got, ref, cost_tol=None, lam_rtol=1e-3)
    from test_gpu_parity import final_errors
    rms, dT, att = final_errors(sc, got, ref)
    print(f"deep point mixed: rms {rms:.3e} px, centres {dT:.3e} m, attitude {att:.3e} rad", flush=True)
    assert rms < 1e-3 and dT < 1e-3 and att < 2e-6


@pytest.mark.parametrize("precision", [FP64, MIXED])
@pytest.mark.parametrize("depth_factor,lam0", [(4.0, 0.0215), (1.8, 0.01)])
def test_one_point_control(depth_factor, lam0, precision):
    """Every camera fixed: the reduced system is empty and the step is the
    point blocks' alone."""
    sc = one_point_scene(depth_factor)
    ref = oracle.solve(sc, max_iters=5, lambda0=lam0)
    got = gpu_run(sc, 5, precision=precision, lambda0=lam0)
    check_control(got, ref, cost_tol=1e-8 if precision == FP64 else None, lam_rtol=1e-6 if precision == FP64 else 1e-3)


@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_failed_factorisation_stalls(precision):
    sc = stall_scene()
    ref = oracle.solve(sc, max_iters=20, lambda0=1e-4)
    assert ref["status"] == 2 and ref["iterations"] == 15 and ref["accepted"] == 0
    got = gpu_run(sc, 20, precision=precision, lambda0=1e-4)
    check_control(got, ref, cost_tol=1e-8 if precision == FP64 else 1e-6)
    assert got["status"] == 4
    # lam0 2^(i (i + 1) / 2): exact in binary floating point
    lam = 1e-4 * 2.0 ** (np.arange(15) * (np.arange(15) + 1) / 2)
    assert np.array_equal(got["lambda_log"], lam)
