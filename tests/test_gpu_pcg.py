"""GPU parity of the conjugate-gradient solve of the reduced camera system
(whole-flight global adjustment, Eq. 6 over every image of the block) against
the FP64 oracle, which solves the same reduced system by dense Cholesky.

Bars:
  * FP64 path with a tight PCG tolerance (1e-12 relative residual): cost after
    every LM iteration within 1e-8 relative of the oracle's, same accepted
    steps;
  * mixed path (FP32 products) with a tight PCG tolerance (1e-6), so that it
    follows the exact LM's trajectory: after 60 iterations RMS
    |p_gpu - p_oracle| < 1e-3 px, camera centres < 1 mm, attitude < 2e-6 rad;
  * default inexact steps (forcing term min(0.1, sqrt(|b|/|b_0|))): these take a
    different path down the same cost, so they are held to the oracle's cost
    and RMS reprojection error at equal iteration count, not to its state;
  * a cluster solved by PCG gives bit-identical results alone and batched with
    dense-solver clusters.
"""
import numpy as np
import pytest

import oracle
from synth import aerial as A
from test_gpu_parity import check_cost_log, final_errors

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1
PCG, DENSE = 2, 1


def run(sc, iters, precision=FP64, solver=PCG, **kw):
    from paper_2511_06152_amd import Context
    with Context(precision=precision, solver=solver, **kw) as ctx:
        t = ctx.submit(sc, max_iters=iters)
        ctx.ba_step(t, iters)
        return ctx.ba_fetch(t)


def medium(seed=7):
    """40 cameras (4 strips x 10), 40k points: m = 240."""
    return A.scene_global(seed, n_strips=4, imgs_per_strip=10, n_points=40000)


def test_pcg_fp64_cost_per_iteration_small():
    """PCG forced on a 6-camera pinhole scene (the dense solver's domain)."""
    sc = A.make_scene(A.spec_micro(n_strips=2, imgs_per_strip=3, n_points=1500, obs_model=("all",)), 51)
    print("case pcg small seed 51", sc["n_cams"], sc["n_points"], sc["n_obs"], flush=True)
    ref = oracle.solve(sc, max_iters=8)
    got = run(sc, 8, pcg_tol=1e-12, pcg_max_iters=2000)
    check_cost_log(got, ref)


def test_pcg_fp64_cost_per_iteration_40_cams():
    sc = medium(7)
    print("case pcg medium seed 7", sc["n_cams"], sc["n_points"], sc["n_obs"], flush=True)
    ref = oracle.solve(sc, max_iters=8)
    got = run(sc, 8, pcg_tol=1e-12, pcg_max_iters=4000)
    check_cost_log(got, ref)


def test_pcg_fp64_with_fixed_cameras_and_prior_only_camera():
    """Two fixed cameras; one free camera with no observations (its block row
    is its prior alone)."""
    sc = A.make_scene(A.SceneSpec(n_strips=3, imgs_per_strip=5, n_points=4000, obs_model=("tgeom", 0.5, 2, 6),
                                  n_fixed=2, outlier_frac=0.05), 52)
    keep = sc["obs_cam"] != 14
    sc.update(obs_cam=np.ascontiguousarray(sc["obs_cam"][keep]), obs_pt=np.ascontiguousarray(sc["obs_pt"][keep]),
              obs_uv=np.ascontiguousarray(sc["obs_uv"][keep]), n_obs=int(keep.sum()))
    print("case pcg fixed + lone camera seed 52", sc["n_cams"], sc["n_points"], sc["n_obs"], flush=True)
    ref = oracle.solve(sc, max_iters=6)
    got = run(sc, 6, pcg_tol=1e-12, pcg_max_iters=4000)
    check_cost_log(got, ref)


def test_pcg_mixed_tight_tolerance_40_cams():
    sc = medium(8)
    print("case pcg mixed medium seed 8", sc["n_cams"], sc["n_points"], sc["n_obs"], flush=True)
    ref = oracle.solve(sc, max_iters=60)
    got = run(sc, 60, precision=MIXED, pcg_tol=1e-6)
    rms, dT, att = final_errors(sc, got, ref)
    print("rms px", rms, "centre m", dT, "attitude rad", att, flush=True)
    assert rms < 1e-3
    assert dT < 1e-3
    assert att < 2e-6


def rms_reprojection(sc, R, T, X, k):
    e = A.project_obs(R, T, X, k, sc["obs_cam"], sc["obs_pt"]) - sc["obs_uv"]
    return float(np.sqrt((e ** 2).sum(1).mean()))


@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_pcg_default_forcing_reaches_oracle_cost_40_cams(precision):
    """Inexact steps (default forcing term): after 40 iterations the cost is at
    most the exact LM's (relative slack 1e-7) and the RMS reprojection error
    over all observations equals the oracle's within 1e-3 px."""
    sc = medium(8)
    print("case pcg default forcing seed 8 precision", precision, flush=True)
    ref = oracle.solve(sc, max_iters=40)
    got = run(sc, 40, precision=precision)
    e_gpu = oracle.cost(sc, got["state"])
    e_ref = ref["cost_log"][-1]
    r_gpu, r_ref = rms_reprojection(sc, *got["state"]), rms_reprojection(sc, *ref["state"])
    print("cost gpu", e_gpu, "oracle", e_ref, "rms px", r_gpu, r_ref, "cg iters", got["cg_iters"], flush=True)
    assert e_gpu <= e_ref * (1 + 1e-7)
    assert abs(r_gpu - r_ref) < 1e-3


def test_auto_solver_uses_pcg_above_24_free_cameras():
    """AUTO picks the conjugate-gradient solve for 40 free cameras; the dense
    solver refuses them."""
    from paper_2511_06152_amd import BAError, Context
    sc = medium(9)
    with Context(precision=FP64, solver=DENSE) as ctx:
        with pytest.raises(BAError) as e:
            ctx.submit(sc, max_iters=2)
        assert e.value.code == -1
    ref = oracle.solve(sc, max_iters=3)
    got = run(sc, 3, solver=0, pcg_tol=1e-12, pcg_max_iters=4000)
    check_cost_log(got, ref)


def test_pcg_rejects_intrinsics():
    from paper_2511_06152_amd import BAError, Context
    sc = A.scene_cluster12(2)
    with Context(precision=FP64, solver=PCG) as ctx:
        with pytest.raises(BAError) as e:
            ctx.submit(sc, max_iters=2)
        assert e.value.code == -1


@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_pcg_cluster_same_alone_and_batched_with_dense(precision):
    """A 40-camera PCG cluster batched with two dense-solver clusters (one of
    them with intrinsics) returns bit-identical results to each run alone."""
    from paper_2511_06152_amd import Context
    scs = [medium(10), A.scene_cluster12(2), A.scene_batched(5)]
    alone = [run(sc, 5, precision=precision, solver=0) for sc in scs]
    with Context(precision=precision, solver=0) as ctx:
        ts = [ctx.submit(sc, max_iters=5) for sc in scs]
        ctx.ba_solve_batch(ts)
        got = [ctx.ba_fetch(t) for t in ts]
    for a, g in zip(alone, got):
        for key in ("R", "T", "X", "k", "cost_log"):
            assert np.array_equal(a[key], g[key]), key


def test_global_400_cams_full_size():
    """The whole-flight workload at full size (400 cameras, 800k points,
    3.5M observations) in the configuration bench.py times (mixed, default
    forcing term): the oracle's FP64 cost of the returned state equals the
    cost the GPU reports for it (1e-11), the first iteration's cost matches
    the oracle's evaluation of the initial state, and the cost decreases."""
    from paper_2511_06152_amd import Context
    from paper_2511_06152_amd.ba import Cluster
    sc = A.scene_global(5)
    print("case global full size", sc["n_cams"], sc["n_points"], sc["n_obs"], flush=True)
    cl = Cluster(sc, max_iters=3)
    with Context(precision=MIXED, max_slots=2, hbm_budget_bytes=2 << 30, chunks_per_task=8) as ctx:
        t = ctx.ba_submit_cluster(cl)
        ctx.ba_step(t, 3)
        got = ctx.ba_fetch(t)
    e0 = oracle.cost(sc, (sc["R"], sc["T"], sc["X"], sc["k"]))
    e3 = oracle.cost(sc, got["state"])
    log = got["cost_log"]
    print("cost log", log, "oracle initial", e0, "oracle final", e3, "cg", got["cg_iters"], flush=True)
    assert abs(log[0] - e0) <= 1e-11 * e0
    assert abs(log[-1] - e3) <= 1e-11 * e3
    assert np.all(np.diff(log) < 0)
    assert got["accepted"] == 3
