"""GPU parity of the resident state across overlapping clusters (Sec. 3.2:
each arriving image triggers a cluster that shares images and tie points with
the previous ones and starts from their solution).

The oracle side replays the same chain on the host: each cluster starts from
the caller's initial values, overwritten by the last oracle solution of every
camera and point ID an earlier cluster contained; the GPU side keeps that
state on the device, keyed by the same IDs.  Bars: plain FP64 path, cost after
every iteration within 1e-8 relative of the oracle's for every cluster of the
chain; the serving loop (clusters submitted together, ordered by their
shared IDs) bit-identical to the cluster-at-a-time API path.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from synth import aerial as A
from test_gpu_parity import check_cost_log, final_errors

pytestmark = pytest.mark.gpu

FP64, MIXED = 0, 1


def small_stream(seed=61):
    """2 strips x 12 images, ~300 points spawned per image, clusters of 6-12 images."""
    return A.make_stream(seed, n_strips=2, imgs_per_strip=12, pts_per_image=300, max_cams=12, min_cams=6)


def oracle_chain(clusters, iters, lambdas=None):
    cam, pt, refs = {}, {}, []
    for n, sc in enumerate(clusters):
        R, T, X = sc["R"].copy(), sc["T"].copy(), sc["X"].copy()
        for k, cid in enumerate(sc["cam_ids"]):
            if cid in cam:
                R[k], T[k] = cam[cid]
        for j, pid in enumerate(sc["point_ids"]):
            if pid in pt:
                X[j] = pt[pid]
        s2 = dict(sc, R=R, T=T, X=X)
        lam = 1e-4 if lambdas is None else lambdas[n]
        ref = oracle.solve(s2, max_iters=iters, lambda0=lam)
        Rf, Tf, Xf, _ = ref["state"]
        for k, cid in enumerate(sc["cam_ids"]):
            cam[cid] = (Rf[k].copy(), Tf[k].copy())
        for j, pid in enumerate(sc["point_ids"]):
            pt[pid] = Xf[j].copy()
        refs.append(ref)
    return refs


def nobs_per_cam(sc):
    return np.bincount(sc["obs_cam"], minlength=sc["n_cams"]).astype(np.float64)


def oracle_chain_fused(clusters, iters):
    """The chain with Eq. (8) fusion on write-back: a free camera whose ID holds
    an earlier pose stores the match-count weighted mean of that pose and the
    new solution (weights: observations of the camera, accumulated); fixed
    and first-seen cameras store the solution with this cluster's count."""
    cam, pt, refs = {}, {}, []
    for sc in clusters:
        R, T, X = sc["R"].copy(), sc["T"].copy(), sc["X"].copy()
        for k, cid in enumerate(sc["cam_ids"]):
            if cid in cam:
                R[k], T[k] = cam[cid][0], cam[cid][1]
        for j, pid in enumerate(sc["point_ids"]):
            if pid in pt:
                X[j] = pt[pid]
        ref = oracle.solve(dict(sc, R=R, T=T, X=X), max_iters=iters)
        Rf, Tf, Xf, _ = ref["state"]
        n = nobs_per_cam(sc)
        for k, cid in enumerate(sc["cam_ids"]):
            if not sc["fixed"][k] and cid in cam:
                cam[cid] = oracle.fuse_pose(cam[cid][0], cam[cid][1], cam[cid][2], Rf[k], Tf[k], n[k])
            else:
                cam[cid] = (Rf[k].copy(), Tf[k].copy(), float(n[k]))
        for j, pid in enumerate(sc["point_ids"]):
            pt[pid] = Xf[j].copy()
        refs.append(ref)
    return refs, cam


def api_chain(clusters, iters, precision=FP64, lambda0=1e-4, fuse=False, ctx_out=None):
    from paper_2511_06152_amd import Context
    out = []
    ctx = Context(precision=precision)
    try:
        for sc in clusters:
            t = ctx.submit(sc, max_iters=iters, use_resident=True, fuse_resident=fuse, lambda0=lambda0)
            ctx.ba_step(t, iters)
            out.append(ctx.ba_fetch(t))
            ctx.ba_release(t)
        if ctx_out is not None:
            ids = np.unique(np.concatenate([sc["cam_ids"] for sc in clusters]))
            ctx_out["ids"] = ids
            ctx_out["poses"] = ctx.ba_resident_poses(ids)
    finally:
        ctx.close()
    return out


def test_resident_chain_fp64_matches_oracle():
    st = small_stream()
    cl = st["clusters"][:5]
    print("case resident chain", [(c["image"], c["n_cams"], c["n_points"]) for c in cl], flush=True)
    refs = oracle_chain(cl, 6)
    got = api_chain(cl, 6)
    for g, r in zip(got, refs):
        check_cost_log(g, r)


def test_resident_state_is_used():
    """A later cluster that shares IDs starts from the earlier solution: its
    initial cost is the oracle's cost of the caller's values with the shared
    IDs replaced, not of the caller's values."""
    st = small_stream()
    cl = st["clusters"][:2]
    got = api_chain(cl, 6)
    refs = oracle_chain(cl, 6)
    e_caller = oracle.cost(cl[1], (cl[1]["R"], cl[1]["T"], cl[1]["X"], cl[1]["k"]))
    e0 = got[1]["cost_log"][0]
    print("initial cost with resident state", e0, "oracle", refs[1]["cost_log"][0], "caller values", e_caller,
          flush=True)
    assert abs(e0 - refs[1]["cost_log"][0]) <= 1e-10 * refs[1]["cost_log"][0]
    assert e0 < 0.5 * e_caller


def test_resident_lambda_nan_takes_previous_damping():
    st = small_stream()
    cl = st["clusters"][:3]
    got = api_chain(cl, 5, lambda0=float("nan"))
    lams = [1e-4] + [g["lambda_"] for g in got[:-1]]
    refs = oracle_chain(cl, 5, lambdas=lams)
    for g, r in zip(got, refs):
        check_cost_log(g, r)
    assert math.isfinite(got[-1]["lambda_"])


@pytest.mark.parametrize("precision,fuse", [(FP64, False), (MIXED, False), (MIXED, True)])
def test_resident_serving_equals_api(precision, fuse):
    """All clusters of the stream handed to the serving loop at once: shared
    IDs order them; results (and, with fusion, the resident poses) bit-identical
    to solving them one at a time."""
    from paper_2511_06152_amd import Context
    st = small_stream()
    cl = st["clusters"][:6]
    res = {}
    ref = api_chain(cl, 8, precision=precision, fuse=fuse, ctx_out=res)
    with Context(precision=precision, serve=True, max_slots=8) as ctx:
        ts = []
        for sc in cl:
            t = ctx.submit(sc, max_iters=8, use_resident=True, fuse_resident=fuse)
            ctx.ba_solve(t)
            ts.append(t)
        got = []
        for t in ts:
            ctx.ba_wait(t)
            got.append(ctx.ba_fetch(t))
        poses = ctx.ba_resident_poses(res["ids"])
    for a, g in zip(ref, got):
        for key in ("R", "T", "X", "cost_log"):
            assert np.array_equal(a[key], g[key]), key
    for a, g in zip(res["poses"], poses):
        assert np.array_equal(a, g)


def store_errors(res, store):
    """Largest attitude (rad) and centre (m) difference between the resident
    poses read back and the oracle's store; the weights must be equal."""
    R, T, w = res["poses"]
    att, dT = 0.0, 0.0
    for n, cid in enumerate(res["ids"]):
        Ro, To, wo = store[cid]
        att = max(att, float(np.linalg.norm(Rotation.from_matrix(R[n].T @ Ro).as_rotvec())))
        dT = max(dT, float(np.abs(T[n] - To).max()))
        assert w[n] == wo, (cid, w[n], wo)
    print("resident poses vs oracle store: attitude", att, "rad, centre", dT, "m", flush=True)
    return att, dT


def test_fused_chain_fp64_matches_oracle():
    """Eq. (8) fusion on write-back: every cluster of the chain starts from the
    fused poses, so its cost per iteration matches the oracle's fused chain
    (1e-8 relative); the resident poses after the chain match the oracle's
    store (attitude 2e-8 rad, centres 10 um) and the weights exactly."""
    st = small_stream()
    cl = st["clusters"][:6]
    print("case fused chain", [(c["image"], c["n_cams"], c["n_points"]) for c in cl], flush=True)
    refs, store = oracle_chain_fused(cl, 6)
    res = {}
    got = api_chain(cl, 6, fuse=True, ctx_out=res)
    for g, r in zip(got, refs):
        check_cost_log(g, r)
    att, dT = store_errors(res, store)
    assert att < 2e-8 and dT < 1e-5


def small_chain():
    """The paper's chaining (60 images in two strips, clusters of 12, the last
    three reused, one of them fixed) over a lighter tie-point pool."""
    return A.make_chain(9, pts_per_image=300)


def test_paper_chain_fp64_matches_oracle():
    cl = small_chain()["clusters"]
    print("case paper chain", [(c["image"], c["n_cams"], c["n_points"]) for c in cl], flush=True)
    refs, store = oracle_chain_fused(cl, 6)
    res = {}
    got = api_chain(cl, 6, fuse=True, ctx_out=res)
    for g, r in zip(got, refs):
        check_cost_log(g, r)
    att, dT = store_errors(res, store)
    assert att < 2e-8 and dT < 1e-5


def test_paper_chain_mixed_within_bars():
    """The mixed path over the whole chain, 30 iterations per cluster: every
    cluster's solution within the mixed-precision bars of the oracle's fused
    chain (RMS reprojection difference 1e-3 px, centres 1 mm, attitude
    2e-6 rad), and so are the fused resident poses after the chain."""
    cl = small_chain()["clusters"]
    print("case paper chain mixed", len(cl), flush=True)
    refs, store = oracle_chain_fused(cl, 30)
    res = {}
    got = api_chain(cl, 30, precision=MIXED, fuse=True, ctx_out=res)
    for sc, g, r in zip(cl, got, refs):
        rms, dT, att = final_errors(sc, g, r)
        print("cluster", sc["image"], "rms", rms, "px, centre", dT, "m, attitude", att, "rad", flush=True)
        assert rms < 1e-3 and dT < 1e-3 and att < 2e-6
    att, dT = store_errors(res, store)
    assert att < 2e-6 and dT < 1e-3


def test_fusion_arithmetic_matches_oracle():
    """The write-back fusion alone, on identical inputs: the resident poses
    before a cluster, its own solution (ba_fetch) and its observation counts
    give, through the oracle's Eq. (8), the resident poses after it
    (rotation 1e-13, centre 1e-9 m: rounding only)."""
    from paper_2511_06152_amd import Context
    st = small_stream()
    cl = st["clusters"][:4]
    fused = 0
    with Context(precision=FP64) as ctx:
        for sc in cl:
            ids = sc["cam_ids"]
            known = [k for k, cid in enumerate(ids) if int(cid) in ctx_known(ctx, cid)]
            before = ctx.ba_resident_poses(ids[known]) if known else None
            t = ctx.submit(sc, max_iters=5, use_resident=True, fuse_resident=True)
            ctx.ba_step(t, 5)
            out = ctx.ba_fetch(t)
            ctx.ba_release(t)
            R, T, w = ctx.ba_resident_poses(ids)
            n = nobs_per_cam(sc)
            for k in range(sc["n_cams"]):
                if k in known and not sc["fixed"][k]:
                    i = known.index(k)
                    eR, eT, ew = oracle.fuse_pose(before[0][i], before[1][i], before[2][i], out["R"][k], out["T"][k], n[k])
                    fused += 1
                else:
                    eR, eT, ew = out["R"][k], out["T"][k], n[k]
                assert np.abs(R[k] - eR).max() < 1e-13, (sc["image"], k)
                assert np.abs(T[k] - eT).max() < 1e-9, (sc["image"], k)
                assert w[k] == ew
    print("cameras fused", fused, flush=True)
    assert fused > 0


def ctx_known(ctx, cid):
    """{cid} when the context holds a written-back pose for it, else {}."""
    from paper_2511_06152_amd import BAError
    try:
        ctx.ba_resident_poses([cid])
        return {int(cid)}
    except BAError as e:
        assert e.code == -1
        return set()


def test_resident_pose_query_errors():
    from paper_2511_06152_amd import BAError, Context
    st = small_stream()
    a, b = st["clusters"][:2]
    with Context(precision=FP64) as ctx:
        with pytest.raises(BAError) as e:
            ctx.submit(a, max_iters=2, fuse_resident=True)          # fusion needs the resident state
        assert e.value.code == -1
        ta = ctx.submit(a, max_iters=2, use_resident=True, fuse_resident=True)
        with pytest.raises(BAError) as e:
            ctx.ba_resident_poses(a["cam_ids"][:1])                 # writer not finished
        assert e.value.code == -4
        ctx.ba_step(ta, 2)
        R, T, w = ctx.ba_resident_poses(a["cam_ids"])
        assert np.all(w == nobs_per_cam(a))
        with pytest.raises(BAError) as e:
            ctx.ba_resident_poses([10 ** 12])                       # never submitted
        assert e.value.code == -1
        assert ctx.ba_resident_poses([])[0].shape == (0, 3, 3)


def test_resident_dependency_order_enforced():
    from paper_2511_06152_amd import BAError, Context
    st = small_stream()
    a, b = st["clusters"][:2]
    with Context(precision=FP64) as ctx:
        ta = ctx.submit(a, max_iters=2, use_resident=True)
        tb = ctx.submit(b, max_iters=2, use_resident=True)
        with pytest.raises(BAError) as e:
            ctx.ba_step(tb, 2)
        assert e.value.code == -4
        ctx.ba_step(ta, 2)
        ctx.ba_step(tb, 2)
        assert ctx.ba_fetch(tb)["iterations"] == 2


def test_resident_rejects_duplicate_ids():
    from paper_2511_06152_amd import BAError, Context
    st = small_stream()
    sc = dict(st["clusters"][0])
    ids = sc["point_ids"].copy()
    ids[1] = ids[0]
    sc["point_ids"] = ids
    with Context(precision=FP64) as ctx:
        with pytest.raises(BAError) as e:
            ctx.submit(sc, max_iters=2, use_resident=True)
        assert e.value.code == -1


def test_batched_submit_equals_single():
    """ba_submit_clusters (layout on host threads, queued in array order):
    the chained stream through the serving loop gives the same results,
    bit for bit, as submitting the clusters one by one."""
    from paper_2511_06152_amd import Context
    from paper_2511_06152_amd.ba import Cluster
    cl = small_stream()["clusters"][:6]
    res = {}
    ref = api_chain(cl, 8, precision=MIXED, fuse=True, ctx_out=res)
    with Context(precision=MIXED, serve=True, max_slots=8) as ctx:
        ts = ctx.ba_submit_clusters([Cluster(sc, max_iters=8, use_resident=True, fuse_resident=True) for sc in cl])
        assert len(set(ts)) == len(cl) and ts == sorted(ts)
        for t in ts:
            ctx.ba_solve(t)
        got = []
        for t in ts:
            ctx.ba_wait(t)
            got.append(ctx.ba_fetch(t))
        poses = ctx.ba_resident_poses(res["ids"])
    for a, g in zip(ref, got):
        for key in ("R", "T", "X", "cost_log"):
            assert np.array_equal(a[key], g[key]), key
    for a, g in zip(res["poses"], poses):
        assert np.array_equal(a, g)


@pytest.mark.parametrize("stage_threads", [0, 2])
def test_batched_submit_rejects_before_queueing(stage_threads):
    """One invalid cluster fails the whole call before any is queued: the
    valid ones submitted afterwards run with no pending writers in the way.
    With layout threads the duplicate ID is one of the checks made at
    submission, before any cluster is copied or queued."""
    from paper_2511_06152_amd import BAError, Context
    from paper_2511_06152_amd.ba import Cluster
    cl = small_stream()["clusters"][:3]
    bad = dict(cl[1])
    ids = bad["point_ids"].copy()
    ids[1] = ids[0]
    bad["point_ids"] = ids
    with Context(precision=FP64, stage_threads=stage_threads) as ctx:
        with pytest.raises(BAError) as e:
            ctx.ba_submit_clusters([Cluster(sc, max_iters=3, use_resident=True) for sc in (cl[0], bad, cl[2])])
        assert e.value.code == -1 and "cluster 1" in str(e.value)
        ts = ctx.ba_submit_clusters([Cluster(sc, max_iters=3, use_resident=True) for sc in cl])
        for t in ts:
            ctx.ba_step(t, 3)
            assert ctx.ba_fetch(t)["iterations"] == 3
        assert ctx.ba_submit_clusters([]) == []
