"""Background layout (ba_options.stage_threads): clusters submitted to a
context whose layout runs on a pool of host threads give bit-identical
results to synchronous submission, through the batched solve, the serving
loop and a resident stream with Eq. (8) fusion; a cluster that the layout
refuses is reported on its ticket; latency is stamped on entry to
ba_submit_cluster."""
import numpy as np
import pytest

from synth import aerial as A

pytestmark = pytest.mark.gpu

MIXED = 1


def scenes(n, seed0):
    return [A.make_scene(A.spec_micro(n_strips=2, imgs_per_strip=2 + i % 3, n_points=300 + 200 * i), seed0 + i)
            for i in range(n)]


def same(a, b):
    assert a["iterations"] == b["iterations"]
    assert np.array_equal(a["cost_log"], b["cost_log"])
    for key in ("R", "T", "X", "k"):
        assert np.array_equal(a[key], b[key]), key


def test_background_layout_batched_and_serving_equal_synchronous():
    from paper_2511_06152_amd import Context
    scs = scenes(8, 300)
    kw = dict(max_iters=10, stop_on_ftol=True, ftol=1e-8)
    with Context(precision=MIXED) as ctx:
        ts = [ctx.submit(sc, **kw) for sc in scs]
        ctx.ba_solve_batch(ts)
        ref = [ctx.ba_fetch(t) for t in ts]
    print("case background layout: batched", flush=True)
    with Context(precision=MIXED, stage_threads=4) as ctx:
        ts = ctx.submit_many(scs, **kw)
        ctx.ba_solve_batch(ts)
        for r, t in zip(ref, ts):
            same(ctx.ba_fetch(t), r)
    print("case background layout: serving loop", flush=True)
    with Context(precision=MIXED, stage_threads=4, serve=True, max_slots=3, iters_per_tick=1) as ctx:
        ts = []
        for sc in scs:
            t = ctx.submit(sc, **kw)
            ctx.ba_solve(t)
            ts.append(t)
        for r, t in zip(ref, ts):
            ctx.ba_wait(t, 60.0)
            g = ctx.ba_fetch(t)
            same(g, r)
            assert g["t_done"] >= g["t_admit"] >= g["t_submit"] > 0


def test_background_layout_resident_stream_equals_synchronous():
    from paper_2511_06152_amd import Context
    cl = A.make_stream(61, n_strips=2, imgs_per_strip=10, pts_per_image=300, max_cams=10, min_cams=6)["clusters"][:6]
    kw = dict(max_iters=6, use_resident=True, fuse_resident=True)
    res = []
    for stage_threads in (0, 3):
        print("case resident stream, stage_threads", stage_threads, flush=True)
        with Context(precision=MIXED, serve=True, max_slots=4, stage_threads=stage_threads) as ctx:
            ts = ctx.submit_many(cl, **kw)
            for t in ts:
                ctx.ba_solve(t)
            out = []
            for t in ts:
                ctx.ba_wait(t, 60.0)
                out.append(ctx.ba_fetch(t))
            ids = np.unique(np.concatenate([c["cam_ids"] for c in cl]))
            out.append(ctx.ba_resident_poses(ids))
        res.append(out)
    for a, b in zip(res[0][:-1], res[1][:-1]):
        same(a, b)
    for x, y in zip(res[0][-1], res[1][-1]):
        assert np.array_equal(x, y)


def test_background_layout_reports_refused_cluster():
    """A camera observing one point twice is found by the layout: with
    background layout the submit succeeds and the ticket reports BA_E_ARG;
    the clusters around it are unaffected."""
    from paper_2511_06152_amd import BAError, Context
    good = scenes(3, 320)
    bad = dict(good[1])
    j = int(bad["obs_pt"][0])
    o2 = [o for o in range(bad["n_obs"]) if bad["obs_pt"][o] == j][1]
    bad["obs_cam"] = bad["obs_cam"].copy()
    bad["obs_cam"][o2] = bad["obs_cam"][0]
    with Context(precision=MIXED, stage_threads=2, serve=True) as ctx:
        ts = [ctx.submit(sc, max_iters=4) for sc in (good[0], bad, good[2])]
        for t in ts:
            try:
                ctx.ba_solve(t)
            except BAError as e:     # refused already: ba_solve reports it too
                assert t == ts[1] and e.code == -1
        with pytest.raises(BAError) as e:
            ctx.ba_wait(ts[1], 60.0)
        assert e.value.code == -1 and "twice" in str(e.value)
        for t in (ts[0], ts[2]):
            ctx.ba_wait(t, 60.0)
            assert ctx.ba_fetch(t)["iterations"] == 4
    with Context(precision=MIXED, stage_threads=2) as ctx:
        t = ctx.submit(bad, max_iters=4)
        with pytest.raises(BAError) as e:
            ctx.ba_solve_batch([t])
        assert e.value.code == -1
        with pytest.raises(BAError):
            ctx.submit(dict(bad, n_cams=0), max_iters=4)    # sizes are still checked at once


def test_stage_threads_option_limits():
    from paper_2511_06152_amd import BAError, Context
    for n in (-1, 65):
        with pytest.raises(BAError) as e:
            Context(stage_threads=n)
        assert e.value.code == -1


def test_clusters_arriving_during_a_tick_equal_alone():
    """A long cluster keeps the serving loop in ticks of ten iterations while
    small clusters arrive one by one: their layouts finish while a tick runs,
    so the loop admits them at once (upload beside the tick) and starts them
    at the next boundary.  Each result equals the one the cluster gets alone,
    bit for bit, and so does the long cluster's."""
    import time
    from paper_2511_06152_amd import Context
    long_sc = A.make_scene(A.spec_micro(n_strips=2, imgs_per_strip=4, n_points=3000), 411)
    small = scenes(5, 420)
    kw_long = dict(max_iters=150, stop_on_ftol=False)
    kw = dict(max_iters=12, stop_on_ftol=False)
    with Context(precision=MIXED) as ctx:
        t = ctx.submit(long_sc, **kw_long)
        ctx.ba_solve_batch([t])
        ref_long = ctx.ba_fetch(t)
        ts = [ctx.submit(sc, **kw) for sc in small]
        ctx.ba_solve_batch(ts)
        ref = [ctx.ba_fetch(t) for t in ts]
    print("case arrivals during a tick", flush=True)
    with Context(precision=MIXED, stage_threads=2, serve=True, max_slots=4, iters_per_tick=10) as ctx:
        tl = ctx.submit(long_sc, **kw_long)
        ctx.ba_solve(tl)
        ts = []
        for sc in small:
            time.sleep(0.002)
            t = ctx.submit(sc, **kw)
            ctx.ba_solve(t)
            ts.append(t)
        for r, t in zip(ref, ts):
            ctx.ba_wait(t, 60.0)
            same(ctx.ba_fetch(t), r)
        ctx.ba_wait(tl, 60.0)
        same(ctx.ba_fetch(tl), ref_long)
