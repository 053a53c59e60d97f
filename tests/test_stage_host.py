"""The host layout of a submitted cluster (paper_2511_06152_amd/csrc/
ba_stage.cpp), built alone with the host compiler under AddressSanitizer and
UndefinedBehaviorSanitizer (and, for concurrent layouts, ThreadSanitizer),
run on seeded scenes, and its output checked against the invariants the
kernels rely on (CPU only):

  * points are ordered by observation count, then Morton order; each point
    chunk holds up to 64 consecutive points of one count n, and observation
    t (camera order) of its lane l sits at the chunk's first lane + 64 t + l,
    with its camera and pixel: every observation exactly once, padding lanes
    camera 0 and pixel 0; the point-pass workgroups cover the chunks in
    order;
  * each free camera's lanes hold all its observations, in point order, each
    naming its point and its observation lane (whose camera, point and pixel
    are the observation's), its run padded to whole chunks;
  * the pair lanes hold every pair of observations of one point whose
    cameras are both free, once, in camera-pair blocks, naming both
    observation lanes: their number is sum_j n_j (n_j - 1) / 2 over the free
    observations n_j of each point;
  * tasks tile the camera and pair lanes; targets list every free camera and
    camera pair with their task ranges;
  * the conjugate-gradient layout's block rows list the diagonal block first
    and every co-visible pair both ways;
  * invalid clusters are refused with a message (a camera observing one point
    twice, an index out of range, a non-finite value, a point with more than
    64 observations);
  * several threads laying out the same cluster at once get identical
    layouts, with no data race; a second layout into the same storage on the
    same thread (reused vectors and scratch) is the same.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from synth import aerial as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "paper_2511_06152_amd", "csrc", "ba_stage.cpp"), os.path.join(ROOT, "tests", "stage_check.cpp")]
WAVE = 64
TASK_CAM, TASK_PAIR, TARGET_INTR = 0, 1, 2

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")


def build(tmp, kind):
    exe = os.path.join(tmp, f"stage_check_{kind}")
    if not os.path.exists(exe):
        san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"] if kind == "asan" else ["-fsanitize=thread"]
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *san, "-I", os.path.join(ROOT, "include"),
               *SRC, "-o", exe, "-lpthread"]
        subprocess.run(cmd, check=True)
    return exe


@pytest.fixture(scope="module")
def tools(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("stage"))
    return d, build(d, "asan"), build(d, "tsan")


def write_cluster(path, sc):
    C, P, O = sc["n_cams"], sc["n_points"], sc["n_obs"]
    res = sc.get("cam_ids") is not None
    with open(path, "wb") as fh:
        fh.write(np.array([C, P, O, sc["intr_mask"], 10, 1 if res else 0], np.int32).tobytes())
        for key, dt in (("R", np.float64), ("T", np.float64), ("X", np.float64), ("k", np.float64),
                        ("prior_R", np.float64), ("prior_T", np.float64), ("prior_sigma", np.float64),
                        ("fixed", np.uint8), ("obs_cam", np.int32), ("obs_pt", np.int32), ("obs_uv", np.float64)):
            fh.write(np.ascontiguousarray(sc[key], dt).tobytes())
        fh.write(np.array([sc["f"], sc["cx"], sc["cy"], sc["sigma_px"], sc["huber_delta"]], np.float64).tobytes())
        if res:
            fh.write(np.ascontiguousarray(sc["cam_ids"], np.int64).tobytes())
            fh.write(np.ascontiguousarray(sc["point_ids"], np.int64).tobytes())


def run(tools, sc, cpw=16, cpt=4, solver=0, threads=1, exe=None):
    d, asan, tsan = tools
    src, dst = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
    write_cluster(src, sc)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    p = subprocess.run([exe or asan, src, dst, str(cpw), str(cpt), str(solver), str(threads)], env=env,
                       capture_output=True, text=True)
    assert p.returncode == 0, p.stderr[-3000:]
    with open(dst, "rb") as fh:
        buf = fh.read()
    hdr = np.frombuffer(buf[:48], np.int32)
    pos = 48
    names = ["err", "pt_orig", "pchunk", "wg_chunk", "ob_cam", "ob_uv", "cl_pt", "cl_ob", "ql_pt", "ql_ob", "tasks",
             "targets", "cam_col", "brow", "bcol"]
    types = [np.int8, np.int32, np.int32, np.int32, np.int32, np.float64, np.int32, np.int32, np.int32, np.int32, np.int32,
             np.int32, np.int32, np.int32, np.int32]
    out = dict(zip(["rc", "L", "n_chunks", "Lc", "Lq", "n_tasks", "n_targets", "m", "n_free", "sparse",
                    "n_cam_tasks", "n_wg"], hdr.tolist()))
    for name, dt in zip(names, types):
        if pos >= len(buf):
            break
        n = int(np.frombuffer(buf[pos:pos + 8], np.int64)[0]) * {"tasks": 4, "targets": 4, "pchunk": 4, "ql_ob": 2}.get(name, 1)
        pos += 8
        out[name] = np.frombuffer(buf[pos:pos + n * np.dtype(dt).itemsize], dt).copy()
        pos += n * np.dtype(dt).itemsize
    out["err"] = bytes(out["err"].astype(np.uint8)).decode()
    for key in ("tasks", "targets", "pchunk"):
        if key in out:
            out[key] = out[key].reshape(-1, 4)
    return out


def check_layout(sc, lay):
    C, P, O = sc["n_cams"], sc["n_points"], sc["n_obs"]
    assert lay["rc"] == 0, lay["err"]
    inv = np.empty(P, np.int64)
    inv[lay["pt_orig"]] = np.arange(P)                 # caller point -> internal point
    assert np.array_equal(np.sort(lay["pt_orig"]), np.arange(P))
    # point order: by observation count (never decreasing)
    nobs = np.bincount(inv[sc["obs_pt"]], minlength=P)
    assert np.all(np.diff(nobs) >= 0)
    # point chunks: consecutive points of one count, 64 at most, lanes in order
    L, pc = lay["L"], lay["pchunk"]
    assert lay["n_chunks"] == len(pc)
    first_pt = nobs.tolist().index(next((n for n in nobs if n > 0), 0)) if np.any(nobs > 0) else P
    lane = 0
    pnext = first_pt
    for ch in pc:
        off, n, p0, nv = (int(x) for x in ch)
        assert off == lane and p0 == pnext and 1 <= nv <= WAVE and n >= 1
        assert np.all(nobs[p0:p0 + nv] == n)
        assert nv == WAVE or p0 + nv == P or nobs[p0 + nv] != n     # only a count's last chunk is partial
        lane += WAVE * n
        pnext = p0 + nv
    assert lane == L and pnext == P
    # every observation exactly once, with its camera and pixel, cameras
    # ascending along a point's lanes; padding lanes hold camera 0 and pixel 0
    cam, uv = lay["ob_cam"], lay["ob_uv"].reshape(-1, 2)
    got, pad = [], []
    for off, n, p0, nv in pc:
        for l in range(WAVE):
            idx = off + WAVE * np.arange(n) + l
            if l < nv:
                assert np.all(np.diff(cam[idx]) > 0)
                got += [(p0 + l, int(cam[i]), float(uv[i, 0]), float(uv[i, 1])) for i in idx]
            else:
                pad += idx.tolist()
    want = sorted(zip(inv[sc["obs_pt"]].tolist(), sc["obs_cam"].tolist(), sc["obs_uv"][:, 0].tolist(),
                      sc["obs_uv"][:, 1].tolist()))
    assert sorted(got) == want
    assert np.all(cam[pad] == 0) and np.all(uv[pad] == 0)
    lane_pt = np.full(L, -1, np.int64)                 # point of each observation lane
    for off, n, p0, nv in pc:
        for t in range(n):
            lane_pt[off + WAVE * t: off + WAVE * t + nv] = p0 + np.arange(nv)
    # point-pass workgroups: increasing chunk ranges covering every chunk
    wg = lay["wg_chunk"]
    assert wg[0] == 0 and wg[-1] == len(pc) and np.all(np.diff(wg) >= 1) and len(wg) == lay["n_wg"] + 1
    # camera lanes: each free camera's observations in point order, runs padded to chunks
    free = np.nonzero(sc["fixed"] == 0)[0]
    col = lay["cam_col"]
    assert np.array_equal(np.nonzero(col >= 0)[0], free) and np.array_equal(col[free], 6 * np.arange(free.size))
    # (each lane names its point and its observation lane, whose camera,
    # point and pixel are the observation's)
    cl_pt, cl_ob = lay["cl_pt"], lay["cl_ob"]
    base = 0
    for k in free:
        o = np.nonzero(sc["obs_cam"] == k)[0]
        order = np.argsort(inv[sc["obs_pt"][o]], kind="stable")
        sl = slice(base * WAVE, base * WAVE + o.size)
        assert np.array_equal(cl_pt[sl], inv[sc["obs_pt"][o]][order])
        ob = cl_ob[sl]
        assert np.all(cam[ob] == k) and np.array_equal(lane_pt[ob], cl_pt[sl])
        assert np.array_equal(uv[ob], sc["obs_uv"][o][order])
        n_ch = -(-o.size // WAVE)
        pad_sl = slice(base * WAVE + o.size, (base + n_ch) * WAVE)
        assert np.all(cl_pt[pad_sl] == -1) and np.all(cl_ob[pad_sl] == 0)
        base += n_ch
    assert base * WAVE == lay["Lc"]
    # pair lanes: every pair of free observations of a point, once
    isfree = sc["fixed"][sc["obs_cam"]] == 0
    nfree = np.bincount(inv[sc["obs_pt"][isfree]], minlength=P)
    n_pairs = int((nfree * (nfree - 1) // 2).sum())
    ql, ql_ob = lay["ql_pt"], lay["ql_ob"].reshape(-1, 2)
    assert (ql >= 0).sum() == n_pairs and lay["Lq"] % WAVE == 0
    uv_of = {(int(inv[p]), int(c)): (float(u), float(v)) for p, c, (u, v) in
             zip(sc["obs_pt"], sc["obs_cam"], sc["obs_uv"])}
    # tasks: camera tasks tile the camera lanes, pair tasks the pair lanes, in order
    tasks = lay["tasks"]
    kind = tasks[:, 0] >> 24
    ct, pt_ = tasks[kind == TASK_CAM], tasks[kind == TASK_PAIR]
    assert lay["n_cam_tasks"] == len(ct) and np.all(kind[:len(ct)] == TASK_CAM)
    for tt, total in ((ct, lay["Lc"]), (pt_, lay["Lq"])):
        if len(tt):
            assert tt[0, 1] == 0 and np.all(tt[1:, 1] == tt[:-1, 1] + tt[:-1, 2]) and tt[-1, 1] + tt[-1, 2] == total // WAVE
    # pair lanes of each block belong to points both cameras of the block observe
    seen = set()
    for t in pt_:
        a, b = int((t[0] >> 12) & 0xFFF), int(t[0] & 0xFFF)
        assert a < b and col[a] >= 0 and col[b] >= 0
        for lane in range(t[1] * WAVE, (t[1] + t[2]) * WAVE):
            j = int(ql[lane])
            if j >= 0:
                assert (j, a, b) not in seen
                seen.add((j, a, b))
                la, lb = ql_ob[lane]
                assert cam[la] == a and cam[lb] == b and lane_pt[la] == j and lane_pt[lb] == j
                assert tuple(uv[la]) + tuple(uv[lb]) == uv_of[(j, a)] + uv_of[(j, b)]
            else:
                assert tuple(ql_ob[lane]) == (0, 0)
    assert len(seen) == n_pairs
    # targets: every free camera, then (dense) every camera pair, with contiguous task ranges
    tg = lay["targets"]
    assert np.array_equal((tg[:free.size, 0] >> 12) & 0xFFF, free)
    if not lay["sparse"]:
        n_pairs_tg = free.size * (free.size - 1) // 2
        assert len(tg) == free.size + n_pairs_tg + (1 if lay["m"] > 6 * free.size else 0)
    return lay


SCENES = {
    "tiny": lambda: A.scene_tiny(1),
    "fixed_and_intrinsics": lambda: A.make_scene(A.spec_micro(n_strips=2, imgs_per_strip=3, n_points=700, n_fixed=2,
                                                              intr_mask=3, k_true=(-0.05, 0.02)), 11),
    "uneven": lambda: A.make_scene(A.SceneSpec(n_strips=3, imgs_per_strip=8, n_points=3000,
                                               obs_model=("tgeom", 0.5, 2, 6), outlier_frac=0.05), 12),
    "resident": lambda: A.make_stream(61, n_strips=2, imgs_per_strip=10, pts_per_image=300, max_cams=10,
                                      min_cams=6)["clusters"][3],
}


@pytest.mark.parametrize("name", list(SCENES))
def test_layout_invariants_under_sanitizers(tools, name):
    sc = SCENES[name]()
    check_layout(sc, run(tools, sc))
    check_layout(sc, run(tools, sc, cpw=3, cpt=1))       # other chunk and task sizes


def test_points_with_64_observations_share_a_chunk(tools):
    rng = np.random.default_rng(5)
    C, P = 64, 40
    sc = A.make_scene(A.spec_micro(n_points=5), 3)
    T = np.array([[10.0 * (c % 8), 10.0 * (c // 8), 300.0] for c in range(C)])
    R = np.stack([A.R_NADIR] * C)
    X = np.column_stack([rng.uniform(20, 50, P), rng.uniform(20, 50, P), rng.uniform(0, 20, P)])
    oc, op = [], []
    for j in range(P):
        cams = np.arange(C) if j % 5 == 0 else rng.choice(C, int(rng.integers(2, 9)), replace=False)
        oc += list(cams)
        op += [j] * len(cams)
    oc, op = np.array(oc, np.int32), np.array(op, np.int32)
    fixed = np.zeros(C, np.uint8)
    fixed[24:] = 1
    sc = dict(sc, n_cams=C, n_points=P, n_obs=len(oc), R=R, T=T, X=X, prior_R=R, prior_T=T,
              prior_sigma=np.ones((C, 6)), fixed=fixed, obs_cam=oc, obs_pt=op,
              obs_uv=A.project_obs(R, T, X, (0.0, 0.0), oc, op), intr_mask=0)
    lay = check_layout(sc, run(tools, sc))
    full = [ch for ch in lay["pchunk"] if ch[1] == 64]
    assert len(full) == 1 and full[0][3] == P // 5


def test_conjugate_gradient_block_structure(tools):
    sc = A.scene_global(7, n_strips=3, imgs_per_strip=10, n_points=15000)
    lay = check_layout(sc, run(tools, sc, solver=2))
    brow, bcol = lay["brow"], lay["bcol"]
    F = lay["n_free"]
    assert lay["sparse"] == 1 and len(brow) == F + 1
    pairs = set()
    for f in range(F):
        row = bcol[brow[f]:brow[f + 1]]
        assert row[0] == f and np.all(np.diff(row[1:]) > 0)
        pairs |= {(f, int(g)) for g in row[1:]}
    assert all((g, f) in pairs for f, g in pairs)


def test_invalid_clusters_are_refused(tools):
    base = A.make_scene(A.spec_micro(n_points=60), 13)
    cases = []
    s = dict(base, obs_cam=base["obs_cam"].copy())
    j = int(base["obs_pt"][0])
    o2 = [o for o in range(base["n_obs"]) if base["obs_pt"][o] == j][1]
    s["obs_cam"][o2] = base["obs_cam"][0]
    cases.append((s, "twice"))
    s = dict(base, obs_pt=base["obs_pt"].copy())
    s["obs_pt"][3] = base["n_points"]
    cases.append((s, "out of range"))
    s = dict(base, obs_uv=base["obs_uv"].copy())
    s["obs_uv"][5, 0] = np.inf
    cases.append((s, "non-finite"))
    s = dict(base, X=base["X"].copy())
    s["X"][1, 2] = np.nan
    cases.append((s, "non-finite"))
    for s, msg in cases:
        lay = run(tools, s)
        assert lay["rc"] == -1 and msg in lay["err"], lay["err"]


def test_concurrent_layouts_identical_and_race_free(tools):
    """ThreadSanitizer: eight threads lay out the same cluster at once (the
    way ba_submit_clusters and the background layout threads do)."""
    d, asan, tsan = tools
    for name in ("tiny", "uneven"):
        sc = SCENES[name]()
        check_layout(sc, run(tools, sc, threads=8, exe=tsan))


def test_paper_scale_layout(tools):
    """A paper-scale cluster (74k observations, 170k pair lanes); stage_check
    also lays it out a second time into the same storage on the same thread
    and requires the same layout."""
    sc = A.scene_cluster12(2)
    check_layout(sc, run(tools, sc))
