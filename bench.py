#!/usr/bin/env python3
"""Local bundle-adjustment benchmark on one MI355X.

Workload: the paper-scale local cluster -- 12 images (2 adjacent strips x 6),
50 MP 8000x6000 px camera at 300 m, 80 % forward / 60 % side overlap, one tie
point per 150x150 px cell (~20k points, ~85k observations), k1/k2 radial
distortion estimated, Huber delta 1 px, GNSS/IMU pose priors; synthetic and
seeded (synth/aerial.py).

One step = every LM iteration of a batch of B resident clusters solved to the
termination rule (ftol on the relative cost decrease, or max_iters) with the
mixed path: FP32 residuals/Jacobians/Schur assembly, FP64 Cholesky, FP64 cost
and gain ratio, LM control on the device, every cluster of the batch in the
same launches.  Inputs are resident in HBM when a step's timer starts
(admission is done before).  `value` = clusters solved per second.

Reported beside it: the plain FP64 GPU LM (one cluster at a time, host-driven,
status read back every iteration) on the same clusters and rule, p50/p99
solve latency of both, p50/p99 of the continuous-batching serving loop, final
RMS reprojection of both paths, the dominant kernel's roofline position
measured with HIP events on the library's stream, and the FP64 oracle timed on
the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from synth import aerial as A  # noqa: E402

PEAK_FP32_TFLOPS = 157.3     # MI355X published FP32 vector peak (packed FP32: two FMAs per lane per clock)
PEAK_VALU_TFLOPS = 78.6      # non-packed FP32 / FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz; the
                             # ceiling of code built without packed FP32 instructions, as this library is
PEAK_MFMA_F64_TFLOPS = 78.6  # dense FP64 matrix cores (MI355X)
# Algorithmic work of the two Schur block kernels (flops; an FMA counts 2), in
# the 2x2 / 2-vector formulation they use.  k_camblk, per observation of a free
# camera: T = J_p Q (36), M = w I - w^2 T J_p^T (25), w e and w T g_p (16),
# M J_c (36), the 21 entries of J_c^T M J_c (84), J_c^T of the three 2-vectors
# for g, Y g_p and diag U (84): 281; the intrinsic border when k1/k2 are
# estimated, 40 per intrinsic.  k_pairblk, per observation pair of one point
# with both cameras free: T_a = J_pa Q (36), M = -w_a w_b T_a J_pb^T (30),
# M J_cb (36), J_ca^T (M J_cb) (144): 246.
FLOP_CAM_OBS = 281
FLOP_CAM_INTR_OBS = 80
FLOP_PAIR = 246


# HBM traffic per launch of the two block kernels on 64 paper-scale clusters,
# from two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE; KiB per
# dispatch) over `bench.py --steps 1 --warmup 0 --batch 64 --plain 0 --serve 0
# --uneven 0 --stream-reps 0 --chain-reps 0 --geo-reps 0 --global-iters 0 --cpu-clusters 0` (the batch
# runs as S parts on S streams, so a launch covers 1/S of the batch; key
# (S, kernel)) and the same with `--batch-streams 1` (one launch covers the
# batch: the kernel alone on the GPU), each scaled by what the same counter reads for a
# plain copy of known size (`bench.py --copy-calibration 256`: FETCH_SIZE
# reads 131084.9 KiB for 262144 KiB read, WRITE_SIZE 262144.0 KiB for 262144
# KiB written).  Valid only for the kernel sources they were taken on (sha256
# of csrc/ba_kernels.hip and csrc/ba_device.h); otherwise reported as null.
TRAFFIC = {
    "fetch_scale": 262144.0 / 131084.9, "write_scale": 262144.0 / 262144.0,
    "clusters": 64,
    "chunks": (32, 10),   # (chunks_per_wg, chunks_per_task) of the measured launches
    "kib": {  # (streams, kernel): (FETCH_SIZE, WRITE_SIZE)
        (2, "blocks"): (96011.7, 1961.7),
        (1, "blocks"): (177742.1, 3923.3),
    },
    "sources_sha256": {
        "ba_kernels.hip": "be030a02ca766ad622db062abcc26acff0d8bee6f3d954287e0b87add4f0dea6",
        "ba_device.h": "45093471b96384b378a47b719b8dd54046152bcd82b097b1d9331eb892ddbd1f",
    },
}


def traffic_bytes(kernel: str, batch: int, streams: int, chunks=None):
    """Measured HBM bytes per launch of `kernel`, or None when the counters
    were taken on other kernel sources, another batch size, other chunk
    sizes (chunks = (chunks_per_wg, chunks_per_task)) or not at all."""
    import hashlib
    key = (streams, kernel)
    if key not in TRAFFIC["kib"] or batch != TRAFFIC["clusters"]:
        return None
    if chunks is not None and tuple(chunks) != tuple(TRAFFIC["chunks"]):
        return None
    csrc = os.path.join(ROOT, "paper_2511_06152_amd", "csrc")
    for name, sha in TRAFFIC["sources_sha256"].items():
        with open(os.path.join(csrc, name), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != sha:
                return None
    f, w = TRAFFIC["kib"][key]
    return 1024.0 * (f * TRAFFIC["fetch_scale"] + w * TRAFFIC["write_scale"])


# kernels timed inside the timed region (bits of ba_profile_enable): the
# Schur-block launch (camera and pair tasks), the dominant kernel; timing all
# of them costs ~7 % of the step, so the full breakdown is taken on one more,
# untimed step
BLOCK_KERNELS = 1 << 1


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def block_flops(sc):
    """Algorithmic flops of one pass of the camera tasks and of the pair tasks
    over the cluster, and their sum (the Schur-block launch k_blocks)."""
    free = sc["fixed"][sc["obs_cam"]] == 0
    cnt = np.bincount(sc["obs_pt"][free], minlength=sc["n_points"])
    pairs = int((cnt * (cnt - 1) // 2).sum())
    n_free_obs = int(free.sum())
    cam = (FLOP_CAM_OBS + (FLOP_CAM_INTR_OBS if sc["intr_mask"] else 0)) * n_free_obs
    pair = FLOP_PAIR * pairs
    return {"camblk": cam, "pairblk": pair, "blocks": cam + pair}


def solve_mfma_flops(sc):
    """FP64 matrix-core flops of one dense solve of the cluster's reduced
    system: m = 6 free cameras + estimated intrinsics, nb = ceil(m/16) blocks
    per side.  The factorisation's block column K does nb-K-1 panel products
    and (nb-K-1)(nb-K)/2 trailing products; the block inverse W = L^-1 then
    takes, for each block (I, J) below the diagonal, I-J products for its sum
    and one by the inverted diagonal block.  Each is a 16x16x16 product (8192
    flops)."""
    m = 6 * int((sc["fixed"] == 0).sum()) + bin(int(sc["intr_mask"]) & 31).count("1")
    nb = -(-m // 16)
    prods = sum((nb - K - 1) + (nb - K - 1) * (nb - K) // 2 for K in range(nb))
    prods += sum((nb - d) * (d + 1) for d in range(1, nb))
    return 8192.0 * prods


def rms_px(sc, R, T, X, k):
    """RMS reprojection error (px) over all observations, from the scene's
    forward camera model."""
    e = A.project_obs(R, T, X, k, sc["obs_cam"], sc["obs_pt"]) - sc["obs_uv"]
    return float(np.sqrt((e ** 2).sum(1).mean()))


def pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else float("nan")


def measure_isolated(args, Context, ctx_kw, scenes, kw, flops):
    """One step of the same batch on a single stream with the two block
    kernels timed: their roofline when nothing else shares the GPU."""
    B = args.batch
    ctx = Context(batch_streams=1, **ctx_kw)
    ids = [i % len(scenes) for i in range(B)]
    tickets = [ctx.submit(scenes[j], **kw) for j in ids]
    for t in tickets:
        ctx.ba_step(t, 0)
    ctx.ba_profile_enable(BLOCK_KERNELS)
    ctx.ba_solve_batch(tickets)
    ctx.ba_profile_enable(False)
    prof = ctx.ba_profile_read()
    fl = 0.0
    for t, j in zip(tickets, ids):
        fl += ctx.ba_fetch(t)["iterations"] * flops[j]["blocks"]
        ctx.ba_release(t)
    ctx.close()
    dom = "blocks"
    ms, n = prof[dom]
    avg = ms / max(n, 1)
    ach = fl / max(n, 1) / (avg / 1e3) / 1e12 if n else float("nan")
    return {"bound": "alu", "kernel": f"k_{dom}<float>", "achieved": ach, "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS, "peak_nonpacked": PEAK_VALU_TFLOPS,
            "frac_of_nonpacked": ach / PEAK_VALU_TFLOPS,
            "traffic": traffic_bytes(dom, B, 1, (args.chunks_per_wg, args.chunks_per_task)),
            "traffic_unit": "bytes per launch", "avg_launch_us": avg * 1e3, "algorithmic_flop_per_launch": fl / max(n, 1),
            "batch_streams": 1,
            "note": "one more step of the same batch on one stream: each launch covers the batch, alone on the GPU"}


def copy_calibration(mib: int):
    """A plain elementwise copy of known size on cuda:0: each launch reads and
    writes mib MiB."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.rand(n, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                      "launches": 5}), flush=True)


def run_uneven(args, Context, precision, kw):
    """The batched-uneven workload: N resident clusters of 6-24 cameras with
    log-uniform 5k-60k points and 2-6 observations per point, solved as one
    batch per step (inputs resident before the timer)."""
    t_gen = time.perf_counter()
    scs = [A.scene_batched(i) for i in range(args.uneven_scenes)]
    log(f"uneven: generated {len(scs)} clusters in {time.perf_counter() - t_gen:.1f}s")
    from paper_2511_06152_amd.ba import Cluster
    N = args.uneven
    probe = Context(precision=precision, max_slots=4, hbm_budget_bytes=64 << 20)
    foot = [probe.ba_footprint(Cluster(sc, **kw)) for sc in scs]
    probe.close()
    budget = int(sum(foot[i % len(scs)] for i in range(N)) * 1.02) + (64 << 20)
    ctx = Context(precision=precision, max_slots=N, hbm_budget_bytes=budget, chunks_per_task=args.chunks_per_task,
                  chunks_per_wg=args.chunks_per_wg, batch_streams=args.batch_streams, iters_per_tick=args.iters_per_tick)
    times, iters, its_max = [], 0, 0
    # the two smallest distinct clusters: their results are compared with the oracle's
    sample = sorted(range(min(N, len(scs))), key=lambda i: scs[i]["n_obs"])[:2]
    sample_res = {}
    statuses = set()
    for step in range(1 + max(args.steps // 2, 1)):
        tickets = ctx.submit_many([scs[i % len(scs)] for i in range(N)], **kw)
        for t in tickets:
            ctx.ba_step(t, 0)
        t0 = time.perf_counter()
        ctx.ba_solve_batch(tickets)
        dt = time.perf_counter() - t0
        res = [ctx.ba_fetch(t) for t in tickets]
        its = [r["iterations"] for r in res]
        statuses |= {r["status"] for r in res}
        if step == 0:
            sample_res = {i: res[i] for i in sample}
        for t in tickets:
            ctx.ba_release(t)
        if step:
            times.append(dt)
            iters += sum(its)
            its_max = max(its_max, max(its))
        log(f"uneven step {step}{'' if step else ' (warmup)'}: {dt * 1e3:.1f} ms for {N} clusters")
    ctx.close()
    cams = [scs[i % len(scs)]["n_cams"] for i in range(N)]
    pts = [scs[i % len(scs)]["n_points"] for i in range(N)]
    obs = [scs[i % len(scs)]["n_obs"] for i in range(N)]
    rep = {"clusters": N, "distinct": len(scs), "clusters_per_s": N / float(np.mean(times)),
           "ms_per_batch": 1e3 * float(np.mean(times)), "mean_iterations": iters / (N * len(times)),
           "max_iterations": its_max, "cams_range": [min(cams), max(cams)],
           "points_range": [min(pts), max(pts)], "obs_total": int(sum(obs)), "hbm_budget_bytes": budget,
           "statuses": sorted(int(x) for x in statuses)}
    rep["_sample"] = [(scs[i], sample_res[i]) for i in sample]
    if not args.uneven_serve:
        return rep
    # the same clusters through the serving loop under a quarter of their total
    # footprint: admission by HBM budget, continuous batching
    total = sum(foot[i % len(scs)] for i in range(N))
    sctx = Context(precision=precision, serve=True, max_slots=N, hbm_budget_bytes=int(0.25 * total),
                   chunks_per_task=args.chunks_per_task, stage_threads=args.stage_threads)
    t0 = time.perf_counter()
    # they arrive together: one batched submit lays them out on host threads
    tickets = sctx.submit_many([scs[i % len(scs)] for i in range(N)], **kw)
    for t in tickets:
        sctx.ba_solve(t)
    lat = []
    for t in tickets:
        sctx.ba_wait(t)
        r = sctx.ba_fetch(t)
        lat.append((r["t_done"] - r["t_submit"]) * 1e3)
        sctx.ba_release(t)
    wall = time.perf_counter() - t0
    sctx.close()
    log(f"uneven, quarter budget through the serving loop: {wall * 1e3:.1f} ms for {N} clusters")
    rep["serving_quarter_budget"] = {"hbm_budget_bytes": int(0.25 * total), "total_footprint_bytes": int(total),
                                     "clusters_per_s": N / wall, "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99)}
    return rep


def run_stream(args, Context, precision, kw):
    """The serving stream: 4 strips x 40 images flown in order, each arriving
    image triggering a sliding cluster of 8-20 images over one global
    tie-point pool.  Clusters go to the continuous-batching loop with resident
    state keyed by image and point IDs (each starts from the state the clusters
    before it left, in submission order; free images already solved by an
    earlier cluster are written back by the match-count weighted pose fusion
    of Eq. (8)), closed loop with a fixed number in flight.  Latency =
    submit -> result available."""
    from collections import deque
    from paper_2511_06152_amd import Geo
    from paper_2511_06152_amd.ba import Cluster
    from synth import geo as SG
    t_gen = time.perf_counter()
    sf = A.stream_flight(3)
    fl = sf["flight"]
    # cluster formation (Sec. 3.1-3.2) on the GPU: footprints of the GNSS/IMU
    # poses on the flight's DSM, then the images each arriving image's
    # footprint overlaps, within and across strips
    cam = {"f": fl["f"], "cx": fl["cx"], "cy": fl["cy"], "width": A.IMG_W, "height": A.IMG_H}
    rule = dict(max_back=7, free_back=3, max_cams=20, min_cams=8, min_overlap=0.05)
    with Geo(SG.flight_dsm(fl)) as geo:
        fp, _ = geo.ba_footprints(fl["R"], fl["T"], cam)
        fp_ms = geo.ba_geo_last_ms()
        members = geo.ba_cluster_membership(fp, fl["truth"]["strip"], **rule)
        mem_ms = geo.ba_geo_last_ms()
    cl = A.cut_clusters(sf, members)
    formation = {"images": int(fl["n_cams"]), "clusters_formed": len(cl), "rule": rule,
                 "footprints_ms": fp_ms, "membership_ms": mem_ms,
                 "note": "each cluster's images from ba_footprints + ba_cluster_membership on the flight's "
                         "GNSS/IMU poses and DSM"}
    log(f"stream: {len(cl)} clusters formed from {fl['n_cams']} images' footprints "
        f"({fp_ms * 1e3:.0f} + {mem_ms * 1e3:.0f} us), {fl['n_points']} pool points in "
        f"{time.perf_counter() - t_gen:.1f}s")
    probe = Context(precision=precision, max_slots=2, hbm_budget_bytes=64 << 20)
    foot = max(probe.ba_footprint(Cluster(sc, **kw)) for sc in cl)
    probe.close()
    W = max(args.stream_window, 1)
    lat, walls = [], []
    first = []          # results of the first clusters of repetition 0, in submission order
    for rep in range(args.stream_reps):
        ctx = Context(precision=precision, serve=True, max_slots=W + 2, hbm_budget_bytes=(W + 2) * foot + (64 << 20),
                      stage_threads=args.stage_threads)
        pending = deque()
        t0 = time.perf_counter()

        def retire():
            t = pending.popleft()
            ctx.ba_wait(t)
            r = ctx.ba_fetch(t)
            lat.append((r["t_done"] - r["t_submit"]) * 1e3)
            if rep == 0 and len(first) < args.stream_oracle_clusters:
                first.append(r)
            ctx.ba_release(t)

        for sc in cl:
            while len(pending) >= W:
                retire()
            t = ctx.submit(sc, use_resident=True, fuse_resident=True, **kw)
            ctx.ba_solve(t)
            pending.append(t)
        while pending:
            retire()
        walls.append(time.perf_counter() - t0)
        ctx.close()
        log(f"stream rep {rep}: {len(cl)} clusters in {walls[-1] * 1e3:.0f} ms")
    return {"clusters_per_rep": len(cl), "reps": args.stream_reps, "window": W, "formation": formation,
            "cams_range": [min(c["n_cams"] for c in cl), max(c["n_cams"] for c in cl)],
            "points_range": [min(c["n_points"] for c in cl), max(c["n_points"] for c in cl)],
            "obs_range": [min(c["n_obs"] for c in cl), max(c["n_obs"] for c in cl)],
            "clusters_per_s": len(cl) * len(walls) / sum(walls), "latencies": len(lat),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "budget_ms": 2080.0,
            "p99_fraction_of_budget": pct(lat, 99) / 2080.0,
            "_sample": list(zip(cl[:len(first)], first))}


def run_chain(args, Context, precision, kw):
    """The paper's evaluation shape (Sec. 4): a 60-image, two-strip flight cut
    into clusters of 12 that reuse the last three images of the cluster
    before (the first of them fixed, the other two free and fused by Eq. 8 on
    write-back), each with up to 8 overlapping images of the previous strip
    (fixed).  All clusters go to the serving loop at once (one batched
    submit); their shared IDs order them, so the flight runs as a chain.  Reports the flight's wall
    time (first submit to last result), per-cluster latency, and the mean and
    standard deviation of the reprojection error norms at each cluster's
    solution.  Returns the report and the clusters (for the oracle timing)."""
    t_gen = time.perf_counter()
    cl = A.make_chain(9)["clusters"]
    log(f"chain: {len(cl)} clusters of {[c['n_cams'] for c in cl]} images in {time.perf_counter() - t_gen:.1f}s")
    walls, lat, errs = [], [], []
    res0 = []
    for rep in range(args.chain_reps):
        ctx = Context(precision=precision, serve=True, max_slots=4, hbm_budget_bytes=1 << 30,
                      stage_threads=args.stage_threads)
        t0 = time.perf_counter()
        ts = ctx.submit_many(cl, use_resident=True, fuse_resident=True, **kw)
        for t in ts:
            ctx.ba_solve(t)
        res = []
        for t in ts:
            ctx.ba_wait(t)
            res.append(ctx.ba_fetch(t))
        walls.append(time.perf_counter() - t0)
        lat += [(r["t_done"] - r["t_submit"]) * 1e3 for r in res]
        if rep == 0:
            res0 = res
            for sc, r in zip(cl, res):
                e = A.project_obs(r["R"], r["T"], r["X"], r["k"], sc["obs_cam"], sc["obs_pt"]) - sc["obs_uv"]
                errs.append(np.sqrt((e ** 2).sum(1)))
        ctx.close()
        log(f"chain rep {rep}: {len(cl)} clusters in {walls[-1] * 1e3:.1f} ms")
    e = np.concatenate(errs)
    n_img = len({int(k) for sc in cl for k in sc["cam_ids"]})
    return {"images": n_img, "clusters": len(cl), "reps": args.chain_reps,
            "cams_range": [min(c["n_cams"] for c in cl), max(c["n_cams"] for c in cl)],
            "points_range": [min(c["n_points"] for c in cl), max(c["n_points"] for c in cl)],
            "ms_per_flight": 1e3 * float(np.mean(walls)), "ms_per_image": 1e3 * float(np.mean(walls)) / n_img,
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "reproj_err_mean_px": float(e.mean()), "reproj_err_std_px": float(e.std()),
            "paper_context": "MATLAB on an i7 laptop CPU, 60 images: 66.45 s total with feature extraction and "
                             "matching, 1.11 s per image pair (Table 1)",
            "_sample": list(zip(cl, res0))}, cl


def run_geo(args):
    """Sec. 3.1 on the serving stream's flight (4 strips x 40 images over a
    12 m DSM): the 160 footprints (corner and centre rays intersected with the
    DSM), the overlap areas of all 12,720 footprint pairs, and the Eq. (3)
    transfer of all 2120 patch centres (150 px grid) of every image into every
    image whose footprint overlaps it (and into itself).  Device time of each
    call's kernels from HIP events, best of `geo_reps`; the projection
    kernel's roofline position (HBM: 16-byte uv and 4-byte flag per output,
    32-byte ground point per source patch read once).  Returns the report
    and the inputs (for the oracle timing)."""
    from synth import geo as SG
    from paper_2511_06152_amd import Geo
    g = SG.make_geo_flight(21)
    cam = {k: g[k] for k in ("f", "cx", "cy", "width", "height")}
    uv0 = SG.patch_grid()
    n = g["n_images"]
    t_fp, t_ov, t_tr, t_pr = [], [], [], []
    with Geo(g["dsm"]) as geo:
        for rep in range(args.geo_reps + 1):
            fp, st = geo.ba_footprints(g["R"], g["T"], cam)
            t_fp.append(geo.ba_geo_last_ms())
            area = geo.ba_footprint_overlaps(fp)
            t_ov.append(geo.ba_geo_last_ms())
            if rep == 0:
                iu, ju = np.triu_indices(n, 1)
                pos = area > 0
                pairs = np.concatenate([np.stack([iu[pos], ju[pos]], 1), np.stack([ju[pos], iu[pos]], 1),
                                        np.stack([np.arange(n), np.arange(n)], 1)]).astype(np.int32)
            uv, fl, _ = geo.ba_patch_transfer(g["R"], g["T"], uv0, pairs, cam)
            t_tr.append(geo.ba_geo_last_ms())
            t_pr.append(geo.ba_geo_last_ms(last_kernel=True))
    best = lambda v: float(min(v[1:])) if len(v) > 1 else float(v[0])   # the first call loads the code object
    P, Q = len(pairs), len(uv0)
    outputs = P * Q
    byts = outputs * (16 + 4) + n * Q * 32 + P * 8 + n * 96
    pr_ms = best(t_pr)
    ach = byts / (pr_ms * 1e-3) / 1e9
    rep = {"images": n, "dsm_nodes": [g["dsm"]["nx"], g["dsm"]["ny"]], "dsm_cell_m": g["dsm"]["cell"],
           "footprints_ms": best(t_fp), "rays_footprint": 5 * n,
           "overlap_pairs": n * (n - 1) // 2, "overlapping_pairs": int((area > 0).sum()), "overlaps_ms": best(t_ov),
           "transfer_pairs": P, "patches": Q, "transfers": outputs, "reinitialised": int((fl == 2).sum()),
           "transfer_ms": best(t_tr), "transfers_per_s": outputs / (best(t_tr) * 1e-3),
           "project_roofline": {"bound": "hbm", "kernel": "k_project", "achieved": ach, "peak": 8000.0,
                                "unit": "GB/s", "frac": ach / 8000.0, "algorithmic_bytes": byts,
                                "avg_launch_us": pr_ms * 1e3}}
    log(f"geo: footprints {rep['footprints_ms'] * 1e3:.1f} us, overlaps {rep['overlaps_ms'] * 1e3:.1f} us, "
        f"transfer {rep['transfer_ms'] * 1e3:.1f} us ({outputs} outputs; projection {pr_ms * 1e3:.1f} us)")
    sel = list(range(0, len(pairs), max(1, len(pairs) // 8)))[:8]
    rep["_sample"] = [(int(pairs[i][0]), int(pairs[i][1]), uv[i].copy(), fl[i].copy()) for i in sel]
    return rep, (g, cam, uv0, pairs)


def run_global(args, Context, precision):
    """Whole-flight global adjustment: 400 cameras (10 strips x 40), 800k points,
    ~3.5M observations; the reduced camera system (m = 2400) by block-Jacobi
    PCG with FP32 products.  Times LM iterations with the cluster resident.
    Returns the report and the scene (for the oracle timing of the CPU
    baseline leg)."""
    from paper_2511_06152_amd.ba import Cluster
    t_gen = time.perf_counter()
    sc = A.scene_global(5)
    log(f"global: generated C={sc['n_cams']} P={sc['n_points']} O={sc['n_obs']} "
        f"in {time.perf_counter() - t_gen:.1f}s")
    n = args.global_iters
    total = max(args.global_total_iters, n + 1)
    # the timed iterations, then (untimed) on to `total` iterations for the
    # comparison with the oracle's state after as many
    cl = Cluster(sc, max_iters=total)
    probe = Context(precision=precision, max_slots=2, hbm_budget_bytes=64 << 20)
    foot = probe.ba_footprint(cl)
    probe.close()
    ctx = Context(precision=precision, max_slots=2, hbm_budget_bytes=int(foot * 1.05) + (64 << 20),
                  chunks_per_task=args.chunks_per_task, pcg_tol=args.global_pcg_tol, pcg_max_iters=20000)
    t = ctx.ba_submit_cluster(cl)
    ctx.ba_step(t, 1)             # admission, initial cost and the first iteration (warmup)
    cg_warm = ctx.ba_fetch(t)["cg_iters"]
    ctx.ba_profile_enable(True)
    t0 = time.perf_counter()
    ctx.ba_step(t, n)
    dt = time.perf_counter() - t0
    prof = ctx.ba_profile_read()
    r = ctx.ba_fetch(t)
    cg_timed = r["cg_iters"] - cg_warm
    out = {"cams": sc["n_cams"], "points": sc["n_points"], "obs": sc["n_obs"], "m": 6 * sc["n_cams"],
           "pcg_tol": args.global_pcg_tol, "lm_iterations_timed": n, "ms_per_lm_iteration": 1e3 * dt / n,
           "cg_iterations_total": r["cg_iters"], "cg_iterations_timed": cg_timed,
           "pcg_avg_ms": prof["pcg"][0] / max(prof["pcg"][1], 1),
           "pcg_us_per_cg_iteration": 1e3 * prof["pcg"][0] / max(cg_timed, 1),
           "kernel_avg_us": {k: 1e3 * v[0] / max(v[1], 1) for k, v in prof.items() if v[1]},
           "cost_initial": float(r["cost_log"][0]), "cost_after_timed": float(r["cost_log"][-1]),
           "hbm_footprint_bytes": foot}
    if total > n + 1:
        t0 = time.perf_counter()
        ctx.ba_step(t, total - n - 1)
        dt2 = time.perf_counter() - t0
        r = ctx.ba_fetch(t)
        out["continued"] = {"status": int(r["status"]), "iterations": int(r["iterations"]),
                            "wall_s": dt2, "cost_final": float(r["cost_log"][-1]),
                            "error_vs_oracle": global_error_vs_golden(sc, r)}
        log(f"global: {r['iterations']} iterations (status {r['status']}); error vs the oracle's state after as "
            f"many {out['continued']['error_vs_oracle']}")
    ctx.close()
    log(f"global: {out['ms_per_lm_iteration']:.2f} ms per LM iteration, {r['cg_iters']} CG iterations")
    return out, sc


GOLDEN_GLOBAL = os.path.join(ROOT, "tests", "golden", "global_400cams_seed5_iter150.txt")


def read_golden_global(path=GOLDEN_GLOBAL):
    """The oracle's converged solution of the 400-camera flight (written by
    tests/golden/make_global_solution.py): cameras R [C,3,3], T [C,3], and
    the sampled points' indices and positions; None when absent."""
    if not os.path.exists(path):
        return None
    cams, pts = [], []
    meta = {}
    part = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                if line.startswith("# iterations"):
                    tok = line[1:].split()
                    meta = {tok[i]: float(tok[i + 1]) for i in range(0, len(tok) - 1, 2)}
                part = "pts" if "points:" in line else ("cams" if "cameras:" in line else part)
                continue
            v = [float(x) for x in line.split()]
            (cams if part == "cams" else pts).append(v)
    cams, pts = np.array(cams), np.array(pts)
    return {"R": cams[:, :9].reshape(-1, 3, 3), "T": cams[:, 9:12], "idx": pts[:, 0].astype(np.int64),
            "X": pts[:, 1:4], "meta": meta}


def state_errors(sc, R_a, T_a, X_a, R_b, T_b, X_b, k=(0.0, 0.0), k_b=None, obs_sel=None):
    """RMS over observations of |p_a - p_b| (each state with its own radial
    k1, k2; the generator's forward model), max camera-centre difference, max
    attitude angle of R_a^T R_b."""
    oc, op = sc["obs_cam"], sc["obs_pt"]
    if obs_sel is not None:
        oc, op = oc[obs_sel], op[obs_sel]
    d = A.project_obs(R_a, T_a, X_a, k, oc, op) - A.project_obs(R_b, T_b, X_b, k if k_b is None else k_b, oc, op)
    rms = float(np.sqrt((d ** 2).sum(1).mean())) if len(d) else 0.0
    return {"rms_px": rms, "centres_m": float(np.abs(T_a - T_b).max()), "attitude_rad": max_angle(R_a, R_b)}


def max_angle(R_a, R_b):
    """Largest rotation angle of R_a[c]^T R_b[c] over the cameras, as
    atan2(|sin|, cos) from the skew and trace parts (accurate for small
    angles, where arccos of the trace loses half the digits)."""
    M = np.einsum("cji,cjk->cik", np.asarray(R_a), np.asarray(R_b))
    v = 0.5 * np.stack([M[:, 2, 1] - M[:, 1, 2], M[:, 0, 2] - M[:, 2, 0], M[:, 1, 0] - M[:, 0, 1]], 1)
    c = 0.5 * (np.trace(M, axis1=1, axis2=2) - 1.0)
    return float(np.max(np.arctan2(np.linalg.norm(v, axis=1), c))) if len(M) else 0.0


def global_error_vs_golden(sc, r):
    """The GPU's converged global solution against the oracle's (stored):
    every camera, and the predicted pixels of every observation of the
    stored sample of points."""
    g = read_golden_global()
    if g is None:
        return None
    sel = np.isin(sc["obs_pt"], g["idx"])
    X_ref = np.array(r["X"], copy=True)
    X_ref[g["idx"]] = g["X"]
    e = state_errors(sc, r["R"], r["T"], r["X"], g["R"], g["T"], X_ref, obs_sel=sel)
    e.update(observations_compared=int(sel.sum()), points_compared=int(len(g["idx"])),
             oracle_iterations=int(g["meta"].get("iterations", 0)))
    return e


def run_tiny(args, Context, precisions):
    """The tiny workload (6 cameras in 2 strips x 3, 2000 points, ~6k
    observations, 10 LM iterations): latency of one cluster, submit to
    result, in each precision (the FP64 path host-driven as the plain LM,
    the mixed path through ba_solve_batch)."""
    sc = A.scene_tiny(1)
    out = {"cams": sc["n_cams"], "points": sc["n_points"], "obs": sc["n_obs"], "iterations": 10}
    for name, prec in precisions:
        ctx = Context(precision=prec, max_slots=4, hbm_budget_bytes=64 << 20)
        lat = []
        for i in range(args.tiny_reps + 1):
            t0 = time.perf_counter()
            t = ctx.submit(sc, max_iters=10)
            if name == "plain_fp64":
                ctx.ba_step(t, 10)
            else:
                ctx.ba_solve_batch([t])
            r = ctx.ba_fetch(t)
            t1 = time.perf_counter()
            ctx.ba_release(t)
            if i:
                lat.append((t1 - t0) * 1e3)
        ctx.close()
        out[name] = {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "runs": len(lat),
                     "final_rms_px": r["reproj_rms"]}
    out["note"] = "submit (validation, layout, upload) to fetched result, one cluster at a time"
    return out


def run_selfcal(args, Context, ctx_kw, scenes, kw):
    """The headline batch with all five intrinsics (k1, k2, f, cx, cy)
    estimated, f submitted 0.1 % and the principal point 2 px off: the
    self-calibrating kernel instantiations, timed like the headline steps."""
    B = args.batch
    sc5 = [dict(s, intr_mask=0b11111, f=s["f"] * 1.001, cx=s["cx"] + 2.0, cy=s["cy"] - 2.0) for s in scenes]
    ctx = Context(batch_streams=args.batch_streams, **ctx_kw)
    step_ms, iters = [], []
    statuses, sample = set(), []
    for rep in range(args.selfcal_reps + 1):
        ids = [(rep * B + i) % len(sc5) for i in range(B)]
        tickets = [ctx.submit(sc5[j], **kw) for j in ids]
        for t in tickets:
            ctx.ba_step(t, 0)
        t0 = time.perf_counter()
        ctx.ba_solve_batch(tickets)
        t1 = time.perf_counter()
        for t, j in zip(tickets, ids):
            r = ctx.ba_fetch(t)
            statuses.add(int(r["status"]))
            if rep > 0:
                iters.append(r["iterations"])
            if rep == 0 and j == 0 and not sample:
                sample.append((sc5[0], r))
            ctx.ba_release(t)
        if rep > 0:
            step_ms.append((t1 - t0) * 1e3)
        log(f"self-calibration rep {rep}{'' if rep else ' (warmup)'}: {(t1 - t0) * 1e3:.2f} ms for {B} clusters")
    ctx.close()
    ms = float(np.mean(step_ms))
    bad = statuses & {4, 5}
    if bad:
        raise RuntimeError(f"self-calibration leg: clusters ended stalled or with a bad initial state {bad}")
    return {"clusters": B, "reps": args.selfcal_reps, "intr_mask": "k1 k2 f cx cy", "m": 6 * 12 + 5,
            "ms_per_batch": ms, "clusters_per_s": B / (ms / 1e3), "mean_iterations": float(np.mean(iters)),
            "statuses": sorted(statuses), "_sample": sample}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_leg(args, scenes, mixed_final, plain_final, uneven, selfcal, stream, chain, geo, geo_in,
                     glob_scene):
    """The FP64 oracle on the host: throughput at one thread and at the
    cores this process may use (clusters are independent, so the threads
    solve different clusters), and the final error of each GPU leg's results
    against the oracle's on the same inputs and rule."""
    import concurrent.futures as cf
    import oracle
    oracle.build(force=False)
    kw = dict(max_iters=args.max_iters, stop_on_ftol=True, ftol=args.ftol)

    def errs(sc, got, ref):
        """|p_gpu - p_oracle| RMS over every observation (each state with
        its own intrinsics, the oracle's projection), centres, attitude."""
        kg = np.concatenate([got["k"], got["intr"]])
        uv_g = oracle.residuals(sc, (got["R"], got["T"], got["X"], kg))["uv"]
        uv_o = oracle.residuals(sc, ref["state"])["uv"]
        R_o, T_o = ref["state"][0], ref["state"][1]
        att = max_angle(got["R"], R_o)
        return {"rms_px": float(np.sqrt(((uv_g - uv_o) ** 2).sum(1).mean())) if len(uv_g) else 0.0,
                "centres_m": float(np.abs(got["T"] - T_o).max()), "attitude_rad": att,
                "iterations_gpu": int(got["iterations"]), "iterations_oracle": int(ref["iterations"])}

    def worst(rows):
        if not rows:
            return None
        out = {k: max(r[k] for r in rows) for k in ("rms_px", "centres_m", "attitude_rad")}
        out["results_compared"] = len(rows)
        out["iterations_equal"] = all(r["iterations_gpu"] == r["iterations_oracle"] for r in rows)
        return out

    # throughput: one thread, then the host's cores
    n1 = args.cpu_clusters
    t0 = time.perf_counter()
    refs = [oracle.solve(scenes[i % len(scenes)], **kw) for i in range(n1)]
    dt1 = time.perf_counter() - t0
    nth = args.cpu_threads or min(len(os.sched_getaffinity(0)), 16)
    n_par = 2 * nth
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(nth) as ex:       # the oracle's ctypes calls release the GIL
        list(ex.map(lambda i: oracle.solve(scenes[i % len(scenes)], **kw), range(n_par)))
    dtn = time.perf_counter() - t0
    cpu = {"value": n_par / dtn, "unit": "clusters/s", "cores": nth, "kind": "oracle",
           "sample": f"{n_par} clusters of the headline workload, same termination rule, FP64 C++ oracle, "
                     f"{nth} threads each solving whole clusters ({dtn:.1f} s)",
           "cpu_model": cpu_model(), "cpus_visible": len(os.sched_getaffinity(0)),
           "single_thread": {"value": n1 / dt1, "unit": "clusters/s", "cores": 1,
                             "sample": f"{n1} clusters, one thread ({dt1:.1f} s)"}}
    fe = {}
    fe["headline_mixed"] = worst([errs(scenes[i % len(scenes)], mixed_final[i % len(scenes)], refs[i])
                                  for i in range(n1) if i % len(scenes) in mixed_final])
    fe["plain_fp64"] = worst([errs(scenes[i % len(scenes)], plain_final[i % len(scenes)], refs[i])
                              for i in range(n1) if i % len(scenes) in plain_final])
    if uneven is not None and uneven.get("_sample"):
        fe["batched_uneven"] = worst([errs(sc, r, oracle.solve(sc, **kw)) for sc, r in uneven["_sample"]])
    if selfcal is not None and selfcal.get("_sample"):
        fe["self_calibration"] = worst([errs(sc, r, oracle.solve(sc, **kw)) for sc, r in selfcal["_sample"]])

    def replay(clusters, results, from_gpu=False):
        """Clusters chained by resident state, replayed on the host in
        submission order: each starts from the values the clusters before it
        left (fused poses by Eq. 8, solved points), and is solved by the oracle
        with the same rule; returns the errors of the GPU's results.  The
        values left are the oracle's own solutions (the whole chain against
        the oracle's chain), or with from_gpu the GPU's results (each
        cluster's solve against the oracle's from the same start)."""
        store_c, store_p, rows = {}, {}, []
        for sc, got in zip(clusters, results):
            R, T, X = sc["R"].copy(), sc["T"].copy(), sc["X"].copy()
            for k, cid in enumerate(sc["cam_ids"]):
                if cid in store_c:
                    R[k], T[k] = store_c[cid][0], store_c[cid][1]
            for j, pid in enumerate(sc["point_ids"]):
                if pid in store_p:
                    X[j] = store_p[pid]
            sc2 = dict(sc, R=R, T=T, X=X)
            ref = oracle.solve(sc2, **kw)
            if got is not None:
                rows.append(errs(sc2, got, ref))
            Rf, Tf, Xf, _ = ref["state"]
            if from_gpu and got is not None:
                Rf, Tf, Xf = got["R"], got["T"], got["X"]
            n = np.bincount(sc["obs_cam"], minlength=sc["n_cams"]).astype(np.float64)
            for k, cid in enumerate(sc["cam_ids"]):
                if not sc["fixed"][k] and cid in store_c:
                    store_c[cid] = oracle.fuse_pose(*store_c[cid], Rf[k], Tf[k], n[k])
                else:
                    store_c[cid] = (Rf[k], Tf[k], float(n[k]))
            for j, pid in enumerate(sc["point_ids"]):
                store_p[pid] = Xf[j]
        return rows

    if chain is not None and chain.get("_sample"):
        cl = [c for c, _ in chain["_sample"]]
        t0 = time.perf_counter()
        rows = replay(cl, [r for _, r in chain["_sample"]])
        cpu["chain_s_per_flight"] = time.perf_counter() - t0
        cpu["chain_sample"] = f"the chained {len(cl)}-cluster flight once, same termination rule, single-threaded"
        fe["paper_chain"] = worst(rows)
        if fe["paper_chain"]:
            per = worst(replay(cl, [r for _, r in chain["_sample"]], from_gpu=True))
            fe["paper_chain"]["per_cluster"] = per
            fe["paper_chain"]["note"] = ("the GPU's chain against the oracle's chain (each cluster started from "
                                         "what the earlier clusters of its own chain left); per_cluster: each "
                                         "GPU cluster against the oracle's solve from the same start (the "
                                         "GPU's chain values), so that solve error and its propagation along "
                                         "the chain are told apart")
    if stream is not None and stream.get("_sample"):
        fe["serving_stream"] = worst(replay([c for c, _ in stream["_sample"]], [r for _, r in stream["_sample"]]))
        if fe["serving_stream"]:
            fe["serving_stream"]["note"] = "the stream's first clusters (repetition 0), replayed in submission order"
    if geo_in is not None:
        from oracle import geo as OG
        g, cam, uv0, pairs = geo_in
        t0 = time.perf_counter()
        n_out, d_uv, fl_eq = 0, 0.0, True
        for s_, d_, uv_g, fl_g in geo["_sample"]:
            uv_o, _, fl_o = OG.transfer_eq3(g["dsm"], g["R"][s_], g["T"][s_], g["R"][d_], g["T"][d_], cam["f"],
                                            cam["cx"], cam["cy"], cam["width"], cam["height"], uv0)
            n_out += len(uv0)
            ok = np.isfinite(uv_o).all(1) & np.isfinite(uv_g).all(1)
            if ok.any():
                d_uv = max(d_uv, float(np.abs(uv_g[ok] - uv_o[ok]).max()))
            fl_eq = fl_eq and bool(np.array_equal(np.isfinite(uv_o).all(1), np.isfinite(uv_g).all(1)))
        dt = time.perf_counter() - t0
        cpu["geo_transfers_per_s"] = n_out / dt
        cpu["geo_sample"] = f"{n_out} Eq. (3) transfers (8 pairs x {len(uv0)} patches), single-threaded numpy"
        fe["geo_transfer"] = {"max_abs_px": d_uv, "hits_equal": fl_eq, "transfers_compared": n_out}
    if glob_scene is not None and args.global_oracle_iters > 0:
        t0 = time.perf_counter()
        oracle.solve(glob_scene, max_iters=args.global_oracle_iters)
        cpu["global_ba_s_per_lm_iteration"] = (time.perf_counter() - t0) / args.global_oracle_iters
        cpu["global_ba_sample"] = (f"{args.global_oracle_iters} LM iteration(s) of the 400-camera flight "
                                   "(dense FP64 Schur complement and Cholesky, m = 2400), single-threaded")
    fe["bars"] = {"rms_px": 1e-3, "centres_m": 1e-3, "attitude_rad": 2e-6}
    return cpu, fe


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64, help="clusters per step")
    ap.add_argument("--scenes", type=int, default=8, help="distinct seeded clusters (cycled)")
    ap.add_argument("--max-iters", type=int, default=20)
    ap.add_argument("--ftol", type=float, default=1e-6)
    ap.add_argument("--plain", type=int, default=8, help="clusters solved by the plain FP64 path")
    ap.add_argument("--serve", type=int, default=192, help="clusters timed at each serving load level (0: skip)")
    ap.add_argument("--serve-slots", default="4,8,16", help="serving load levels: clusters kept in flight")
    ap.add_argument("--stage-threads", type=int, default=8,
                    help="host threads laying out the clusters submitted to the serving loops (0: the caller's)")
    ap.add_argument("--cpu-clusters", type=int, default=3, help="clusters solved by the oracle (0: skip)")
    ap.add_argument("--chunks-per-task", type=int, default=10, help="64-lane chunks per block task (batched context)")
    ap.add_argument("--chunks-per-wg", type=int, default=32,
                    help="observation lanes of a point-pass workgroup, in units of 64 (batched context)")
    ap.add_argument("--batch-streams", type=int, default=2,
                    help="streams a batch is split across (1: one stream, no overlap)")
    ap.add_argument("--iters-per-tick", type=int, default=10,
                    help="LM iterations launched between control read-backs (batched context)")
    ap.add_argument("--uneven", type=int, default=256,
                    help="clusters of the uneven batched workload (6-24 cameras, 5k-60k points; 0: skip)")
    ap.add_argument("--uneven-scenes", type=int, default=64, help="distinct seeded uneven clusters (cycled)")
    ap.add_argument("--uneven-serve", type=int, default=1,
                    help="also pass the uneven clusters through the serving loop under a quarter budget (0: skip)")
    ap.add_argument("--global-iters", type=int, default=10,
                    help="LM iterations of the whole-flight global adjustment (400 cameras, 800k points; 0: skip)")
    ap.add_argument("--global-oracle-iters", type=int, default=1,
                    help="oracle LM iterations timed on the whole-flight scene (0: skip)")
    ap.add_argument("--stream-reps", type=int, default=5,
                    help="repetitions of the serving stream (4 strips x 40 images, one cluster per arriving "
                         "image, resident state; 0: skip)")
    ap.add_argument("--stream-window", type=int, default=2, help="stream clusters in flight (closed loop)")
    ap.add_argument("--selfcal-reps", type=int, default=3,
                    help="timed batches of the headline clusters with all five intrinsics estimated (0: skip)")
    ap.add_argument("--chain-reps", type=int, default=5,
                    help="repetitions of the chained 60-image flight (clusters of 12 reusing 3 images, Eq. 8 "
                         "fusion; 0: skip)")
    ap.add_argument("--geo-reps", type=int, default=5,
                    help="timed repetitions of the footprint / overlap / Eq. (3) transfer leg (0: skip)")
    ap.add_argument("--global-pcg-tol", type=float, default=1e-5,
                    help="cap of the PCG forcing term in the global leg (1e-5: the state after 150 iterations "
                         "within the mixed-path bars of the oracle's)")
    ap.add_argument("--global-total-iters", type=int, default=150,
                    help="after the timed global iterations, further ones (untimed) up to this many in all, "
                         "for the comparison with the oracle's state after as many (stored by "
                         "tests/golden/make_global_solution.py); at most the timed ones + 1: skip")
    ap.add_argument("--stream-oracle-clusters", type=int, default=6,
                    help="first serving-stream clusters replayed by the oracle for the final-error figures")
    ap.add_argument("--batched-fp64", type=int, default=1,
                    help="also time the headline batch through ba_solve_batch in plain FP64 (0: skip)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the multi-threaded oracle timing (0: the cores this process may "
                         "use, at most 16)")
    ap.add_argument("--tiny-reps", type=int, default=20,
                    help="timed single-cluster runs of the tiny workload in each precision (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times) and exit: the reference "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(clusters are independent: see the sharding note in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return

    from paper_2511_06152_amd import BA_FP64, BA_MIXED, Context

    t_gen = time.perf_counter()
    scenes = [A.make_scene(A.spec_cluster12(), 2 + i) for i in range(args.scenes)]
    log(f"generated {len(scenes)} clusters in {time.perf_counter() - t_gen:.1f}s: "
        + ", ".join(f"C={s['n_cams']} P={s['n_points']} O={s['n_obs']}" for s in scenes[:3]) + " ...")
    kw = dict(max_iters=args.max_iters, stop_on_ftol=True, ftol=args.ftol)
    flops = [block_flops(s) for s in scenes]

    # ---- mixed, batched: the timed steps --------------------------------------------------
    B = args.batch
    ctx_kw = dict(precision=BA_MIXED, max_slots=max(B, 1), hbm_budget_bytes=int(B * 16e6) + (256 << 20),
                  chunks_per_task=args.chunks_per_task, chunks_per_wg=args.chunks_per_wg,
                  iters_per_tick=args.iters_per_tick)
    ctx = Context(batch_streams=args.batch_streams, **ctx_kw)
    step_ms, iters_total, mixed_final = [], 0, {}
    fl_total = {"blocks": 0.0}
    ctx.ba_profile_enable(False)
    for step in range(args.warmup + args.steps):
        timed = step >= args.warmup
        ids = [(step * B + i) % len(scenes) for i in range(B)]
        tickets = [ctx.submit(scenes[j], **kw) for j in ids]
        for t in tickets:
            ctx.ba_step(t, 0)     # admission: upload, origin shift, initial FP64 cost
        if timed:
            ctx.ba_profile_enable(BLOCK_KERNELS)   # the two roofline candidates only
        t0 = time.perf_counter()
        ctx.ba_solve_batch(tickets)
        t1 = time.perf_counter()
        if timed:
            ctx.ba_profile_enable(False)
            step_ms.append((t1 - t0) * 1e3)
        for t, j in zip(tickets, ids):
            r = ctx.ba_fetch(t)
            if timed:
                iters_total += r["iterations"]
                for k in fl_total:
                    fl_total[k] += r["iterations"] * flops[j][k]
            if j not in mixed_final:
                mixed_final[j] = r
            ctx.ba_release(t)
        log(f"step {step}{'' if timed else ' (warmup)'}: {(t1 - t0) * 1e3:.2f} ms for {B} clusters")
    prof = ctx.ba_profile_read()
    # one more step, untimed, with every kernel timed: the per-kernel breakdown
    tickets = [ctx.submit(scenes[i % len(scenes)], **kw) for i in range(B)]
    for t in tickets:
        ctx.ba_step(t, 0)
    ctx.ba_profile_enable(True)
    ctx.ba_solve_batch(tickets)
    ctx.ba_profile_enable(False)
    prof_all = ctx.ba_profile_read()
    mfma_total = 0.0
    for i, t in enumerate(tickets):
        mfma_total += ctx.ba_fetch(t)["iterations"] * solve_mfma_flops(scenes[i % len(scenes)])
        ctx.ba_release(t)
    ctx.close()
    sv_ms, sv_n = prof_all["solve"]
    solve_mc = {"kernel": "k_solve", "unit": "TFLOP/s", "peak": PEAK_MFMA_F64_TFLOPS,
                "mfma_flop_per_launch": mfma_total / max(sv_n, 1), "avg_launch_us": sv_ms / max(sv_n, 1) * 1e3,
                "achieved": (mfma_total / max(sv_n, 1)) / (sv_ms / max(sv_n, 1) / 1e3) / 1e12 if sv_n else None,
                "note": "FP64 matrix-core work of the dense solve (16x16x16 panel and trailing block products "
                        "of the factorisation, products of the block inverse W = L^-1) over the kernel's whole "
                        "launch; the kernel is latency-bound (m <= 149)"}
    solve_mc["frac"] = solve_mc["achieved"] / PEAK_MFMA_F64_TFLOPS if solve_mc["achieved"] else None
    ms_per_step = float(np.mean(step_ms))
    # the block kernels alone on the GPU: one more step on a single stream
    iso = measure_isolated(args, Context, ctx_kw, scenes, kw, flops) if args.batch_streams > 1 else None
    value = B / (ms_per_step / 1e3)
    selfcal = run_selfcal(args, Context, ctx_kw, scenes, kw) if args.selfcal_reps > 0 else None

    # ---- the same batch through ba_solve_batch in plain FP64: what FP32 assembly alone buys
    batched_fp64 = None
    if args.batched_fp64:
        fctx = Context(batch_streams=args.batch_streams, **dict(ctx_kw, precision=BA_FP64))
        f_ms, f_it = [], 0
        for step in range(1 + max(args.steps // 2, 1)):
            ids = [(step * B + i) % len(scenes) for i in range(B)]
            tickets = [fctx.submit(scenes[j], **kw) for j in ids]
            for t in tickets:
                fctx.ba_step(t, 0)
            t0 = time.perf_counter()
            fctx.ba_solve_batch(tickets)
            t1 = time.perf_counter()
            for t in tickets:
                if step:
                    f_it += fctx.ba_fetch(t)["iterations"]
                fctx.ba_release(t)
            if step:
                f_ms.append((t1 - t0) * 1e3)
            log(f"batched FP64 step {step}{'' if step else ' (warmup)'}: {(t1 - t0) * 1e3:.2f} ms for {B} clusters")
        fctx.close()
        batched_fp64 = {"clusters_per_s": B / (float(np.mean(f_ms)) / 1e3), "ms_per_batch": float(np.mean(f_ms)),
                        "mean_iterations": f_it / (B * len(f_ms)),
                        "note": "ba_solve_batch with precision BA_FP64 on the same batch, context options and "
                                "rule: FP64 assembly, everything else as the headline"}

    dom = "blocks"
    asm_ms, asm_n = prof[dom]
    asm_avg_ms = asm_ms / max(asm_n, 1)
    achieved_tflops = fl_total[dom] / max(asm_n, 1) / (asm_avg_ms / 1e3) / 1e12 if asm_n else float("nan")
    # (the mixed path has no separate pair-task launch: that slot is empty)
    kernels = {k: {"avg_us": (v[0] / max(v[1], 1)) * 1e3, "launches": v[1]} for k, v in prof_all.items()
               if k != "pairblk"}

    in_step = {"bound": "alu", "kernel": f"k_{dom}<float>", "achieved": achieved_tflops,
               "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP32_TFLOPS,
               "peak_nonpacked": PEAK_VALU_TFLOPS, "frac_of_nonpacked": achieved_tflops / PEAK_VALU_TFLOPS,
               "traffic": traffic_bytes(dom, B, args.batch_streams, (args.chunks_per_wg, args.chunks_per_task)),
               "traffic_unit": "bytes per launch",
               "avg_launch_us": asm_avg_ms * 1e3, "algorithmic_flop_per_launch": fl_total[dom] / max(asm_n, 1),
               "batch_streams": args.batch_streams,
               "note": "timed steps: launches of one part of the batch, beside the other parts' kernels"}

    # ---- plain FP64 GPU LM: one cluster at a time, host-driven ---------------------------
    plain_lat, plain_e2e, plain_final = [], [], {}
    if args.plain > 0:
        pctx = Context(precision=BA_FP64, max_slots=4, hbm_budget_bytes=256 << 20)
        for i in range(args.plain + 1):
            j = i % len(scenes)
            ts = time.perf_counter()
            t = pctx.submit(scenes[j], **kw)
            pctx.ba_step(t, 0)
            t0 = time.perf_counter()
            pctx.ba_step(t, args.max_iters)
            t1 = time.perf_counter()
            r = pctx.ba_fetch(t)
            t2 = time.perf_counter()
            pctx.ba_release(t)
            if i == 0:
                continue  # warmup
            plain_lat.append((t1 - t0) * 1e3)
            plain_e2e.append((t2 - ts) * 1e3)
            plain_final.setdefault(j, r)
        pctx.close()
    plain_cps = 1e3 / float(np.mean(plain_lat)) if plain_lat else float("nan")

    # ---- mixed-path solve latency of one cluster alone ---------------------------------
    one_lat = []
    octx = Context(precision=BA_MIXED, max_slots=4, hbm_budget_bytes=256 << 20)
    for i in range(args.plain + 1 if args.plain > 0 else 0):
        j = i % len(scenes)
        t = octx.submit(scenes[j], **kw)
        octx.ba_step(t, 0)
        t0 = time.perf_counter()
        octx.ba_solve_batch([t])
        t1 = time.perf_counter()
        octx.ba_release(t)
        if i:
            one_lat.append((t1 - t0) * 1e3)
    octx.close()

    # ---- continuous-batching serving loop (closed loop, submit -> result) --------------
    # Each load level: a context whose slots equal the clusters kept in flight,
    # a warm-up of two rounds of the slots (pinned buffers, layout storage),
    # then args.serve clusters timed from ba_submit_cluster to the result.
    serve = {}
    if args.serve > 0:
        levels = []
        for slots in sorted({int(x) for x in args.serve_slots.split(",") if x}):
            sctx = Context(precision=BA_MIXED, serve=True, max_slots=slots,
                           hbm_budget_bytes=int(slots * 16e6) + (256 << 20), stage_threads=args.stage_threads)
            warm = 2 * slots
            inflight, lat = [], []
            nxt = done = 0
            t_start = time.perf_counter()
            while done < args.serve + warm:
                while len(inflight) < slots and nxt < args.serve + warm:
                    t = sctx.submit(scenes[nxt % len(scenes)], **kw)
                    sctx.ba_solve(t)
                    inflight.append(t)
                    nxt += 1
                t = inflight.pop(0)
                sctx.ba_wait(t)
                r = sctx.ba_fetch(t)
                if done >= warm:
                    lat.append((r["t_done"] - r["t_submit"]) * 1e3)
                sctx.ba_release(t)
                done += 1
                if done == warm:
                    t_start = time.perf_counter()
            wall = time.perf_counter() - t_start
            sctx.close()
            levels.append({"slots": slots, "clusters": len(lat), "clusters_per_s": len(lat) / wall,
                           "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99)})
        top = levels[-1]
        serve = {"clusters": top["clusters"], "slots": top["slots"], "stage_threads": args.stage_threads,
                 "clusters_per_s": top["clusters_per_s"], "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"],
                 "levels": levels,
                 "note": "closed loop with `slots` clusters in flight, after a warm-up of two rounds; latency from "
                         "ba_submit_cluster to the result (validation, background layout, upload and admission "
                         "included); the top-level figures are the highest load level"}

    # ---- equal-RMS check -------------------------------------------------------------------
    rms = {}
    common = sorted(set(mixed_final) & set(plain_final))
    if common:
        d, dp = [], []
        for j in common:
            rm = mixed_final[j]["reproj_rms"]
            rp = plain_final[j]["reproj_rms"]
            d.append(abs(rm - rp))
            # RMS over the observations of |p_mixed - p_plain| at the two final states
            dp.append(state_errors(scenes[j], *mixed_final[j]["state"][:3], *plain_final[j]["state"][:3],
                                   k=mixed_final[j]["k"], k_b=plain_final[j]["k"])["rms_px"])
            rms.setdefault("mixed_px", rm)
            rms.setdefault("plain_fp64_px", rp)
        rms["max_abs_diff_of_rms_px"] = float(max(d))
        rms["max_rms_of_prediction_diff_px"] = float(max(dp))
        rms["clusters_compared"] = len(common)
        rms["note"] = ("reprojection RMS of each path from ba_fetch (device FP64); the prediction difference "
                       "is the RMS over all observations of |p_mixed - p_plain|")

    # ---- the tiny workload: one cluster's latency, submit to result ---------------------------
    tiny = run_tiny(args, Context, [("plain_fp64", BA_FP64), ("mixed", BA_MIXED)]) if args.tiny_reps > 0 else None

    # ---- uneven batched clusters: 6-24 cameras, 5k-60k points, one batch --------------------
    uneven = run_uneven(args, Context, BA_MIXED, kw) if args.uneven > 0 else None

    # ---- serving stream: one cluster per arriving image, resident state -------------------
    stream = run_stream(args, Context, BA_MIXED, kw) if args.stream_reps > 0 else None

    # ---- the paper's chained flight: clusters of 12 reusing 3 images, Eq. (8) fusion --------
    chain, chain_cl = run_chain(args, Context, BA_MIXED, kw) if args.chain_reps > 0 else (None, None)

    # ---- footprints, overlaps and Eq. (3) patch transfer over the DSM (Sec. 3.1) -------------
    geo, geo_in = run_geo(args) if args.geo_reps > 0 else (None, None)

    # ---- whole-flight global adjustment (PCG on the reduced camera system) ------------------
    glob, glob_scene = run_global(args, Context, BA_MIXED) if args.global_iters > 0 else (None, None)

    # ---- CPU baseline: the FP64 oracle on the host cores, and the final error -----------------
    # of every leg's results against the oracle's (the only place the oracle runs)
    cpu, final_err = None, None
    if args.cpu_clusters > 0:
        cpu, final_err = cpu_baseline_leg(args, scenes, mixed_final, plain_final, uneven, selfcal, stream, chain,
                                          geo, geo_in, glob_scene)
    if glob is not None and glob.get("continued"):
        final_err = final_err or {}
        final_err["global_ba"] = dict(glob["continued"]["error_vs_oracle"] or {},
                                      note=f"GPU state (mixed, PCG forcing term capped at {args.global_pcg_tol:g}) "
                                           "after 150 LM iterations against the oracle's (exact steps) after 150, "
                                           "stored by "
                                           "tests/golden/make_global_solution.py; every camera, and every "
                                           "observation of 5000 sampled points")
    for leg in (uneven, stream, chain, geo, selfcal):
        if leg is not None:
            leg.pop("_sample", None)

    O_mean = float(np.mean([s["n_obs"] for s in scenes]))
    P_mean = float(np.mean([s["n_points"] for s in scenes]))
    out = {
        "metric": "local-BA clusters/sec + p50/p99 solve latency vs plain FP64 LM at equal RMS",
        "value": value,
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded aerial scenes, synth/aerial.py)",
        "config": {
            "workload": "paper-scale local cluster: 12 cameras (2 strips x 6), 8000x6000 px, f=50 mm, 300 m, "
                        "80/60 % overlap, one tie point per 150 px cell, k1/k2 estimated",
            "clusters_per_step": B, "points_mean": P_mean, "obs_mean": O_mean,
            "max_iters": args.max_iters, "ftol": args.ftol, "mean_iterations": iters_total / max(B * args.steps, 1),
            "path": "mixed: FP32 assembly, FP64 Cholesky + refinement, FP64 cost/gain ratio, batched device-side LM",
        },
        "latency_ms": {"one_cluster_mixed_p50": pct(one_lat, 50), "one_cluster_mixed_p99": pct(one_lat, 99),
                       "serving": serve},
        "plain_fp64": {"clusters_per_s": plain_cps, "p50_ms": pct(plain_lat, 50), "p99_ms": pct(plain_lat, 99),
                       "clusters": len(plain_lat),
                       "submit_to_result_p50_ms": pct(plain_e2e, 50), "submit_to_result_p99_ms": pct(plain_e2e, 99),
                       "note": "p50/p99: the LM iterations of an admitted cluster; submit_to_result: from "
                               "ba_submit_cluster (validation, layout, upload, admission) to the fetched result, "
                               "as the serving latencies"},
        "speedup_vs_plain_fp64": value / plain_cps if plain_lat else None,
        "rms": rms,
        "kernels": kernels,
        # the dominant kernel's roofline position: measured on its own (one
        # stream; with several, each launch shares the GPU with the other
        # parts' kernels and a trace, which perturbs that overlap, cannot
        # confirm its duration); the in-step figure beside it
        "roofline": iso if iso is not None else in_step,
        "roofline_in_step": in_step,
        "solve_matrix_cores": solve_mc,
        "cpu_baseline": cpu,
        "final_error_vs_oracle": final_err,
        "batched_fp64": batched_fp64,
        "speedup_vs_batched_fp64": value / batched_fp64["clusters_per_s"] if batched_fp64 else None,
        "tiny": tiny,
        "batched_uneven": uneven,
        "serving_stream": stream,
        "self_calibration": selfcal,
        "paper_chain": chain,
        "geo": geo,
        "global_ba": glob,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
