"""Host-side checks of bench.py: the one-GPU contract, the algorithmic flop
counts it divides by (against a brute-force count over the observations),
and the guard that withholds measured traffic from other configurations."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from synth import aerial as A  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_block_flops_against_brute_force():
    sc = A.make_scene(A.spec_micro(n_strips=2, imgs_per_strip=3, n_points=400, n_fixed=1, intr_mask=3,
                                   k_true=(-0.05, 0.02)), 5)
    fl = bench.block_flops(sc)
    free = sc["fixed"] == 0
    n_cam_obs, n_pairs = 0, 0
    for j in range(sc["n_points"]):
        cams = [int(c) for c in sc["obs_cam"][sc["obs_pt"] == j] if free[c]]
        n_cam_obs += len(cams)
        n_pairs += sum(1 for a in range(len(cams)) for b in range(a + 1, len(cams)))
    assert fl["camblk"] == (bench.FLOP_CAM_OBS + bench.FLOP_CAM_INTR_OBS) * n_cam_obs
    assert fl["pairblk"] == bench.FLOP_PAIR * n_pairs
    sc["intr_mask"] = 0
    assert bench.block_flops(sc)["camblk"] == bench.FLOP_CAM_OBS * n_cam_obs


def test_traffic_only_for_the_measured_configuration():
    k = next(iter(bench.TRAFFIC["kib"]))
    streams, kernel = k
    assert bench.traffic_bytes(kernel, bench.TRAFFIC["clusters"] + 1, streams) is None
    assert bench.traffic_bytes(kernel, bench.TRAFFIC["clusters"], 7) is None
    assert bench.traffic_bytes("no_such_kernel", bench.TRAFFIC["clusters"], streams) is None
    cpw, cpt = bench.TRAFFIC["chunks"]
    assert bench.traffic_bytes(kernel, bench.TRAFFIC["clusters"], streams, (cpw + 1, cpt)) is None


def test_solve_mfma_flops_against_a_count_of_block_products():
    """Panel and trailing products of the right-looking 16x16-block Cholesky
    and the products of the block inverse W = L^-1, counted by walking the
    loops, for systems of 1..10 blocks per side."""
    for free, intr in [(1, 0), (2, 2), (5, 3), (11, 3), (12, 3), (16, 0), (24, 3), (24, 0), (24, 31), (12, 28)]:
        sc = {"fixed": np.array([0] * free + [1] * 3, np.uint8), "intr_mask": intr}
        m = 6 * free + bin(intr).count("1")
        nb = -(-m // 16)
        prods = 0
        for K in range(nb):
            prods += sum(1 for I in range(K + 1, nb))                                   # L_IK = A_IK L_KK^-T
            prods += sum(1 for J in range(K + 1, nb) for I in range(J, nb))             # A_IJ -= L_IK L_JK^T
        for I in range(1, nb):
            for J in range(I):
                prods += sum(1 for K in range(J, I)) + 1                                # W_IJ = -Li_I sum L_IK W_KJ
        assert bench.solve_mfma_flops(sc) == 2 * 16 ** 3 * prods
