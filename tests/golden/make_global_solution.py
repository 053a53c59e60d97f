"""Writes the FP64 oracle's solution of the whole-flight global adjustment
(400 cameras in 10 strips of 40, 800k tie points, ~3.5M observations;
synth.aerial.scene_global(5)), the reference the GPU's PCG solve is held to
at full size:

  global_400cams_seed5_iter20.txt   the state after 20 Levenberg-Marquardt
                                    iterations from the initial state
                                    (lambda0 = 1e-4), one continuous run;
  global_400cams_seed5_iter150.txt  the state after 150 iterations: the
                                    first run continued in chunks of 10, each
                                    starting from the previous chunk's state
                                    and final damping.

Calls only the oracle (oracle/) and the seeded scene generator.  Stored
per file: every camera's R (row-major) and T, the index and position of 5000
points drawn without replacement by numpy's default_rng(20251106), the
final cost and the iteration count.  Run (about 25 minutes on one core):

    python tests/golden/make_global_solution.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import aerial as A  # noqa: E402

N_SAMPLE = 5000
SAMPLE_SEED = 20251106
FIRST, TOTAL = 20, 150


def sample_points(n_points):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n_points, N_SAMPLE, replace=False))


def moved(sc, sel_obs, a, b):
    uv_a = oracle.residuals(sc, a)["uv"][sel_obs]
    uv_b = oracle.residuals(sc, b)["uv"][sel_obs]
    rms = float(np.sqrt(((uv_a - uv_b) ** 2).sum(1).mean()))
    dT = float(np.abs(a[1] - b[1]).max())
    M = np.einsum("cji,cjk->cik", a[0], b[0])
    v = 0.5 * np.stack([M[:, 2, 1] - M[:, 1, 2], M[:, 0, 2] - M[:, 2, 0], M[:, 1, 0] - M[:, 0, 1]], 1)
    att = float(np.max(np.arctan2(np.linalg.norm(v, axis=1), 0.5 * (np.trace(M, axis1=1, axis2=2) - 1.0))))
    return rms, dT, att


def write(path, sc, idx, state, iters, E):
    R, T, X, _ = state
    with open(path, "w") as fh:
        fh.write("# FP64 oracle state of synth.aerial.scene_global(5), written by make_global_solution.py\n")
        fh.write(f"# iterations {iters} final_cost {E:.17g} n_cams {sc['n_cams']} n_points {sc['n_points']} "
                 f"sample_seed {SAMPLE_SEED} n_sample {N_SAMPLE}\n")
        fh.write("# cameras: R00 R01 R02 R10 R11 R12 R20 R21 R22 T0 T1 T2\n")
        for c in range(sc["n_cams"]):
            fh.write(" ".join(f"{v:.17g}" for v in list(R[c].ravel()) + list(T[c])) + "\n")
        fh.write("# points: index X Y Z\n")
        for j in idx:
            fh.write(f"{j} " + " ".join(f"{v:.17g}" for v in X[j]) + "\n")
    print(f"wrote {path}", flush=True)


def main():
    t0 = time.time()
    sc = A.scene_global(5)
    print(f"scene: C={sc['n_cams']} P={sc['n_points']} O={sc['n_obs']} ({time.time() - t0:.0f} s)", flush=True)
    idx = sample_points(sc["n_points"])
    sel_obs = np.isin(sc["obs_pt"], idx)
    S = oracle.Scene(sc)
    r = oracle.solve(S, oracle.initial_state(sc), max_iters=FIRST, lambda0=1e-4)
    state, lam, total = r["state"], r["lambda"], r["iterations"]
    print(f"{total} iterations ({r['accepted']} accepted): E {r['cost_log'][-1]:.12g} ({time.time() - t0:.0f} s)",
          flush=True)
    write(os.path.join(HERE, f"global_400cams_seed5_iter{FIRST}.txt"), sc, idx, state, total, r["cost_log"][-1])
    while total < TOTAL:
        r = oracle.solve(S, state, max_iters=10, lambda0=lam)
        total += r["iterations"]
        d = moved(sc, sel_obs, state, r["state"])
        state, lam = r["state"], r["lambda"]
        print(f"{total} iterations: E {r['cost_log'][-1]:.12g}, chunk moved {d[0]:.2e} px, {d[1]:.2e} m, "
              f"{d[2]:.2e} rad ({time.time() - t0:.0f} s)", flush=True)
    write(os.path.join(HERE, f"global_400cams_seed5_iter{TOTAL}.txt"), sc, idx, state, total, r["cost_log"][-1])


if __name__ == "__main__":
    main()
