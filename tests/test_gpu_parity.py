"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs."""
import numpy as np
import pytest

import oracle
from synth import aerial as A

pytestmark = pytest.mark.gpu


def gpu_step(sc, iters, precision=0, **kw):
    from paper_2511_06152_amd import Context
    with Context(precision=precision) as ctx:
        t = ctx.submit(sc, max_iters=iters, **kw)
        ctx.ba_step(t, iters)
        return ctx.ba_fetch(t)


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1e-300)


def test_tiny_fp64_cost_per_iteration():
    """Plain FP64 GPU LM matches the oracle's cost at every iteration to 1e-8."""
    sc = A.scene_tiny(1)
    print("case tiny seed 1", sc["n_cams"], sc["n_points"], sc["n_obs"], flush=True)
    ref = oracle.solve(sc, max_iters=10)
    got = gpu_step(sc, 10)
    print("oracle", ref["cost_log"], flush=True)
    print("gpu   ", got["cost_log"], flush=True)
    assert got["iterations"] == ref["iterations"]
    assert np.all(rel(got["cost_log"], ref["cost_log"]) <= 1e-8)
    assert got["accepted"] == ref["accepted"]
    R, T, X, k = ref["state"]
    assert np.abs(got["T"] - T).max() < 1e-6
    assert np.abs(got["X"] - X).max() < 1e-5
