"""Device memory from the caller's provider (ba_options.dev_alloc/dev_free):
with PyTorch's caching allocator every block of the context is a torch
allocation, all of them are returned at ba_destroy, and the results equal
those of a hipMalloc context bit for bit."""
import numpy as np
import pytest

from synth import aerial as A

pytestmark = pytest.mark.gpu


def run(allocator, sc, stream_cl):
    from paper_2511_06152_amd import BA_MIXED, Context
    with Context(precision=BA_MIXED, hbm_budget_bytes=256 << 20, max_slots=8, allocator=allocator) as ctx:
        held = sum(t.numel() for t in ctx.allocator.live.values()) if ctx.allocator else None
        t = ctx.submit(sc, max_iters=6)
        ctx.ba_step(t, 6)
        a = ctx.ba_fetch(t)
        ts = [ctx.submit(c, max_iters=4, use_resident=True, fuse_resident=True) for c in stream_cl]
        for x in ts:
            ctx.ba_step(x, 4)
        b = [ctx.ba_fetch(x) for x in ts]
        n_live = len(ctx.allocator.live) if ctx.allocator else None
        alloc = ctx.allocator
    return a, b, held, n_live, alloc


def test_torch_allocator_matches_hipmalloc():
    import torch
    sc = A.make_scene(A.spec_micro(n_strips=2, imgs_per_strip=3, n_points=800, k_true=(-0.05, 0.02), intr_mask=3), 9)
    stream_cl = A.make_stream(61, n_strips=2, imgs_per_strip=12, pts_per_image=300, max_cams=12,
                              min_cams=6)["clusters"][:3]
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    a, b, held, n_live, alloc = run("torch", sc, stream_cl)
    print("torch blocks held", held, "bytes; live blocks with the resident store", n_live, flush=True)
    assert held >= 256 << 20                      # the arena came from torch
    assert n_live > 0 and len(alloc.live) == 0    # the resident store too; everything returned at destroy
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == base
    ra, rb, _, _, _ = run(None, sc, stream_cl)
    for key in ("R", "T", "X", "k", "cost_log"):
        assert np.array_equal(a[key], ra[key]), key
        for g, r in zip(b, rb):
            assert np.array_equal(g[key], r[key]), key
