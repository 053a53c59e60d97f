"""The allocation-free patch transfer (ba_patch_transfer_noalloc) against
ba_patch_transfer, through the C ABI: the same Eq. (3) transfers, bit for
bit, on two calls in a row (the second smaller, so the shared scratch holds
the first call's contents when it starts), and a call larger than the
scratch refused before anything runs.

The caller's device buffers come from hipMalloc of the HIP runtime the
library itself links (the caller, not the entry point, allocates them)."""
import ctypes as ct

import numpy as np
import pytest

from synth import geo as SG

pytestmark = pytest.mark.gpu

H2D, D2H = 1, 2


def hip():
    """The HIP runtime libba.so is linked against (the same instance): its
    symbols looked up through libba's own handle, which searches the
    libraries libba was loaded with.  (In a process that imported torch
    first, that is torch's copy of the runtime, not the one under /opt/rocm.)"""
    from paper_2511_06152_amd import ba
    lib = ba.load()
    h = ct.CDLL(ba.LIB_PATH)
    h.hipMalloc.argtypes = [ct.POINTER(ct.c_void_p), ct.c_size_t]
    h.hipFree.argtypes = [ct.c_void_p]
    h.hipMemcpy.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_int]
    h.hipDeviceSynchronize.argtypes = []
    return lib, h


class DevBuf:
    def __init__(self, h, host: np.ndarray):
        self.h, self.shape, self.dtype, self.nbytes = h, host.shape, host.dtype, host.nbytes
        self.p = ct.c_void_p()
        assert h.hipMalloc(ct.byref(self.p), max(self.nbytes, 256)) == 0
        self.put(host)

    def put(self, host):
        host = np.ascontiguousarray(host, self.dtype)
        assert h_ok(self.h.hipMemcpy(self.p, host.ctypes.data, self.nbytes, H2D))

    def get(self):
        out = np.empty(self.shape, self.dtype)
        assert h_ok(self.h.hipMemcpy(out.ctypes.data, self.p, self.nbytes, D2H))
        return out

    def free(self):
        self.h.hipFree(self.p)


def h_ok(rc):
    return rc == 0


def run_both(geo, h, g, cam, uv0, pairs):
    ref_uv, ref_fl, _ = geo.ba_patch_transfer(g["R"], g["T"], uv0, pairs, cam)
    n_img, n_patch, n_pairs = g["T"].shape[0], uv0.shape[0], len(pairs)
    bR, bT, bU = DevBuf(h, g["R"].reshape(n_img, 9)), DevBuf(h, g["T"]), DevBuf(h, uv0)
    buv = DevBuf(h, np.full((n_pairs, n_patch, 2), -7.0))
    bfl = DevBuf(h, np.full((n_pairs, n_patch), -7, np.int32))
    try:
        geo.ba_patch_transfer_noalloc(n_img, bR.p.value, bT.p.value, n_patch, bU.p.value, pairs, cam, buv.p.value,
                                      bfl.p.value)
        return ref_uv, ref_fl, buv.get(), bfl.get()
    finally:
        for b in (bR, bT, bU, buv, bfl):
            b.free()


def test_noalloc_transfer_equals_allocating_transfer():
    from paper_2511_06152_amd import Geo
    _, h = hip()
    g = SG.make_geo_flight(21, n_strips=2, imgs_per_strip=6)
    cam = {k: g[k] for k in ("f", "cx", "cy", "width", "height")}
    grid = SG.patch_grid()
    n = g["n_images"]
    with Geo(g["dsm"]) as geo:
        # first call: every ordered pair of neighbouring images and each image into itself, all 2120 patches
        pairs1 = [(a, b) for a in range(n) for b in range(n) if abs(a - b) <= 2]
        print("case no-alloc call 1:", len(pairs1), "pairs x", grid.shape[0], "patches", flush=True)
        r_uv, r_fl, uv, fl = run_both(geo, h, g, cam, grid, pairs1)
        assert np.array_equal(uv, r_uv, equal_nan=True) and np.array_equal(fl, r_fl)
        assert np.isfinite(uv).any() and (fl == 0).any()
        # second call, smaller: fewer sources, pairs and patches, in another order
        pairs2 = [(3, 1), (1, 3), (0, 0), (3, 4)]
        sub = np.ascontiguousarray(grid[::7])
        print("case no-alloc call 2:", len(pairs2), "pairs x", sub.shape[0], "patches", flush=True)
        r_uv, r_fl, uv, fl = run_both(geo, h, g, cam, sub, pairs2)
        assert np.array_equal(uv, r_uv, equal_nan=True) and np.array_equal(fl, r_fl)
        assert np.allclose(uv[2], sub, atol=1e-6)      # the identity pair returns the centres


def test_noalloc_transfer_refuses_more_than_its_scratch():
    """Four sources of 80 copies of the 2120-patch grid need 21.7 MB of
    ground points, more than the 16 MiB scratch: refused by the host before
    any device work (no device buffer is even read)."""
    from paper_2511_06152_amd import BAError, Geo
    _, h = hip()
    g = SG.make_geo_flight(21, n_strips=2, imgs_per_strip=2)
    cam = {k: g[k] for k in ("f", "cx", "cy", "width", "height")}
    uv0 = np.tile(SG.patch_grid(), (80, 1))
    n_img, n_patch = g["T"].shape[0], uv0.shape[0]
    pairs = [(a, a) for a in range(4)]
    bufs = [DevBuf(h, g["R"].reshape(n_img, 9)), DevBuf(h, g["T"]), DevBuf(h, uv0),
            DevBuf(h, np.zeros((4, n_patch, 2))), DevBuf(h, np.zeros((4, n_patch), np.int32))]
    try:
        with Geo(g["dsm"]) as geo:
            with pytest.raises(BAError) as e:
                geo.ba_patch_transfer_noalloc(n_img, bufs[0].p.value, bufs[1].p.value, n_patch, bufs[2].p.value,
                                              pairs, cam, bufs[3].p.value, bufs[4].p.value)
            assert e.value.code == -1 and "scratch" in str(e.value)
            assert np.array_equal(bufs[4].get(), np.zeros((4, n_patch), np.int32))   # nothing was written
    finally:
        for b in bufs:
            b.free()
