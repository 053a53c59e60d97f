"""The C-ABI library loads and exports every function include/*.h declares
(CPU only: no compute call is made without a GPU)."""
import ctypes as ct
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
LIB = os.path.join(ROOT, "paper_2511_06152_amd", "libba.so")


def declared_functions():
    src = "\n".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(ba_[a-z_]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["ba_create", "ba_destroy", "ba_submit_cluster", "ba_step", "ba_solve", "ba_solve_batch",
                 "ba_wait", "ba_fetch", "ba_release", "ba_footprint", "ba_profile_enable", "ba_profile_read",
                 "ba_strerror", "ba_last_error", "ba_resident_poses", "ba_geo_create", "ba_geo_destroy",
                 "ba_footprints", "ba_footprint_overlaps", "ba_patch_transfer", "ba_geo_last_ms",
                 "ba_geo_last_error"]:
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libba.so not built")
def test_library_exports_every_declared_symbol():
    lib = ct.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libba.so not built")
def test_strerror_without_gpu():
    lib = ct.CDLL(LIB)
    lib.ba_strerror.restype = ct.c_char_p
    assert lib.ba_strerror(0) == b"ok"
    assert lib.ba_strerror(-2) == b"out of memory"


def test_binding_names_match_header():
    from paper_2511_06152_amd import ba
    assert sorted(ba.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libba.so not built")
def test_options_rejected_before_any_device_call():
    """Option checks come first, so they answer without a GPU: a negative
    count, an unknown precision, or only one of the two allocator hooks."""
    from paper_2511_06152_amd import ba
    lib = ba.load()

    def create(**kw):
        o = ba.ba_options(0, None, 1 << 20, 4, 16, ba.BA_FP64, 0, 2, 16, 4, 0, 500, 0.1, 0, 0, 0)
        for k, v in kw.items():
            setattr(o, k, v)
        h = ct.c_void_p()
        return lib.ba_create(ct.byref(o), ct.byref(h))

    assert create(max_slots=-1) == ba.BA_E_ARG
    assert create(precision=7) == ba.BA_E_ARG
    assert create(pcg_tol=-1.0) == ba.BA_E_ARG
    keep = ba.DEV_ALLOC(lambda n, u: None)
    assert create(dev_alloc=keep) == ba.BA_E_ARG
    keep2 = ba.DEV_FREE(lambda p, u: None)
    assert create(dev_free=keep2) == ba.BA_E_ARG
