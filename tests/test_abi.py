"""The C-ABI library loads and exports every function include/ba.h declares
(CPU only: no compute call is made without a GPU)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ba.h")
LIB = os.path.join(ROOT, "paper_2511_06152_amd", "libba.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(ba_[a-z_]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["ba_create", "ba_destroy", "ba_submit_cluster", "ba_step", "ba_solve", "ba_solve_batch",
                 "ba_wait", "ba_fetch", "ba_release", "ba_footprint", "ba_profile_enable", "ba_profile_read",
                 "ba_strerror", "ba_last_error"]:
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
