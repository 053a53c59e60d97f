"""The Python binding's ctypes structures match the C header's layout: a
small C program built here with the host compiler prints sizeof and
offsetof of every field of every struct in include/*.h, and each must equal
what ctypes computes for the mirrored Structure (CPU only)."""
import ctypes as ct
import os
import shutil
import subprocess

import pytest

from paper_2511_06152_amd import ba

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [ba.ba_options, ba.ba_cluster, ba.ba_result, ba.ba_dsm, ba.ba_pinhole, ba.ba_cluster_rule]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_ctypes_layout_matches_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ba.h"', '#include "ba_geo.h"',
             'int main(void) {']
    for S in STRUCTS:
        n = S.__name__
        lines.append(f'  printf("{n} size %zu\\n", sizeof({n}));')
        for f, _ in S._fields_:
            cf = f[:-1] if f.endswith("_") else f      # a Python keyword gets a trailing underscore
            lines.append(f'  printf("{n} {f} %zu\\n", offsetof({n}, {cf}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    c_vals = {}
    for line in out:
        if line.strip():
            *key, v = line.split()
            c_vals[tuple(key)] = int(v)
    for S in STRUCTS:
        n = S.__name__
        assert c_vals[(n, "size")] == ct.sizeof(S), n
        for f, _ in S._fields_:
            assert c_vals[(n, f)] == getattr(S, f).offset, (n, f)
    # and the header has no field the binding leaves out: the last field ends the struct (up to padding)
    for S in STRUCTS:
        last, typ = S._fields_[-1]
        end = getattr(S, last).offset + ct.sizeof(typ)
        assert ct.sizeof(S) - end < 8, S.__name__
