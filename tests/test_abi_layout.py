"""The ctypes structures of the Python binding have the size and field
offsets of the C structures in include/hofv.h (compiled here with gcc)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2601_18417_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [("hofv_params", L.Params), ("hofv_setup_report", L.SetupReport), ("hofv_krylov_opts", L.KrylovOpts),
         ("hofv_krylov_stats", L.KrylovStats), ("hofv_newton_opts", L.NewtonOpts),
         ("hofv_newton_stats", L.NewtonStats)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_structs_match_the_header(tmp_path):
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hofv.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:  # a trailing _ avoids a Python keyword (lambda_)
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field.rstrip("_")}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:-1]): int(line.split()[-1]) for line in out if line}
    for cname, cls in PAIRS:
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)
