"""The C ABI used from C: tests/c_client/host_only_client.c, compiled with gcc
(-std=c11 -Wall -Wextra -Werror) against include/hofv.h and linked to the
in-tree libhofv.so, runs the setup calls on a host-only context (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2601_18417_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.skipif(not os.path.exists(os.path.join(LIBDIR, "libhofv.so")), reason="libhofv.so not built")
def test_c_client_sets_up_a_host_only_context(tmp_path):
    exe = tmp_path / "client"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_client", "host_only_client.c"), "-L", LIBDIR, "-lhofv",
                    f"-Wl,-rpath,{LIBDIR}", "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    # 22 boundary edges with 2 points each, |S| = 6 + 10, 5 x 5 + 6 x 4 internal
    # edges, the first cell's centroid, and the refused hot call (HOFV_ESTATE)
    assert "boundary 22 nq 2 stencil 16 internal 49 centroid 0.083333 0.100000 hot -8" in r.stdout
