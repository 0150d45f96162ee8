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


@pytest.mark.gpu
@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_c_client_residual_on_the_gpu(tmp_path):
    """tests/c_client/gpu_residual_client.c (C11, HIP runtime API only) against
    the oracle: R of u = (x^2, x y) on the 6 x 5 unit square with zero loads."""
    import numpy as np

    import workloads as w
    from oracle import residual as ores

    exe = tmp_path / "gpu_client"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    os.path.join(ROOT, "tests", "c_client", "gpu_residual_client.c"), "-L", LIBDIR, "-lhofv",
                    "-L", "/opt/rocm/lib", "-lamdhip64", f"-Wl,-rpath,{LIBDIR}", "-Wl,-rpath,/opt/rocm/lib",
                    "-o", str(exe)], check=True)
    print("running", exe, flush=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    Rc = np.array([float(x) for x in r.stdout.split()]).reshape(2, -1).T
    mesh = w.box_mesh((6, 5))
    zero = lambda x, *a: np.zeros((np.atleast_2d(x).shape[0], 2))
    loads = w.fields.Loads(2, lambda xc, n: np.zeros(len(xc), int), zero, zero, zero)
    mu, lam = 0.3846153846153846, 0.5769230769230769
    prob = w.Problem("c_client", mesh, 2, 10, 2, w.LINEAR_ELASTIC, mu, lam, loads, stencil_quantum=1e-9)
    disc = ores.build(prob)
    u = np.stack([disc.cen[:, 0] ** 2, disc.cen[:, 0] * disc.cen[:, 1]], axis=1)
    Ro = ores.residual(disc, u)
    assert np.linalg.norm(Rc - Ro) <= 1e-10 * np.linalg.norm(Ro)
