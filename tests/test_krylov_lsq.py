"""CPU tests of the host-side GMRES least-squares update (csrc/givens.h):
Givens rotations on Hessenberg columns against numpy's least squares, and the
rule for a column whose rotated form is zero (it is dropped, so the triangular
solve never divides by zero)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_18417_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "givens.h"
// stdin: m beta ncols, then ncols columns of m + 1 numbers (rows past j + 1 ignored)
// stdout: per column 1/0 (accepted), then k, the residual and y[0..k)
int main() {
  int m, nc;
  double beta;
  if (std::scanf("%d %lf %d", &m, &beta, &nc) != 3) return 1;
  hofv::GivensLsq lsq;
  lsq.reset(m, beta);
  std::vector<double> col(m + 1);
  for (int j = 0; j < nc; ++j) {
    for (int i = 0; i <= m; ++i) if (std::scanf("%lf", &col[i]) != 1) return 1;
    std::printf("%d\n", lsq.add(col.data()) ? 1 : 0);
  }
  std::vector<double> y(m, 0.0);
  lsq.solve(y.data());
  std::printf("%d %.17g\n", lsq.k, lsq.residual());
  for (int i = 0; i < lsq.k; ++i) std::printf("%.17g\n", y[i]);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not found")
    d = tmp_path_factory.mktemp("givens")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([cxx, "-O2", "-std=c++17", f"-I{CSRC}", str(src), "-o", str(exe)], check=True)
    return str(exe)


def run(exe, m, beta, cols):
    lines = [f"{m} {beta!r} {len(cols)}"] + [" ".join(repr(float(x)) for x in c) for c in cols]
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True).stdout
    vals = out.split()
    acc = [int(x) for x in vals[:len(cols)]]
    k = int(vals[len(cols)])
    res = float(vals[len(cols) + 1])
    y = np.array([float(x) for x in vals[len(cols) + 2:]])
    return acc, k, res, y


def hessenberg(rng, m, k):
    H = np.zeros((m + 1, k))
    for j in range(k):
        H[:j + 2, j] = rng.standard_normal(j + 2)
    return H


@pytest.mark.parametrize("k", [1, 3, 8])
def test_least_squares_matches_numpy(driver, k):
    rng = np.random.default_rng(k)
    m = 10
    H = hessenberg(rng, m, k)
    beta = 1.7
    acc, kk, res, y = run(driver, m, beta, [H[:, j] for j in range(k)])
    assert acc == [1] * k and kk == k
    rhs = np.zeros(k + 1)
    rhs[0] = beta
    yr, *_ = np.linalg.lstsq(H[:k + 1], rhs, rcond=None)
    assert np.allclose(y, yr, rtol=1e-12, atol=1e-13)
    assert res == pytest.approx(np.linalg.norm(rhs - H[:k + 1] @ yr), rel=1e-10, abs=1e-14)


def test_zero_column_is_dropped_and_the_solve_stays_finite(driver):
    """A Hessenberg column that is zero after the earlier rotations (here: all
    zero, as for z_j = 0) adds no direction: it is not accepted, k stays at the
    columns before it, and y is their least-squares solution."""
    rng = np.random.default_rng(3)
    m = 6
    H = hessenberg(rng, m, 2)
    zero = np.zeros(m + 1)
    acc, k, res, y = run(driver, m, 2.0, [H[:, 0], H[:, 1], zero])
    assert acc == [1, 1, 0] and k == 2
    assert np.all(np.isfinite(y))
    rhs = np.zeros(3)
    rhs[0] = 2.0
    yr, *_ = np.linalg.lstsq(H[:3, :2], rhs, rcond=None)
    assert np.allclose(y, yr, rtol=1e-12)


def test_column_in_the_span_after_rotation_is_dropped(driver):
    """Column 1 = (a, b, 0) with (a, b) parallel to column 0 = (a, b): after the
    first rotation its diagonal and subdiagonal entries are both zero."""
    a, b = 0.6, 0.8
    acc, k, res, y = run(driver, 4, 1.0, [[a, b, 0, 0, 0], [2 * a, 2 * b, 0.0, 0, 0]])
    assert acc == [1, 0] and k == 1
    assert np.all(np.isfinite(y)) and y[0] == pytest.approx(a)  # min |e_1 - (a, b) y| at y = a
    # a genuine lucky breakdown (zero subdiagonal, non-zero diagonal) is accepted
    acc, k, res, y = run(driver, 4, 1.0, [[a, 0.0, 0, 0, 0]])
    assert acc == [1] and k == 1 and res == 0.0 and y[0] == pytest.approx(1.0 / a)
