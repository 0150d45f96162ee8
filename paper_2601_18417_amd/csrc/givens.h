// Host-side least-squares update of (F)GMRES (Saad's algorithm with Givens
// rotations): the Arnoldi relation J Z_k = V_{k+1} H_k turns min ||beta e_1 - H y||
// into a triangular solve once each new Hessenberg column is rotated by the
// previous rotations and one new rotation zeroes its subdiagonal entry.
// Plain C++ (no HIP), so the rules below are unit-tested on the CPU.
#pragma once

#include <cmath>
#include <vector>

namespace hofv {

struct GivensLsq {
  int m = 0;                     // largest number of columns
  int k = 0;                     // columns accepted so far
  std::vector<double> H, cs, sn, g;  // H row-major [(m + 1) x m]; g: rotated right-hand side

  void reset(int m_, double beta) {
    m = m_;
    k = 0;
    H.assign((size_t)(m + 1) * m, 0.0);
    cs.assign(m, 1.0);
    sn.assign(m, 0.0);
    g.assign(m + 1, 0.0);
    g[0] = beta;
  }
  // Column j = k of H (entries 0..j+1 in col).  Returns false, accepting
  // nothing, when the rotated column is zero (hypot of its last two entries is
  // 0): the new basis direction adds nothing, and keeping it would leave a zero
  // on the diagonal of the triangular factor.
  bool add(const double* col) {
    const int j = k;
    std::vector<double> c(col, col + j + 2);
    for (int i = 0; i < j; ++i) {
      const double a = c[i], b = c[i + 1];
      c[i] = cs[i] * a + sn[i] * b;
      c[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double den = std::hypot(c[j], c[j + 1]);
    if (!(den > 0.0)) return false;
    cs[j] = c[j] / den;
    sn[j] = c[j + 1] / den;
    c[j] = den;
    c[j + 1] = 0.0;
    for (int i = 0; i <= j + 1; ++i) H[(size_t)i * m + j] = c[i];
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    ++k;
    return true;
  }
  // |g_k|: the least-squares residual norm after k accepted columns
  double residual() const { return std::fabs(g[k]); }
  // y[0..k) solving the k x k triangular system R y = g
  void solve(double* y) const {
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * m + l] * y[l];
      y[i] = s / H[(size_t)i * m + i];
    }
  }
};

}  // namespace hofv
