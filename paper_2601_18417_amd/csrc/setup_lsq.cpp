// Weighted least-squares Taylor reconstruction (paper Sec. 3.5.1, App. B).
//
// Rows of B are sqrt(w_N) q((x_N - x~)/h) with the scaled basis
// q_e(y) = prod_d y_d^{e_d} / e_d!, |e| <= p, h = 2 r_s, and w from the
// exponential weight function of shape k.  B = Q_h R by Householder
// reflections.  The fitted scaled coefficients are a~ = R^{-1} Q_h^T sqrt(W) u,
// so any linear functional t . a~ of the fit equals c . u with
//   c = sqrt(W) Q_h (R^{-T} t)
// which is what is evaluated for each requested target t: gradient rows at
// face quadrature points (t = e_{x_i} / h) and, at cell centroids, the
// extrapolation to a face centre minus the constant term (t_e = q_e(d / h) for
// |e| >= 1), i.e. d.grad u + 1/2 d^2 : grad grad u + 1/6 d^3 ::: grad^3 u.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace hofv {

int n_basis(int D, int p) {
  return D == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
}

void basis_exponents(int D, int p, int (*e)[3]) {
  int r = 0;
  for (int deg = 0; deg <= p; ++deg) {
    if (D == 2) {
      for (int a = deg; a >= 0; --a) { e[r][0] = a; e[r][1] = deg - a; e[r][2] = 0; ++r; }
    } else {
      for (int a = deg; a >= 0; --a)
        for (int b = deg - a; b >= 0; --b) { e[r][0] = a; e[r][1] = b; e[r][2] = deg - a - b; ++r; }
    }
  }
}

bool ls_functionals(int D, int p, double kshape, const double* xt, const double* X, int S,
                    double ghost_w, int kind, int n_targets, const double* targets, double* out,
                    double* cond, double* h_out) {
  const int nt = n_basis(D, p);
  const int m = S + (ghost_w > 0 ? 1 : 0);
  int ex[20][3];
  basis_exponents(D, p, ex);
  static const double inv_fact[4] = {1.0, 1.0, 0.5, 1.0 / 6.0};
  // distances and weights
  double dist[256], sw[256];
  double rs = 0.0;
  for (int i = 0; i < S; ++i) {
    double s = 0;
    for (int d = 0; d < D; ++d) {
      double t = X[i * D + d] - xt[d];
      s += t * t;
    }
    dist[i] = std::sqrt(s);
    rs = std::max(rs, dist[i]);
  }
  const double h = 2.0 * rs;
  const double ek = std::exp(-kshape * kshape);
  for (int i = 0; i < S; ++i) {
    double dt = dist[i] / h;
    double w = (std::exp(-dt * dt * kshape * kshape) - ek) / (1.0 - ek);
    sw[i] = std::sqrt(std::max(w, 0.0));
  }
  if (ghost_w > 0) sw[S] = std::sqrt(ghost_w);
  // B, column-major m x nt
  double B[256 * 20];
  for (int i = 0; i < S; ++i) {
    double y[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) y[d] = (X[i * D + d] - xt[d]) / h;
    for (int c = 0; c < nt; ++c) {
      double v = 1.0;
      for (int d = 0; d < D; ++d) {
        for (int k = 0; k < ex[c][d]; ++k) v *= y[d];
        v *= inv_fact[ex[c][d]];
      }
      B[c * m + i] = sw[i] * v;
    }
  }
  if (ghost_w > 0)
    for (int c = 0; c < nt; ++c) B[c * m + S] = c == 0 ? sw[S] : 0.0;
  // Householder QR: reflector j stored as v in B[j..m) of column j with v_j
  // kept in vhead[j]; R on and above the diagonal in rdiag / upper part.
  double rdiag[20], vhead[20], beta[20];
  for (int j = 0; j < nt; ++j) {
    double* col = &B[j * m];
    double nrm = 0;
    for (int i = j; i < m; ++i) nrm += col[i] * col[i];
    nrm = std::sqrt(nrm);
    double alpha = col[j] > 0 ? -nrm : nrm;
    double v0 = col[j] - alpha;
    double vtv = v0 * v0;
    for (int i = j + 1; i < m; ++i) vtv += col[i] * col[i];
    vhead[j] = v0;
    beta[j] = vtv > 0 ? 2.0 / vtv : 0.0;
    rdiag[j] = alpha;
    for (int c = j + 1; c < nt; ++c) {
      double* cc = &B[c * m];
      double s = v0 * cc[j];
      for (int i = j + 1; i < m; ++i) s += col[i] * cc[i];
      s *= beta[j];
      cc[j] -= s * v0;
      for (int i = j + 1; i < m; ++i) cc[i] -= s * col[i];
    }
  }
  double dmax = 0, dmin = INFINITY;
  for (int j = 0; j < nt; ++j) {
    dmax = std::max(dmax, std::fabs(rdiag[j]));
    dmin = std::min(dmin, std::fabs(rdiag[j]));
  }
  *cond = dmin > 0 ? dmax / dmin : INFINITY;
  if (h_out) *h_out = h;
  if (!(dmin > 1e-14 * dmax)) return false;
  auto R = [&](int i, int j) { return i == j ? rdiag[i] : B[j * m + i]; };  // i < j above diagonal
  for (int r = 0; r < n_targets; ++r) {
    double t[20];
    if (kind == kTargetGradient) {
      // targets[r] = axis i: physical d/dx_i is row e_i of the scaled fit / h
      const int axis = (int)targets[r];
      for (int c = 0; c < nt; ++c)
        t[c] = (ex[c][0] + ex[c][1] + ex[c][2] == 1 && ex[c][axis] == 1) ? 1.0 / h : 0.0;
    } else {
      // targets[r] = displacement d (D values): sum_{|e|>=1} q_e(d/h) a~_e
      const double* d = targets + (size_t)r * D;
      for (int c = 0; c < nt; ++c) {
        double v = (c == 0) ? 0.0 : 1.0;
        for (int a = 0; a < D && c > 0; ++a) {
          for (int k = 0; k < ex[c][a]; ++k) v *= d[a] / h;
          v *= inv_fact[ex[c][a]];
        }
        t[c] = v;
      }
    }
    double y[20];
    for (int i = 0; i < nt; ++i) {  // R^T y = t (forward)
      double s = t[i];
      for (int k = 0; k < i; ++k) s -= R(k, i) * y[k];
      y[i] = s / rdiag[i];
    }
    double z[256];
    for (int i = 0; i < m; ++i) z[i] = i < nt ? y[i] : 0.0;
    for (int j = nt - 1; j >= 0; --j) {  // z = H_0 ... H_{nt-1} [y; 0]
      const double* col = &B[j * m];
      double s = vhead[j] * z[j];
      for (int i = j + 1; i < m; ++i) s += col[i] * z[i];
      s *= beta[j];
      z[j] -= s * vhead[j];
      for (int i = j + 1; i < m; ++i) z[i] -= s * col[i];
    }
    double* o = out + (size_t)r * m;
    for (int i = 0; i < m; ++i) o[i] = sw[i] * z[i];
  }
  return true;
}

}  // namespace hofv
