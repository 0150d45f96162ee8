// Mesh topology and geometry for straight-edged quads and triangles, trilinear
// hexahedra and tetrahedra (paper Sec. 3.1): face matching, owner/neighbour, outward unit
// normals and areas from the exact vector area of each (bi)linear or flat
// face, face and cell quadrature, cell volumes and centroids.  Triangles and
// tetrahedra take conical-product rules (Gauss-Jacobi nodes along the
// collapsed directions, Gauss-Legendre along the last), generated here in
// place of the paper's tabulated symmetric rules; with n points per direction
// they are exact for polynomials of total degree 2n - 1.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

#include "common.h"

namespace hofv {

namespace {

// library-local face tables: vertex cycles whose right-hand normal points out
const int kQuadFace[4][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
const int kTriFace[3][2] = {{0, 1}, {1, 2}, {2, 0}};  // counter-clockwise triangle
const int kHexFace[6][4] = {{0, 3, 2, 1}, {4, 5, 6, 7}, {0, 1, 5, 4},
                            {3, 7, 6, 2}, {0, 4, 7, 3}, {1, 2, 6, 5}};
// tetrahedron with (x1 - x0) x (x2 - x0) . (x3 - x0) > 0
const int kTetFace[4][3] = {{0, 2, 1}, {0, 1, 3}, {1, 2, 3}, {0, 3, 2}};

// Gauss-Jacobi rule for the weight u^beta on [0,1] (weights sum to
// 1 / (beta + 1)): the nodes are the eigenvalues of the Jacobi matrix of the
// monic orthogonal polynomials (the alpha = 0 Jacobi recurrence mapped from
// [-1,1]), found by Sturm-sequence bisection; the weights are the Christoffel
// numbers 1 / sum_k phat_k(x)^2 of the orthonormal polynomials.
void gauss_jacobi01(int n, int beta, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> a(n), b(n, 0.0);  // b[k]: off-diagonal squared between k-1 and k
  for (int k = 0; k < n; ++k) {
    const double t = 2.0 * k + beta;
    a[k] = 0.5 * ((double)beta * beta / (t * (t + 2.0)) + 1.0);
    if (k > 0) b[k] = 0.25 * 4.0 * k * k * (k + beta) * (k + beta) / (t * t * (t + 1.0) * (t - 1.0));
  }
  auto below = [&](double y) {  // eigenvalues < y
    int cnt = 0;
    double q = a[0] - y;
    if (q < 0) ++cnt;
    for (int k = 1; k < n; ++k) {
      if (q == 0.0) q = 1e-300;
      q = (a[k] - y) - b[k] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double mu0 = 1.0 / (beta + 1.0);
  for (int i = 0; i < n; ++i) {
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200 && hi - lo > 1e-17; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (below(mid) > i) hi = mid;
      else lo = mid;
    }
    x[i] = 0.5 * (lo + hi);
    double p0 = 1.0 / std::sqrt(mu0), pm = 0.0, s = p0 * p0;
    for (int k = 0; k + 1 < n; ++k) {
      const double pk = ((x[i] - a[k]) * p0 - (k > 0 ? std::sqrt(b[k]) * pm : 0.0)) / std::sqrt(b[k + 1]);
      pm = p0;
      p0 = pk;
      s += p0 * p0;
    }
    w[i] = 1.0 / s;
  }
}

// Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_n.
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double t = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = t; p0 = 1.0; }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = (n == 1) ? 1.0 : n * (t * p1 - p0) / (t * t - 1.0);
    }
    x[n - 1 - i] = 0.5 * (t + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);  // = (2/((1-t^2)P'^2)) / 2
  }
}

inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// trilinear hex map at reference point (r,s,t) in [0,1]^3: position and Jacobian determinant
void hex_map(const double* X /*8x3*/, double r, double s, double t, double* x, double* detJ) {
  // vertex reference coordinates in VTK order
  static const int ref[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                                {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
  double J[3][3] = {{0}};
  x[0] = x[1] = x[2] = 0.0;
  for (int a = 0; a < 8; ++a) {
    double fr = ref[a][0] ? r : 1 - r, gr = ref[a][0] ? 1.0 : -1.0;
    double fs = ref[a][1] ? s : 1 - s, gs = ref[a][1] ? 1.0 : -1.0;
    double ft = ref[a][2] ? t : 1 - t, gt = ref[a][2] ? 1.0 : -1.0;
    double N = fr * fs * ft;
    double dN[3] = {gr * fs * ft, fr * gs * ft, fr * fs * gt};
    for (int i = 0; i < 3; ++i) {
      x[i] += N * X[3 * a + i];
      for (int j = 0; j < 3; ++j) J[i][j] += X[3 * a + i] * dN[j];
    }
  }
  *detJ = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
          J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

void quad_map(const double* X /*4x2*/, double r, double s, double* x, double* detJ) {
  double N[4] = {(1 - r) * (1 - s), r * (1 - s), r * s, (1 - r) * s};
  double dr[4] = {-(1 - s), (1 - s), s, -s};
  double ds[4] = {-(1 - r), -r, r, (1 - r)};
  double J[2][2] = {{0}};
  x[0] = x[1] = 0;
  for (int a = 0; a < 4; ++a) {
    x[0] += N[a] * X[2 * a];
    x[1] += N[a] * X[2 * a + 1];
    J[0][0] += X[2 * a] * dr[a];
    J[0][1] += X[2 * a] * ds[a];
    J[1][0] += X[2 * a + 1] * dr[a];
    J[1][1] += X[2 * a + 1] * ds[a];
  }
  *detJ = J[0][0] * J[1][1] - J[0][1] * J[1][0];
}

}  // namespace

hofv_status build_topology(hofv_ctx* c) {
  const int D = c->D;
  const bool simplex = c->cells.size() == (size_t)c->nc * (D + 1);
  const int ncv = simplex ? D + 1 : (D == 2 ? 4 : 8), nlf = simplex ? D + 1 : 2 * D, nfv = D == 2 ? 2 : (simplex ? 3 : 4);
  auto lface = [&](int sl, int k) {
    if (D == 2) return simplex ? kTriFace[sl][k] : kQuadFace[sl][k];
    return simplex ? kTetFace[sl][k] : kHexFace[sl][k];
  };
  struct Rec {
    std::array<int64_t, 4> key;
    int64_t cell;
    int32_t slot;
  };
  std::vector<Rec> recs((size_t)c->nc * nlf);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < c->nc; ++e) {
    const int64_t* cv = &c->cells[(size_t)e * ncv];
    for (int s = 0; s < nlf; ++s) {
      Rec& r = recs[(size_t)e * nlf + s];
      r.key = {-1, -1, -1, -1};
      for (int k = 0; k < nfv; ++k) r.key[k] = cv[lface(s, k)];
      std::sort(r.key.begin(), r.key.begin() + nfv);
      r.cell = e;
      r.slot = s;
    }
  }
  std::sort(recs.begin(), recs.end(), [](const Rec& a, const Rec& b) {
    if (a.key != b.key) return a.key < b.key;
    return a.cell < b.cell;
  });
  std::vector<hofv_ctx::Face> inner, bnd;
  inner.reserve(recs.size() / 2);
  for (size_t i = 0; i < recs.size();) {
    size_t j = i + 1;
    while (j < recs.size() && recs[j].key == recs[i].key) ++j;
    if (j - i > 2) return fail(c, HOFV_EINVAL, "non-manifold mesh: a face is shared by more than two cells");
    hofv_ctx::Face f{};
    f.own = recs[i].cell;
    f.sown = recs[i].slot;
    const int64_t* cv = &c->cells[(size_t)f.own * ncv];
    for (int k = 0; k < 4; ++k) f.v[k] = k < nfv ? cv[lface(f.sown, k)] : -1;
    if (j - i == 2) {
      f.nei = recs[i + 1].cell;
      f.snei = recs[i + 1].slot;
      if (f.nei == f.own) return fail(c, HOFV_EINVAL, "degenerate cell: repeated face");
      inner.push_back(f);
    } else {
      f.nei = -1;
      f.snei = -1;
      bnd.push_back(f);
    }
    i = j;
  }
  auto by_owner = [](const hofv_ctx::Face& a, const hofv_ctx::Face& b) {
    return a.own != b.own ? a.own < b.own : a.sown < b.sown;
  };
  std::sort(inner.begin(), inner.end(), by_owner);
  std::sort(bnd.begin(), bnd.end(), by_owner);
  c->n_internal = (int64_t)inner.size();
  c->faces = std::move(inner);
  c->faces.insert(c->faces.end(), bnd.begin(), bnd.end());
  c->bface.resize(bnd.size());
  std::iota(c->bface.begin(), c->bface.end(), c->n_internal);
  c->NS = 2 * D;  // simplices fill D + 1 of them
  return HOFV_OK;
}

// Face-list mesh: face f has the vertex loop face_verts[face_ptr[f] ..
// face_ptr[f + 1]) whose right-hand normal points out of face_cells[2 f] and
// into face_cells[2 f + 1] (-1: boundary).  The owner becomes the lower cell
// id (its loop reversed when that swaps the sides); slots number each cell's
// faces in input order.
hofv_status build_topology_poly(hofv_ctx* c, int64_t n_faces, const int64_t* face_ptr, const int64_t* face_verts,
                                const int64_t* face_cells) {
  const int D = c->D;
  const int64_t nc = c->nc;
  if (face_ptr[0] != 0) return fail(c, HOFV_EINVAL, "face_ptr[0] must be 0");
  std::vector<int32_t> nslot(nc, 0);
  struct Rec {
    hofv_ctx::Face f;
    int64_t src;  // input face
    bool flip;
  };
  std::vector<Rec> inner, bnd;
  for (int64_t f = 0; f < n_faces; ++f) {
    const int64_t m = face_ptr[f + 1] - face_ptr[f];
    if (D == 2 ? m != 2 : m < 3) return fail(c, HOFV_EINVAL, "a face needs 2 vertices in 2D, at least 3 in 3D");
    for (int64_t k = face_ptr[f]; k < face_ptr[f + 1]; ++k)
      if (face_verts[k] < 0 || face_verts[k] >= c->nv) return fail(c, HOFV_EINVAL, "face vertex index out of range");
    int64_t a = face_cells[2 * f], b = face_cells[2 * f + 1];
    if (a < 0 || a >= nc || b < -1 || b >= nc || a == b) return fail(c, HOFV_EINVAL, "bad face cells");
    Rec r{};
    r.src = f;
    r.flip = b >= 0 && b < a;
    r.f.own = r.flip ? b : a;
    r.f.nei = r.flip ? a : b;
    r.f.sown = nslot[r.f.own]++;
    r.f.snei = r.f.nei >= 0 ? nslot[r.f.nei]++ : -1;
    for (int k = 0; k < 4; ++k) r.f.v[k] = -1;
    (b >= 0 ? inner : bnd).push_back(r);
  }
  int ns = 0;
  for (int64_t P = 0; P < nc; ++P) {
    if (nslot[P] < D + 1) return fail(c, HOFV_EINVAL, "a cell has fewer than dim + 1 faces");
    ns = std::max(ns, nslot[P]);
  }
  if (ns > 255) return fail(c, HOFV_EINVAL, "a cell has more than 255 faces");
  auto by_owner = [](const Rec& x, const Rec& y) {
    return x.f.own != y.f.own ? x.f.own < y.f.own : x.f.sown < y.f.sown;
  };
  std::sort(inner.begin(), inner.end(), by_owner);
  std::sort(bnd.begin(), bnd.end(), by_owner);
  c->poly = true;
  c->NS = std::max(ns, 2 * D);  // cells with fewer faces leave slots empty, as simplices do
  c->n_internal = (int64_t)inner.size();
  c->faces.clear();
  c->fv_ptr.assign(1, 0);
  c->fv.clear();
  for (const std::vector<Rec>* part : {&inner, &bnd})
    for (const Rec& r : *part) {
      hofv_ctx::Face F = r.f;
      const int64_t b0 = face_ptr[r.src], e0 = face_ptr[r.src + 1];
      for (int64_t k = 0; k < e0 - b0; ++k) c->fv.push_back(face_verts[r.flip ? e0 - 1 - k : b0 + k]);
      c->fv_ptr.push_back((int64_t)c->fv.size());
      if (D == 2) {  // edges keep using the 2D face path
        F.v[0] = c->fv[c->fv.size() - 2];
        F.v[1] = c->fv[c->fv.size() - 1];
      }
      c->faces.push_back(F);
    }
  c->bface.resize(bnd.size());
  std::iota(c->bface.begin(), c->bface.end(), c->n_internal);
  return HOFV_OK;
}

hofv_status build_geometry(hofv_ctx* c) {
  const int D = c->D, p = c->prm.order_p, ng = c->prm.n_gauss;
  const int64_t nc = c->nc;
  const bool simplex = c->cells.size() == (size_t)nc * (D + 1), tet = simplex && D == 3;
  const int ncv = simplex ? D + 1 : (D == 2 ? 4 : 8);
  c->cen.assign((size_t)nc * D, 0.0);
  c->vol.assign(nc, 0.0);
  std::vector<double> g2x, g2w, gvx, gvw, gfx, gfw;
  gauss_legendre01(2, g2x, g2w);
  gauss_legendre01(p + 2, gvx, gvw);
  gauss_legendre01(ng, gfx, gfw);
  std::vector<double> j1x, j1w, j2x, j2w, t1x, t1w;  // Gauss-Jacobi u^2, u (cells); u (faces)
  gauss_jacobi01(p + 2, 2, j2x, j2w);
  gauss_jacobi01(p + 2, 1, j1x, j1w);
  gauss_jacobi01(ng, 1, t1x, t1w);
  const int nv1 = p + 2;
  bool bad = false;
  if (c->poly) {
    // Cells cut into triangles (2D) or tetrahedra (3D) joining the mean x_a of
    // the cell's distinct vertices to each face's edge or fan triangles,
    // oriented outward (the neighbour side takes the reversed loop); volume and
    // centroid are their sums, the body force takes the simplex rule with
    // p + 2 points per direction on each.
    const int npts = D == 2 ? nv1 * nv1 : nv1 * nv1 * nv1;
    std::vector<std::vector<std::pair<int64_t, int>>> side(nc);  // (face, 0 owner | 1 neighbour)
    std::vector<int64_t> nsimp(nc, 0);
    for (int64_t f = 0; f < (int64_t)c->faces.size(); ++f) {
      const hofv_ctx::Face& F = c->faces[f];
      const int64_t t = D == 2 ? 1 : c->fv_ptr[f + 1] - c->fv_ptr[f] - 2;
      side[F.own].push_back({f, 0});
      nsimp[F.own] += t;
      if (F.nei >= 0) {
        side[F.nei].push_back({f, 1});
        nsimp[F.nei] += t;
      }
    }
    c->vq_ptr.assign(nc + 1, 0);
    for (int64_t e = 0; e < nc; ++e) c->vq_ptr[e + 1] = c->vq_ptr[e] + nsimp[e] * npts;
    c->nqv = 0;
    for (int64_t e = 0; e < nc; ++e) c->nqv = std::max<int64_t>(c->nqv, nsimp[e] * npts);
    c->vq_pts.assign((size_t)c->vq_ptr[nc] * D, 0.0);
    c->vq_w.assign((size_t)c->vq_ptr[nc], 0.0);
    bool open = false;
#pragma omp parallel for schedule(dynamic, 64) reduction(|| : bad, open)
    for (int64_t e = 0; e < nc; ++e) {
      std::vector<int64_t> vs;
      for (auto& [f, sd] : side[e])
        for (int64_t k = c->fv_ptr[f]; k < c->fv_ptr[f + 1]; ++k) vs.push_back(c->fv[k]);
      std::sort(vs.begin(), vs.end());
      vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
      double apex[3] = {0, 0, 0};
      for (int64_t v : vs)
        for (int d = 0; d < D; ++d) apex[d] += c->verts[(size_t)v * D + d];
      for (int d = 0; d < D; ++d) apex[d] /= (double)vs.size();
      double V = 0, mom[3] = {0, 0, 0};
      int64_t q = c->vq_ptr[e];
      auto add_simplex = [&](const double* const* X) {  // X[0] = apex, then the oriented face part
        if (D == 2) {
          const double e1[2] = {X[1][0] - X[0][0], X[1][1] - X[0][1]}, e2[2] = {X[2][0] - X[0][0], X[2][1] - X[0][1]};
          const double det = e1[0] * e2[1] - e1[1] * e2[0];
          V += 0.5 * det;
          for (int d = 0; d < 2; ++d) mom[d] += 0.5 * det * (X[0][d] + X[1][d] + X[2][d]) / 3.0;
          for (int i = 0; i < nv1; ++i)
            for (int j = 0; j < nv1; ++j, ++q) {
              const double a = j1x[i], b = gvx[j];
              for (int d = 0; d < 2; ++d)
                c->vq_pts[(size_t)q * 2 + d] = X[0][d] + a * (X[1][d] - X[0][d] + b * (X[2][d] - X[1][d]));
              c->vq_w[q] = j1w[i] * gvw[j] * det;
            }
          return;
        }
        double e1[3], e2[3], e3[3], f2[3], f3[3], cr[3];
        for (int d = 0; d < 3; ++d) {
          e1[d] = X[1][d] - X[0][d];
          e2[d] = X[2][d] - X[1][d];
          e3[d] = X[3][d] - X[2][d];
          f2[d] = X[2][d] - X[0][d];
          f3[d] = X[3][d] - X[0][d];
        }
        cross3(e1, f2, cr);
        const double det = cr[0] * f3[0] + cr[1] * f3[1] + cr[2] * f3[2];
        V += det / 6.0;
        for (int d = 0; d < 3; ++d) mom[d] += det / 6.0 * 0.25 * (X[0][d] + X[1][d] + X[2][d] + X[3][d]);
        for (int i = 0; i < nv1; ++i)
          for (int j = 0; j < nv1; ++j)
            for (int k = 0; k < nv1; ++k, ++q) {
              const double a = j2x[i], b = j1x[j], cc = gvx[k];
              for (int d = 0; d < 3; ++d) c->vq_pts[(size_t)q * 3 + d] = X[0][d] + a * (e1[d] + b * (e2[d] + cc * e3[d]));
              c->vq_w[q] = j2w[i] * j1w[j] * gvw[k] * det;
            }
      };
      // the faces must close: their outward vector areas (1/2 sum (x_k - a) x
      // (x_k+1 - a) per loop, the rotated edge in 2D) sum to zero for any
      // polygonal surface, warped or not
      double Ssum[3] = {0, 0, 0}, Aabs = 0;
      for (auto& [f, sd] : side[e]) {
        const int64_t b0 = c->fv_ptr[f], m = c->fv_ptr[f + 1] - b0;
        std::vector<int64_t> L(m);
        for (int64_t k = 0; k < m; ++k) L[k] = c->fv[sd ? b0 + m - 1 - k : b0 + k];
        double Sf[3] = {0, 0, 0};
        if (D == 2) {
          Sf[0] = c->verts[(size_t)L[1] * 2 + 1] - c->verts[(size_t)L[0] * 2 + 1];
          Sf[1] = -(c->verts[(size_t)L[1] * 2] - c->verts[(size_t)L[0] * 2]);
        } else {
          for (int64_t k = 0; k < m; ++k) {
            double r0[3], r1[3], cr[3];
            for (int d = 0; d < 3; ++d) {
              r0[d] = c->verts[(size_t)L[k] * 3 + d] - apex[d];
              r1[d] = c->verts[(size_t)L[(k + 1) % m] * 3 + d] - apex[d];
            }
            cross3(r0, r1, cr);
            for (int d = 0; d < 3; ++d) Sf[d] += 0.5 * cr[d];
          }
        }
        for (int d = 0; d < D; ++d) Ssum[d] += Sf[d];
        Aabs += std::sqrt(Sf[0] * Sf[0] + Sf[1] * Sf[1] + Sf[2] * Sf[2]);
        if (D == 2) {
          const double* X[3] = {apex, &c->verts[(size_t)L[0] * 2], &c->verts[(size_t)L[1] * 2]};
          add_simplex(X);
          continue;
        }
        int64_t s0 = 0;
        for (int64_t k = 1; k < m; ++k)
          if (L[k] < L[s0]) s0 = k;
        for (int64_t k = 1; k + 1 < m; ++k) {  // fan triangles (y0, yk, yk+1) from the lowest vertex
          const double* X[4] = {apex, &c->verts[(size_t)L[s0] * 3], &c->verts[(size_t)L[(s0 + k) % m] * 3],
                                &c->verts[(size_t)L[(s0 + k + 1) % m] * 3]};
          add_simplex(X);
        }
      }
      c->vol[e] = V;
      for (int d = 0; d < D; ++d) c->cen[(size_t)e * D + d] = mom[d] / V;
      if (!(V > 0)) bad = true;
      if (!(std::sqrt(Ssum[0] * Ssum[0] + Ssum[1] * Ssum[1] + Ssum[2] * Ssum[2]) <= 1e-9 * Aabs)) open = true;
    }
    if (open)
      return fail(c, HOFV_EINVAL,
                  "the faces of a cell do not close (a missing or repeated face, or a loop whose normal points "
                  "into its first cell)");
  } else {
  c->nqv = D == 2 ? nv1 * nv1 : nv1 * nv1 * nv1;
  c->vq_ptr.resize(nc + 1);
  for (int64_t e = 0; e <= nc; ++e) c->vq_ptr[e] = e * c->nqv;
  c->vq_pts.assign((size_t)nc * c->nqv * D, 0.0);
  c->vq_w.assign((size_t)nc * c->nqv, 0.0);
#pragma omp parallel for schedule(static) reduction(|| : bad)
  for (int64_t e = 0; e < nc; ++e) {
    double X[24];
    for (int a = 0; a < ncv; ++a)
      for (int d = 0; d < D; ++d) X[D * a + d] = c->verts[(size_t)c->cells[(size_t)e * ncv + a] * D + d];
    if (D == 2) {
      // polygon (shoelace) area and centroid of the straight-edged quad or
      // triangle, in coordinates relative to its first vertex: with absolute
      // ones the cross products, of size |x|^2, cancel down to the area, of
      // size h^2, and the centroid loses (|x| / h)^2 of its precision
      double A2 = 0, cx = 0, cy = 0;
      for (int a = 0; a < ncv; ++a) {
        const int b = (a + 1) % ncv;
        const double xa = X[2 * a] - X[0], ya = X[2 * a + 1] - X[1];
        const double xb = X[2 * b] - X[0], yb = X[2 * b + 1] - X[1];
        const double cr = xa * yb - xb * ya;
        A2 += cr;
        cx += (xa + xb) * cr;
        cy += (ya + yb) * cr;
      }
      c->vol[e] = 0.5 * A2;
      c->cen[2 * e] = X[0] + cx / (3.0 * A2);
      c->cen[2 * e + 1] = X[1] + cy / (3.0 * A2);
      int q = 0;
      for (int i = 0; i < nv1; ++i)
        for (int j = 0; j < nv1; ++j, ++q) {
          double* xq = &c->vq_pts[((size_t)e * c->nqv + q) * 2];
          if (simplex) {  // x0 + a (x1 - x0 + b (x2 - x1)), detJ = 2 Omega a
            const double a = j1x[i], b = gvx[j];
            for (int d = 0; d < 2; ++d) xq[d] = X[d] + a * (X[2 + d] - X[d] + b * (X[4 + d] - X[2 + d]));
            c->vq_w[(size_t)e * c->nqv + q] = j1w[i] * gvw[j] * A2;
          } else {
            double dj;
            quad_map(X, gvx[i], gvx[j], xq, &dj);
            c->vq_w[(size_t)e * c->nqv + q] = gvw[i] * gvw[j] * dj;
          }
        }
    } else if (tet) {
      // flat tetrahedron: Omega = det / 6, centroid = vertex mean; the volume
      // rule maps (a, b, c) in [0,1]^3 to x0 + a (e1 + b (e2 + c e3)),
      // e1 = x1 - x0, e2 = x2 - x1, e3 = x3 - x2, with det = 6 Omega a^2 b
      double e1[3], e2[3], e3[3], f2[3], f3[3], cr[3];
      for (int d = 0; d < 3; ++d) {
        e1[d] = X[3 + d] - X[d];
        e2[d] = X[6 + d] - X[3 + d];
        e3[d] = X[9 + d] - X[6 + d];
        f2[d] = X[6 + d] - X[d];
        f3[d] = X[9 + d] - X[d];
      }
      cross3(e1, f2, cr);
      const double det = cr[0] * f3[0] + cr[1] * f3[1] + cr[2] * f3[2];
      c->vol[e] = det / 6.0;
      for (int d = 0; d < 3; ++d) c->cen[3 * e + d] = 0.25 * (X[d] + X[3 + d] + X[6 + d] + X[9 + d]);
      int q = 0;
      for (int i = 0; i < nv1; ++i)
        for (int j = 0; j < nv1; ++j)
          for (int k = 0; k < nv1; ++k, ++q) {
            const double a = j2x[i], b = j1x[j], cc = gvx[k];
            for (int d = 0; d < 3; ++d)
              c->vq_pts[((size_t)e * c->nqv + q) * 3 + d] = X[d] + a * (e1[d] + b * (e2[d] + cc * e3[d]));
            c->vq_w[(size_t)e * c->nqv + q] = j2w[i] * j1w[j] * gvw[k] * det;
          }
    } else {
      double V = 0, m[3] = {0, 0, 0};
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int k = 0; k < 2; ++k) {
            double x[3], dj;
            hex_map(X, g2x[i], g2x[j], g2x[k], x, &dj);
            double wq = g2w[i] * g2w[j] * g2w[k] * dj;
            V += wq;
            for (int d = 0; d < 3; ++d) m[d] += wq * x[d];
          }
      c->vol[e] = V;
      for (int d = 0; d < 3; ++d) c->cen[3 * e + d] = m[d] / V;
      int q = 0;
      for (int i = 0; i < nv1; ++i)
        for (int j = 0; j < nv1; ++j)
          for (int k = 0; k < nv1; ++k, ++q) {
            double x[3], dj;
            hex_map(X, gvx[i], gvx[j], gvx[k], x, &dj);
            for (int d = 0; d < 3; ++d) c->vq_pts[((size_t)e * c->nqv + q) * 3 + d] = x[d];
            c->vq_w[(size_t)e * c->nqv + q] = gvw[i] * gvw[j] * gvw[k] * dj;
          }
    }
    if (!(c->vol[e] > 0)) bad = true;
  }
  }
  if (bad) return fail(c, HOFV_EINVAL, "a cell has non-positive volume (check vertex order)");

  // faces
  const int64_t nf = (int64_t)c->faces.size();
  const bool fan = D == 3 && !simplex && c->prm.face_rule == 1;
  c->nq = D == 2 ? ng : (fan ? 2 * ng * ng : ng * ng);
  if (c->poly && D == 3) {  // polygons: the fan's triangles, padded to the largest count
    int64_t mmax = 3;
    for (int64_t f = 0; f < nf; ++f) mmax = std::max<int64_t>(mmax, c->fv_ptr[f + 1] - c->fv_ptr[f]);
    c->nq = (int)((mmax - 2) * ng * ng);
  }
  const int nq = c->nq;
  c->f_centre.assign((size_t)nf * D, 0.0);
  c->f_normal.assign((size_t)nf * D, 0.0);
  c->f_area.assign(nf, 0.0);
  c->f_qp.assign((size_t)nf * nq * D, 0.0);
  c->f_qw.assign((size_t)nf * nq, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t f = 0; f < nf; ++f) {
    const hofv_ctx::Face& F = c->faces[f];
    double* qp = &c->f_qp[(size_t)f * nq * D];
    double* qw = &c->f_qw[(size_t)f * nq];
    if (c->poly && D == 3) {
      // polygon of m vertices: vector area 1/2 sum x_k x x_{k+1} gives the
      // normal; a fan from the lowest vertex gives m - 2 triangles, each with
      // the triangle rule and its share A_t / sum A of the weight; Gamma_f is
      // the sum of the triangle areas; unused points sit at the centre with
      // zero weight
      const int64_t b0 = c->fv_ptr[f], m = c->fv_ptr[f + 1] - b0;
      double Sv[3] = {0, 0, 0};
      for (int64_t k = 0; k < m; ++k) {
        double cr[3];
        cross3(&c->verts[(size_t)c->fv[b0 + k] * 3], &c->verts[(size_t)c->fv[b0 + (k + 1) % m] * 3], cr);
        for (int d = 0; d < 3; ++d) Sv[d] += 0.5 * cr[d];
      }
      const double Sn = std::sqrt(Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2]);
      for (int d = 0; d < 3; ++d) c->f_normal[3 * f + d] = Sv[d] / Sn;
      int64_t s0 = 0;
      for (int64_t k = 1; k < m; ++k)
        if (c->fv[b0 + k] < c->fv[b0 + s0]) s0 = k;
      auto vx = [&](int64_t k) { return &c->verts[(size_t)c->fv[b0 + (s0 + k) % m] * 3]; };
      std::vector<double> At(m - 2);
      double Asum = 0;
      for (int64_t t = 0; t + 2 < m; ++t) {
        double u1[3], u2[3], cr[3];
        for (int d = 0; d < 3; ++d) {
          u1[d] = vx(t + 1)[d] - vx(0)[d];
          u2[d] = vx(t + 2)[d] - vx(0)[d];
        }
        cross3(u1, u2, cr);
        At[t] = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        Asum += At[t];
      }
      c->f_area[f] = Asum;
      int q = 0;
      for (int64_t t = 0; t + 2 < m; ++t)
        for (int i = 0; i < ng; ++i)
          for (int j = 0; j < ng; ++j, ++q) {
            const double a = t1x[i], b = gfx[j];
            const double *x0 = vx(0), *x1 = vx(t + 1), *x2 = vx(t + 2);
            for (int d = 0; d < 3; ++d) qp[3 * q + d] = x0[d] + a * (x1[d] - x0[d] + b * (x2[d] - x1[d]));
            qw[q] = 2.0 * t1w[i] * gfw[j] * At[t] / Asum;
          }
      double xc[3] = {0, 0, 0};
      for (int k = 0; k < q; ++k)
        for (int d = 0; d < 3; ++d) xc[d] += qw[k] * qp[3 * k + d];
      for (; q < nq; ++q) {
        for (int d = 0; d < 3; ++d) qp[3 * q + d] = xc[d];
        qw[q] = 0.0;
      }
    } else if (D == 2) {
      const double* a = &c->verts[(size_t)F.v[0] * 2];
      const double* b = &c->verts[(size_t)F.v[1] * 2];
      double ex = b[0] - a[0], ey = b[1] - a[1];
      double L = std::sqrt(ex * ex + ey * ey);
      c->f_area[f] = L;
      c->f_normal[2 * f] = ey / L;
      c->f_normal[2 * f + 1] = -ex / L;
      for (int q = 0; q < nq; ++q) {
        qp[2 * q] = a[0] + gfx[q] * ex;
        qp[2 * q + 1] = a[1] + gfx[q] * ey;
        qw[q] = gfw[q];
      }
    } else if (F.v[3] < 0) {
      // flat triangle: x0 + a (x1 - x0 + b (x2 - x1)), area element 2 A a
      const double* x0 = &c->verts[(size_t)F.v[0] * 3];
      const double* x1 = &c->verts[(size_t)F.v[1] * 3];
      const double* x2 = &c->verts[(size_t)F.v[2] * 3];
      double d10[3], d20[3], d21[3], Sv[3];
      for (int d = 0; d < 3; ++d) {
        d10[d] = x1[d] - x0[d];
        d20[d] = x2[d] - x0[d];
        d21[d] = x2[d] - x1[d];
      }
      cross3(d10, d20, Sv);
      for (int d = 0; d < 3; ++d) Sv[d] *= 0.5;
      const double A = std::sqrt(Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2]);
      c->f_area[f] = A;
      for (int d = 0; d < 3; ++d) c->f_normal[3 * f + d] = Sv[d] / A;
      int q = 0;
      for (int i = 0; i < ng; ++i)
        for (int j = 0; j < ng; ++j, ++q) {
          const double a = t1x[i], b = gfx[j];
          for (int d = 0; d < 3; ++d) qp[3 * q + d] = x0[d] + a * (d10[d] + b * d21[d]);
          qw[q] = 2.0 * t1w[i] * gfw[j];  // the weights of u on [0,1] sum to 1/2
        }
    } else {
      const double* x0 = &c->verts[(size_t)F.v[0] * 3];
      const double* x1 = &c->verts[(size_t)F.v[1] * 3];
      const double* x2 = &c->verts[(size_t)F.v[2] * 3];
      const double* x3 = &c->verts[(size_t)F.v[3] * 3];
      double d20[3], d31[3], Sv[3];
      for (int d = 0; d < 3; ++d) { d20[d] = x2[d] - x0[d]; d31[d] = x3[d] - x1[d]; }
      cross3(d20, d31, Sv);
      for (int d = 0; d < 3; ++d) Sv[d] *= 0.5;
      double A = std::sqrt(Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2]);
      c->f_area[f] = A;
      for (int d = 0; d < 3; ++d) c->f_normal[3 * f + d] = Sv[d] / A;
      if (fan) {
        // the fan starts at the face's lowest-numbered vertex y0 (cyclic order
        // kept): triangles (y0, y1, y2) and (y0, y2, y3); a point of triangle
        // (a, b, c) is a + s (b - a + t (c - b)), weight 2 w_s w_t of the
        // triangle's share A_k / (A_0 + A_1) of the face
        int m = 0;
        for (int k = 1; k < 4; ++k)
          if (F.v[k] < F.v[m]) m = k;
        const double* y[4];
        for (int k = 0; k < 4; ++k) y[k] = &c->verts[(size_t)F.v[(m + k) % 4] * 3];
        const double* tri[2][3] = {{y[0], y[1], y[2]}, {y[0], y[2], y[3]}};
        double At[2];
        for (int k = 0; k < 2; ++k) {
          double u1[3], u2[3], cr[3];
          for (int d = 0; d < 3; ++d) {
            u1[d] = tri[k][1][d] - tri[k][0][d];
            u2[d] = tri[k][2][d] - tri[k][0][d];
          }
          cross3(u1, u2, cr);
          At[k] = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        }
        // the face area is the sum of the triangle areas (Sec. 3.1); on a
        // warped face it exceeds |S_f|, whose direction stays the normal
        c->f_area[f] = At[0] + At[1];
        int q = 0;
        for (int k = 0; k < 2; ++k)
          for (int i = 0; i < ng; ++i)
            for (int j = 0; j < ng; ++j, ++q) {
              const double s = t1x[i], t = gfx[j];
              for (int d = 0; d < 3; ++d)
                qp[3 * q + d] = tri[k][0][d] + s * (tri[k][1][d] - tri[k][0][d] + t * (tri[k][2][d] - tri[k][1][d]));
              qw[q] = 2.0 * t1w[i] * gfw[j] * At[k] / (At[0] + At[1]);
            }
      } else {
        double wsum = 0;
        int q = 0;
        for (int i = 0; i < ng; ++i)
          for (int j = 0; j < ng; ++j, ++q) {
            double s = gfx[i], t = gfx[j];
            double xs[3], xt[3], nn[3];
            for (int d = 0; d < 3; ++d) {
              qp[3 * q + d] = (1 - s) * (1 - t) * x0[d] + s * (1 - t) * x1[d] + s * t * x2[d] + (1 - s) * t * x3[d];
              xs[d] = (1 - t) * (x1[d] - x0[d]) + t * (x2[d] - x3[d]);
              xt[d] = (1 - s) * (x3[d] - x0[d]) + s * (x2[d] - x1[d]);
            }
            cross3(xs, xt, nn);
            qw[q] = gfw[i] * gfw[j] * std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
            wsum += qw[q];
          }
        for (int k = 0; k < nq; ++k) qw[k] /= wsum;
      }
    }
    for (int d = 0; d < D; ++d) {
      double s = 0;
      for (int q = 0; q < nq; ++q) s += qw[q] * qp[q * D + d];
      c->f_centre[(size_t)f * D + d] = s;
    }
  }
  // boundary views in caller order
  const size_t nb = c->bface.size();
  c->b_centre.resize(nb * D);
  c->b_normal.resize(nb * D);
  c->b_qp.resize(nb * nq * D);
  for (size_t b = 0; b < nb; ++b) {
    int64_t f = c->bface[b];
    for (int d = 0; d < D; ++d) {
      c->b_centre[b * D + d] = c->f_centre[(size_t)f * D + d];
      c->b_normal[b * D + d] = c->f_normal[(size_t)f * D + d];
    }
    for (int k = 0; k < nq * D; ++k) c->b_qp[b * nq * D + k] = c->f_qp[(size_t)f * nq * D + k];
  }
  return HOFV_OK;
}

}  // namespace hofv
