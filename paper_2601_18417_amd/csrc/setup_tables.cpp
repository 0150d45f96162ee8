// Builds every device table of the residual, J.v and preconditioner kernels
// on the host and uploads it (hofv_setup).
//
//  * face tables (internal faces, then displacement faces): stencil around the
//    face centre, gradient coefficients at each quadrature point (eq.
//    faceQuadGrad with the ghost node of Sec. 3.5.3 on displacement faces),
//    either kept per point or, for linear elasticity, summed with the
//    quadrature weights (n . sigma is linear in grad u, so the face term only
//    needs sum_q alpha_q (grad u)_q when every point shares the face normal);
//  * cell tables: stencil around the centroid and, for every face slot, the
//    coefficients of u*_{f,P} - u_P (eq. alphaJump);
//  * sources at load 1: body force (eq. bodyTerm), traction faces, the ghost
//    part of displacement-face gradients (linear elasticity) and the u_b part
//    of the displacement-face stabilisation;
//  * the compact approximate Jacobian in FP32 with a greedy colouring.
#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.h"

namespace hofv {

hofv_status build_tables(hofv_ctx* c) {
  auto t0 = std::chrono::steady_clock::now();
  const int D = c->D, p = c->prm.order_p, NS = c->NS;
  // u* extrapolation items: cells with NSI slots each, as many as the most
  // faces a cell has (2 dim for quads and hexahedra, dim + 1 for simplices),
  // or, when a cell has more faces than a hexahedron, one item per cell face
  // that needs u*
  const bool hf = NS > 2 * D;
  int NSI = 1;
  if (!hf)
    for (const hofv_ctx::Face& F : c->faces) NSI = std::max(NSI, std::max(F.sown, F.snei) + 1);
  const int64_t nc = c->nc;
  const int nq = c->nq;
  const bool nh = c->prm.material == HOFV_NEO_HOOKEAN;
  const bool fold = !nh && c->prm.fold_quadrature;
  const double mu = c->prm.mu, lam = c->prm.lambda, kbar = 2 * mu + lam;
  const int S0 = n_basis(D, p) + c->prm.n_plus;  // |S| = N_t + n+ (Sec. 3.5.2)
  if (S0 > 255) return fail(c, HOFV_EINVAL, "stencil size above 255");
  if (S0 > nc) return fail(c, HOFV_EINVAL, "stencil size exceeds the number of cells");
  const double kshape = c->prm.k_weight, gw = c->prm.ghost_weight, alpha = c->prm.alpha;

  // kernel faces: internal, then displacement, each along a Morton curve of
  // the face centres (item blocks of the face kernels cover compact patches)
  std::vector<int64_t> kf;
  kf.reserve(c->faces.size());
  for (int64_t f = 0; f < c->n_internal; ++f) kf.push_back(f);
  std::vector<int64_t> trac, symb;
  for (size_t b = 0; b < c->bface.size(); ++b) {
    if (c->btype[b] == HOFV_BC_DISPLACEMENT) kf.push_back(c->bface[b]);
    else if (c->btype[b] == HOFV_BC_SYMMETRY) symb.push_back((int64_t)b);
    else trac.push_back((int64_t)b);
  }
  auto curve = [&](int64_t begin, int64_t end) {
    std::vector<double> x((size_t)(end - begin) * D);
    for (int64_t i = begin; i < end; ++i)
      for (int d = 0; d < D; ++d) x[(i - begin) * D + d] = c->f_centre[(size_t)kf[i] * D + d];
    const std::vector<int64_t> o = morton_order(x.data(), D, end - begin);
    std::vector<int64_t> part(o.size());
    for (size_t r = 0; r < o.size(); ++r) part[r] = kf[begin + o[r]];
    std::copy(part.begin(), part.end(), kf.begin() + begin);
  };
  curve(0, c->n_internal);
  curve(c->n_internal, (int64_t)kf.size());
  // cells along a Morton curve of the centroids: the order of the extrapolation items
  const std::vector<int64_t> corder = morton_order(c->cen.data(), D, nc);
  const int64_t nf = (int64_t)kf.size(), nfi = c->n_internal, nfd = nf - nfi;
  std::vector<int64_t> kf_of_face(c->faces.size(), -1);
  std::vector<int64_t> bidx_of_face(c->faces.size(), -1);
  for (int64_t i = 0; i < nf; ++i) kf_of_face[kf[i]] = i;
  for (size_t b = 0; b < c->bface.size(); ++b) bidx_of_face[c->bface[b]] = (int64_t)b;

  // stencils
  std::vector<double> pts((size_t)nf * D);
  for (int64_t i = 0; i < nf; ++i)
    for (int d = 0; d < D; ++d) pts[i * D + d] = c->f_centre[(size_t)kf[i] * D + d];
  std::vector<int32_t> fst((size_t)nf * S0), cst((size_t)nc * S0);
  nearest_cells(c->cen, D, nc, pts.data(), nf, S0, c->prm.stencil_quantum, fst.data());
  nearest_cells(c->cen, D, nc, c->cen.data(), nc, S0, c->prm.stencil_quantum, cst.data());
  // stencil size per face and per cell: S0, or more where stencil_grow
  // enlarged a stencil that failed the pivot test; the tables take the
  // largest (S) and shorter stencils get zero coefficients past their end
  std::vector<int32_t> fsz(nf, S0), csz(nc, S0);
  std::vector<std::vector<int32_t>> fgrown, cgrown;
  int64_t n_grown = 0;
  if (c->prm.stencil_grow > 0) {
    const double qnt = c->prm.stencil_quantum;
    const int g = c->prm.stencil_grow;
    const double tgt[3] = {0, 1, 2};
    // the cells whose u* is needed: both sides of internal faces and the
    // owners of displacement faces
    std::vector<char> need(nc, 0);
    for (int64_t i = 0; i < nf; ++i) {
      const hofv_ctx::Face& F = c->faces[kf[i]];
      need[F.own] = 1;
      if (F.nei >= 0) need[F.nei] = 1;
    }
    // pivot test of every least-squares system a stencil takes part in
    auto face_ok = [&](int64_t i, const int32_t* ids, int sz) {
      const int64_t f = kf[i];
      const bool disp = c->faces[f].nei < 0;
      double X[256 * 3], out[3 * 257], cond, h;
      for (int k = 0; k < sz; ++k)
        for (int d = 0; d < D; ++d) X[k * D + d] = c->cen[(size_t)ids[k] * D + d];
      for (int q = 0; q < nq; ++q) {
        if (c->f_qw[(size_t)f * nq + q] == 0.0) continue;
        if (!ls_functionals(D, p, kshape, &c->f_qp[((size_t)f * nq + q) * D], X, sz, disp ? gw : 0.0,
                            kTargetGradient, D, tgt, out, &cond, &h))
          return false;
      }
      return true;
    };
    auto cell_ok = [&](int64_t P, const int32_t* ids, int sz) {
      if (!need[P]) return true;
      double X[256 * 3], out[3 * 257], cond, h;
      for (int k = 0; k < sz; ++k)
        for (int d = 0; d < D; ++d) X[k * D + d] = c->cen[(size_t)ids[k] * D + d];
      return ls_functionals(D, p, kshape, &c->cen[(size_t)P * D], X, sz, 0.0, kTargetGradient, D, tgt, out, &cond,
                            &h);
    };
    // a failing stencil becomes the S0 + g, S0 + 2g, ... nearest cells
    auto grow = [&](int64_t n, const double* ref, const std::vector<int32_t>& st, std::vector<int32_t>& sz,
                    std::vector<std::vector<int32_t>>& out,
                    const std::function<bool(int64_t, const int32_t*, int)>& ok) {
      out.assign(n, {});
      std::vector<char> bad(n, 0);
#pragma omp parallel for schedule(dynamic, 64)
      for (int64_t i = 0; i < n; ++i) bad[i] = !ok(i, &st[(size_t)i * S0], S0);
      for (int step = 1;; ++step) {
        std::vector<int64_t> idx;
        for (int64_t i = 0; i < n; ++i)
          if (bad[i]) idx.push_back(i);
        if (idx.empty()) return true;
        const int Sg = S0 + step * g;
        if (Sg > 255 || Sg > nc) return false;
        const int64_t m = (int64_t)idx.size();
        std::vector<double> rp((size_t)m * D);
        for (int64_t j = 0; j < m; ++j)
          for (int d = 0; d < D; ++d) rp[j * D + d] = ref[idx[j] * D + d];
        std::vector<int32_t> tmp((size_t)m * Sg);
        nearest_cells(c->cen, D, nc, rp.data(), m, Sg, qnt, tmp.data());
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t j = 0; j < m; ++j) {
          const int64_t i = idx[j];
          out[i].assign(&tmp[(size_t)j * Sg], &tmp[(size_t)j * Sg] + Sg);
          sz[i] = Sg;
          bad[i] = !ok(i, out[i].data(), Sg);
        }
      }
    };
    if (!grow(nf, pts.data(), fst, fsz, fgrown, face_ok))
      return fail(c, HOFV_ESINGULAR, "a face stencil still fails the pivot test after growing it");
    if (!grow(nc, c->cen.data(), cst, csz, cgrown, cell_ok))
      return fail(c, HOFV_ESINGULAR, "a cell stencil still fails the pivot test after growing it");
    for (int32_t v : fsz) n_grown += v > S0;
    for (int32_t v : csz) n_grown += v > S0;
  }
  const int S = std::max(*std::max_element(fsz.begin(), fsz.end()), *std::max_element(csz.begin(), csz.end()));
  // a stencil is a set: store it in increasing cell id (a canonical order;
  // the block unions are built from it), padded to S with its largest id
  auto relayout = [&](int64_t n, std::vector<int32_t>& st, const std::vector<int32_t>& sz,
                      const std::vector<std::vector<int32_t>>& grown) {
    std::vector<int32_t> out((size_t)n * S);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const int32_t* from = grown.empty() || grown[i].empty() ? &st[(size_t)i * S0] : grown[i].data();
      int32_t* to = &out[(size_t)i * S];
      std::copy_n(from, sz[i], to);
      std::sort(to, to + sz[i]);
      for (int k = sz[i]; k < S; ++k) to[k] = to[sz[i] - 1];
    }
    st.swap(out);
  };
  relayout(nf, fst, fsz, fgrown);
  relayout(nc, cst, csz, cgrown);
  fgrown.clear();
  cgrown.clear();
  const StencilBlocks fblk = make_blocks(fst.data(), nf, S, nc, kBlockItems, kLdsFaceCells);
  if (fblk.max_cells > kLdsFaceCells)
    return fail(c, HOFV_EINVAL, "stencil union of one item exceeds the LDS staging capacity");

  // face coefficients
  const int ncoef = fold ? D : nq * D;
  std::vector<double> fcoef((size_t)S * ncoef * nf, 0.0);
  std::vector<double> fsv((size_t)(fold ? D : nq * D) * nf, 0.0);
  std::vector<double> fstab(nf, 0.0), faj(nf, 0.0);
  std::vector<double> fghost(nh ? (size_t)nq * D * D * std::max<int64_t>(nfd, 1) : 0, 0.0);
  std::vector<double> src((size_t)D * nc, 0.0);
  std::vector<int32_t> fown(nf), fnei(nf), fslots(nf);
  double max_cond = 0.0;
  bool singular = false;
  // per-face constant source contributions, summed into src serially afterwards
  std::vector<double> fsrc((size_t)nf * D, 0.0);
#pragma omp parallel for schedule(dynamic, 64) reduction(max : max_cond) reduction(|| : singular)
  for (int64_t i = 0; i < nf; ++i) {
    const int64_t f = kf[i];
    const hofv_ctx::Face& F = c->faces[f];
    const bool disp = F.nei < 0;
    const int64_t b = disp ? bidx_of_face[f] : -1;
    fown[i] = (int32_t)F.own;
    fnei[i] = (int32_t)F.nei;
    fslots[i] = F.sown | ((disp ? 0 : F.snei) << 8);
    const double* n = &c->f_normal[(size_t)f * D];
    const double A = c->f_area[f];
    const double* qw = &c->f_qw[(size_t)f * nq];
    const int Si = fsz[i];  // this face's stencil (S0, or grown)
    double X[256 * 3];
    for (int k = 0; k < Si; ++k)
      for (int d = 0; d < D; ++d) X[k * D + d] = c->cen[(size_t)fst[i * S + k] * D + d];
    double targets[3] = {0, 1, 2};
    double out[3 * 256];
    double Gg[3][3] = {{0}};  // sum_q alpha_q ghost gradient (LE) at load 1
    for (int q = 0; q < nq; ++q) {
      if (qw[q] == 0.0) continue;  // a padding point of a face with fewer points
      double cond, h;
      bool ok = ls_functionals(D, p, kshape, &c->f_qp[((size_t)f * nq + q) * D], X, Si, disp ? gw : 0.0,
                               kTargetGradient, D, targets, out, &cond, &h);
      if (!ok) singular = true;
      max_cond = std::max(max_cond, cond);
      const int m = Si + (disp ? 1 : 0);
      for (int a = 0; a < D; ++a) {
        for (int k = 0; k < Si; ++k) {
          if (fold) fcoef[fblk.at(i, k, a, D, S)] += qw[q] * out[a * m + k];
          else fcoef[fblk.at(i, k, q * D + a, nq * D, S)] = out[a * m + k];
        }
        if (disp) {
          const double cg = out[a * m + Si];
          const double* ub = &c->ubq[((size_t)b * nq + q) * D];
          for (int j = 0; j < D; ++j) {
            if (nh) fghost[(((size_t)q * D + a) * D + j) * nfd + (i - nfi)] = cg * ub[j];
            else Gg[a][j] += qw[q] * cg * ub[j];
          }
        }
      }
      if (!fold)
        for (int d = 0; d < D; ++d) fsv[((size_t)q * D + d) * nf + i] = qw[q] * A * n[d];
    }
    if (fold)
      for (int d = 0; d < D; ++d) fsv[(size_t)d * nf + i] = A * n[d];
    // stabilisation coefficient alpha Kbar Gamma / |d . n|
    const double* xP = &c->cen[(size_t)F.own * D];
    const double* xo = disp ? &c->f_centre[(size_t)f * D] : &c->cen[(size_t)F.nei * D];
    double dn = 0;
    for (int d = 0; d < D; ++d) dn += (xo[d] - xP[d]) * n[d];
    const double a_f = alpha * kbar * A / std::fabs(dn);
    fstab[i] = a_f;
    faj[i] = kbar * A / std::fabs(dn);
    if (disp) {
      // constant parts: u_b of the stabilisation and (LE) the ghost term
      const double* ubc = &c->ubc[(size_t)b * D];
      for (int j = 0; j < D; ++j) fsrc[i * D + j] += a_f * ubc[j];
      if (!nh) {
        double tr = 0;
        for (int d = 0; d < D; ++d) tr += Gg[d][d];
        for (int j = 0; j < D; ++j) {
          double t = 0;
          for (int a = 0; a < D; ++a) t += A * n[a] * (mu * (Gg[a][j] + Gg[j][a]) + (a == j ? lam * tr : 0.0));
          fsrc[i * D + j] += t;
        }
      }
    }
  }
  if (singular) return fail(c, HOFV_ESINGULAR, "rank-deficient least-squares stencil at a face quadrature point");
  for (int64_t i = nfi; i < nf; ++i)
    for (int j = 0; j < D; ++j) src[(size_t)j * nc + fown[i]] += fsrc[i * D + j];

  // symmetry faces (Sec. 3.5): the ceil(S/2) cells nearest the face centre and
  // their mirror images through the face plane; the images carry R u, R = I - 2 n n.
  // For the linear law the face term is linear in each u_N: folded over the
  // quadrature points into T[N][j][k], the traction t_j per unit u_N,k.
  const int Sh = (S0 + 1) / 2;
  const int64_t nfs = (int64_t)symb.size();
  std::vector<int32_t> sst((size_t)nfs * Sh), sst_t((size_t)Sh * nfs);
  std::vector<double> sT(nh ? 0 : (size_t)Sh * D * D * nfs, 0.0), saj(nfs, 0.0);
  // neo-Hookean: per-point coefficients of each cell and of its image
  // [Sh][nq][2][D][nfs], weighted area vectors [nq][D][nfs], normals [D][nfs]
  std::vector<double> sC(nh ? (size_t)Sh * nq * 2 * D * nfs : 0, 0.0), ssv(nh ? (size_t)nq * D * nfs : 0, 0.0),
      sn(nh ? (size_t)D * nfs : 0, 0.0);
  std::vector<int32_t> sown(nfs), sslot(nfs);
  if (nfs) {
    std::vector<double> spts((size_t)nfs * D);
    for (int64_t i = 0; i < nfs; ++i)
      for (int d = 0; d < D; ++d) spts[i * D + d] = c->f_centre[(size_t)c->bface[symb[i]] * D + d];
    nearest_cells(c->cen, D, nc, spts.data(), nfs, Sh, c->prm.stencil_quantum, sst.data());
  }
#pragma omp parallel for schedule(dynamic, 16) reduction(max : max_cond) reduction(|| : singular)
  for (int64_t i = 0; i < nfs; ++i) {
    const int64_t f = c->bface[symb[i]];
    const hofv_ctx::Face& F = c->faces[f];
    sown[i] = (int32_t)F.own;
    sslot[i] = F.sown;
    const double* n = &c->f_normal[(size_t)f * D];
    const double* xf = &c->f_centre[(size_t)f * D];
    const double A = c->f_area[f];
    double X[512 * 3];
    for (int k = 0; k < Sh; ++k) {
      const double* x = &c->cen[(size_t)sst[i * Sh + k] * D];
      double dn = 0;
      for (int d = 0; d < D; ++d) dn += (x[d] - xf[d]) * n[d];
      for (int d = 0; d < D; ++d) {
        X[k * D + d] = x[d];
        X[(Sh + k) * D + d] = x[d] - 2.0 * dn * n[d];
      }
    }
    double R[3][3];
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) R[a][b] = (a == b ? 1.0 : 0.0) - 2.0 * n[a] * n[b];
    const double targets[3] = {0, 1, 2};
    double out[3 * 512];
    for (int q = 0; q < nq; ++q) {
      if (c->f_qw[(size_t)f * nq + q] == 0.0) continue;  // padding point
      double cond, h;
      const bool ok = ls_functionals(D, p, kshape, &c->f_qp[((size_t)f * nq + q) * D], X, 2 * Sh, 0.0,
                                     kTargetGradient, D, targets, out, &cond, &h);
      if (!ok) singular = true;
      max_cond = std::max(max_cond, cond);
      const double wq = c->f_qw[(size_t)f * nq + q] * A;
      const int m = 2 * Sh;
      if (nh) {
        for (int N = 0; N < Sh; ++N)
          for (int side = 0; side < 2; ++side)
            for (int a = 0; a < D; ++a)
              sC[((((size_t)N * nq + q) * 2 + side) * D + a) * nfs + i] = out[a * m + side * Sh + N];
        for (int d = 0; d < D; ++d) ssv[((size_t)q * D + d) * nfs + i] = wq * n[d];
        continue;
      }
      for (int N = 0; N < Sh; ++N)
        for (int kc = 0; kc < D; ++kc) {
          // gradient G[a][j] produced by a unit u_N,kc: its own coefficient and its image's
          double G[3][3];
          for (int a = 0; a < D; ++a)
            for (int j = 0; j < D; ++j)
              G[a][j] = out[a * m + N] * (j == kc ? 1.0 : 0.0) + out[a * m + Sh + N] * R[j][kc];
          double tr = 0;
          for (int d = 0; d < D; ++d) tr += G[d][d];
          for (int j = 0; j < D; ++j) {
            double t = 0;
            for (int a = 0; a < D; ++a) t += n[a] * (mu * (G[a][j] + G[j][a]) + (a == j ? lam * tr : 0.0));
            sT[(((size_t)N * D + j) * D + kc) * nfs + i] += wq * t;
          }
        }
    }
    if (nh)
      for (int d = 0; d < D; ++d) sn[(size_t)d * nfs + i] = n[d];
    const double* xP = &c->cen[(size_t)F.own * D];
    double dn = 0;
    for (int d = 0; d < D; ++d) dn += (xf[d] - xP[d]) * n[d];
    saj[i] = kbar * A / std::fabs(dn);
  }
  if (singular) return fail(c, HOFV_ESINGULAR, "rank-deficient least-squares stencil at a symmetry face");
  for (int64_t i = 0; i < nfs; ++i)
    for (int N = 0; N < Sh; ++N) sst_t[(size_t)N * nfs + i] = sst[i * Sh + N];

  // face slot codes, extrapolation items and their rows
  std::vector<int32_t> cfaces((size_t)NS * nc, kNoFace);
  for (int64_t i = 0; i < nf; ++i) {
    cfaces[(size_t)(fslots[i] & 0xff) * nc + fown[i]] = (int32_t)i;
    if (i < nfi) cfaces[(size_t)(fslots[i] >> 8) * nc + fnei[i]] = ~(int32_t)i;
  }
  for (int64_t i = 0; i < nfs; ++i) cfaces[(size_t)sslot[i] * nc + sown[i]] = (int32_t)(nf + i);
  // items: cells in Morton order, or (hf) the slots with internal or
  // displacement faces of the cells in that order
  std::vector<int32_t> ccell, cpos(nc, -1), item_of((size_t)NS * nc, -1);
  for (int64_t r = 0; r < nc; ++r) {
    const int64_t P = corder[r];
    cpos[P] = (int32_t)ccell.size();
    if (!hf) {
      ccell.push_back((int32_t)P);
      continue;
    }
    for (int s = 0; s < NS; ++s) {
      const int32_t code = cfaces[(size_t)s * nc + P];
      if (code == kNoFace || code >= nf) continue;
      item_of[(size_t)s * nc + P] = (int32_t)ccell.size();
      ccell.push_back((int32_t)P);
    }
  }
  const int64_t ni = (int64_t)ccell.size();
  std::vector<int32_t> cst_item((size_t)ni * S);  // stencils by extrapolation item
  for (int64_t r = 0; r < ni; ++r) std::copy_n(&cst[(size_t)ccell[r] * S], S, &cst_item[(size_t)r * S]);
  const StencilBlocks cblk = make_blocks(cst_item.data(), ni, S, nc, kBlockItems, kLdsCellCells);
  if (cblk.max_cells > kLdsCellCells)
    return fail(c, HOFV_EINVAL, "stencil union of one item exceeds the LDS staging capacity");
  std::vector<double> cext((size_t)S * NSI * ni, 0.0);
#pragma omp parallel for schedule(dynamic, 64) reduction(max : max_cond) reduction(|| : singular)
  for (int64_t P = 0; P < nc; ++P) {
    const int Sp = csz[P];  // this cell's stencil (S0, or grown)
    double X[256 * 3];
    for (int k = 0; k < Sp; ++k)
      for (int d = 0; d < D; ++d) X[k * D + d] = c->cen[(size_t)cst[P * S + k] * D + d];
    std::vector<double> dvec((size_t)NS * 3);
    std::vector<int> slots(NS);
    int nt = 0;
    for (int s = 0; s < NS; ++s) {
      int32_t code = cfaces[(size_t)s * nc + P];
      if (code == kNoFace || code >= nf) continue;  // traction and symmetry faces need no u*
      int64_t i = code >= 0 ? code : ~code;
      int64_t f = kf[i];
      for (int d = 0; d < D; ++d) dvec[nt * D + d] = c->f_centre[(size_t)f * D + d] - c->cen[(size_t)P * D + d];
      slots[nt++] = s;
    }
    if (nt == 0) continue;
    std::vector<double> out((size_t)nt * Sp);
    double cond, h;
    bool ok = ls_functionals(D, p, kshape, &c->cen[(size_t)P * D], X, Sp, 0.0, kTargetExtrap, nt, dvec.data(),
                             out.data(), &cond, &h);
    if (!ok) singular = true;
    max_cond = std::max(max_cond, cond);
    for (int r = 0; r < nt; ++r)
      for (int k = 0; k < Sp; ++k) {
        if (hf) cext[cblk.at(item_of[(size_t)slots[r] * nc + P], k, 0, 1, S)] = out[r * Sp + k];
        else cext[cblk.at(cpos[P], k, slots[r], NSI, S)] = out[r * Sp + k];
      }
  }
  if (singular) return fail(c, HOFV_ESINGULAR, "rank-deficient least-squares stencil at a cell centroid");

  // body force and traction sources (load 1)
  if (!c->fb.empty()) {
#pragma omp parallel for schedule(static)
    for (int64_t P = 0; P < nc; ++P)
      for (int j = 0; j < D; ++j) {
        double s = 0;
        for (int64_t q = c->vq_ptr[P]; q < c->vq_ptr[P + 1]; ++q) s += c->vq_w[q] * c->fb[(size_t)q * D + j];
        src[(size_t)j * nc + P] += s;
      }
  }
  for (int64_t b : trac) {
    int64_t f = c->bface[b];
    const hofv_ctx::Face& F = c->faces[f];
    for (int j = 0; j < D; ++j) {
      double s = 0;
      for (int q = 0; q < nq; ++q) s += c->f_qw[(size_t)f * nq + q] * c->tq[((size_t)b * nq + q) * D + j];
      src[(size_t)j * nc + F.own] += c->f_area[f] * s;
    }
  }

  // compact approximate Jacobian: scalar A on every component
  std::vector<double> diag(nc, 0.0);
  std::vector<double> offd((size_t)NS * nc, 0.0);
  std::vector<int64_t> nbr((size_t)NS * nc, -1);
  for (int64_t i = 0; i < nf; ++i) {
    const double a = faj[i];  // Kbar Gamma / |d . n|
    const int64_t P = fown[i];
    diag[P] -= a;
    if (i < nfi) {
      const int64_t N = fnei[i];
      diag[N] -= a;
      offd[(size_t)(fslots[i] & 0xff) * nc + P] = a;
      nbr[(size_t)(fslots[i] & 0xff) * nc + P] = N;
      offd[(size_t)(fslots[i] >> 8) * nc + N] = a;
      nbr[(size_t)(fslots[i] >> 8) * nc + N] = P;
    }
  }
  // symmetry faces: the term a_b (R_b - I) u_P = -2 a_b n n^T u_P acts on the
  // normal component only; one scalar matrix for every component takes its
  // isotropic average, -(2/3) a_b on the diagonal
  for (int64_t i = 0; i < nfs; ++i) diag[sown[i]] -= (2.0 / 3.0) * saj[i];
  std::vector<int32_t> colour(nc, -1);
  int ncol = 0;
  for (int64_t P = 0; P < nc; ++P) {
    uint64_t used = 0;
    for (int s = 0; s < NS; ++s) {
      int64_t N = nbr[(size_t)s * nc + P];
      if (N >= 0 && colour[N] >= 0 && colour[N] < 64) used |= 1ull << colour[N];
    }
    int col = 0;
    while (used >> col & 1ull) ++col;
    colour[P] = col;
    ncol = std::max(ncol, col + 1);
  }
  // cells using slots beyond 2 dim (slots are numbered in the order a cell's
  // faces come, so these are exactly the cells with more than 2 dim faces):
  // within a colour they come first, where the sweeps give them lane groups
  // (the order inside a colour does not change a sweep)
  std::vector<uint8_t> big(nc, 0);
  for (const hofv_ctx::Face& F : c->faces) {
    if (F.sown >= 2 * D) big[F.own] = 1;
    if (F.nei >= 0 && F.snei >= 2 * D) big[F.nei] = 1;
  }
  std::vector<int32_t> perm(nc);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
    return colour[a] != colour[b] ? colour[a] < colour[b] : big[a] > big[b];
  });
  std::vector<int32_t> pos(nc);
  for (int64_t i = 0; i < nc; ++i) pos[perm[i]] = (int32_t)i;
  c->dev.colour_start.assign(ncol + 1, 0);
  for (int64_t P = 0; P < nc; ++P) c->dev.colour_start[colour[P] + 1]++;
  // face-neighbour graph of the learned correction: omega_PN = a_PN / sum a,
  // e_PN = unit vector from x_P to x_N; wb holds, for the neighbour N in slot
  // s of P, the weights with which h_P enters N's aggregates
  std::vector<int32_t> gnbr((size_t)NS * nc, -1);
  std::vector<float> gwf((size_t)NS * 4 * nc, 0.f), gwb((size_t)NS * 4 * nc, 0.f), gbf(nc, 0.f);
  for (int64_t i = nfi; i < nf; ++i) gbf[fown[i]] = 1.f;
  for (int64_t P = 0; P < nc; ++P) {
    double asum = 0;
    for (int s = 0; s < NS; ++s)
      if (nbr[(size_t)s * nc + P] >= 0) asum += offd[(size_t)s * nc + P];
    for (int s = 0; s < NS; ++s) {
      const int64_t N = nbr[(size_t)s * nc + P];
      if (N < 0) continue;
      gnbr[(size_t)s * nc + P] = (int32_t)N;
      const double om = offd[(size_t)s * nc + P] / asum;
      double dv[3] = {0, 0, 0}, len = 0;
      for (int d = 0; d < D; ++d) {
        dv[d] = c->cen[(size_t)N * D + d] - c->cen[(size_t)P * D + d];
        len += dv[d] * dv[d];
      }
      len = std::sqrt(len);
      gwf[((size_t)s * nc + P) * 4 + 0] = (float)om;
      for (int d = 0; d < 3; ++d) gwf[((size_t)s * nc + P) * 4 + 1 + d] = (float)(om * dv[d] / len);
    }
  }
  for (int64_t P = 0; P < nc; ++P)
    for (int s = 0; s < NS; ++s) {
      const int64_t N = nbr[(size_t)s * nc + P];
      if (N < 0) continue;
      for (int s2 = 0; s2 < NS; ++s2)
        if (nbr[(size_t)s2 * nc + N] == P)
          for (int d = 0; d < 4; ++d) gwb[((size_t)s * nc + P) * 4 + d] = gwf[((size_t)s2 * nc + N) * 4 + d];
    }

  // the stabilisation term reads u* by extrapolation item (and slot within it)
  std::vector<int32_t> fown_item(nf), fnei_item(nf), fslots_item(fslots);
  for (int64_t i = 0; i < nf; ++i) {
    if (hf) {
      fown_item[i] = item_of[(size_t)(fslots[i] & 0xff) * nc + fown[i]];
      fnei_item[i] = fnei[i] >= 0 ? item_of[(size_t)(fslots[i] >> 8) * nc + fnei[i]] : -1;
      fslots_item[i] = 0;
    } else {
      fown_item[i] = cpos[fown[i]];
      fnei_item[i] = fnei[i] >= 0 ? cpos[fnei[i]] : -1;
    }
  }
  for (int k = 0; k < ncol; ++k) c->dev.colour_start[k + 1] += c->dev.colour_start[k];
  c->dev.n_colours = ncol;
  std::vector<int32_t> pnbr((size_t)NS * nc);
  std::vector<float> pa((size_t)NS * nc), pdinv(nc), pdiag(nc);
  c->pc_diag.assign(nc, 0.0);
  c->pc_perm.assign(nc, 0);
  for (int64_t i = 0; i < nc; ++i) {
    const int64_t P = perm[i];
    pdinv[i] = (float)(1.0 / diag[P]);
    pdiag[i] = (float)diag[P];
    c->pc_diag[i] = diag[P];
    c->pc_perm[i] = P;
    for (int s = 0; s < NS; ++s) {
      int64_t N = nbr[(size_t)s * nc + P];
      pnbr[(size_t)s * nc + i] = N >= 0 ? pos[N] : (int32_t)i;
      pa[(size_t)s * nc + i] = N >= 0 ? (float)offd[(size_t)s * nc + P] : 0.0f;
    }
  }

  if (c->prm.precond_levels >= 2) {
    // level 0 of the multigrid hierarchy: A in CSR, cell order, sorted columns
    std::vector<int64_t> aptr(nc + 1, 0);
    std::vector<int32_t> acol;
    std::vector<double> aval;
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t P = 0; P < nc; ++P) {
      row.clear();
      row.emplace_back((int32_t)P, diag[P]);
      for (int s = 0; s < NS; ++s)
        if (nbr[(size_t)s * nc + P] >= 0) row.emplace_back((int32_t)nbr[(size_t)s * nc + P], offd[(size_t)s * nc + P]);
      std::sort(row.begin(), row.end());
      for (auto& e : row) {
        acol.push_back(e.first);
        aval.push_back(e.second);
      }
      aptr[P + 1] = (int64_t)acol.size();
    }
    hofv_status sm = build_multigrid(c, aptr, acol, aval, pos, c->prm.precond_levels);
    if (sm) return sm;
    c->use_mg = c->dev.mg.size() > 1;
  }

  if (c->prm.host_only) {
    auto keep = [&](const char* name, const auto& v) {
      hofv_ctx::HostTable& h = c->host_tables[name];
      h.elem = (int32_t)sizeof(v[0]);
      h.bytes.resize(v.size() * sizeof(v[0]));
      if (!v.empty()) std::memcpy(h.bytes.data(), v.data(), h.bytes.size());
    };
    // global stencils, k-major, for inspection
    std::vector<int32_t> fst_k((size_t)S * nf), cst_k((size_t)S * ni);
    for (int64_t i = 0; i < nf; ++i)
      for (int k = 0; k < S; ++k) fst_k[(size_t)k * nf + i] = fst[(size_t)i * S + k];
    for (int64_t r = 0; r < ni; ++r)
      for (int k = 0; k < S; ++k) cst_k[(size_t)k * ni + r] = cst_item[(size_t)r * S + k];
    keep("face_stencil", fst_k);
    keep("cell_stencil", cst_k);
    keep("cell_order", ccell);
    keep("face_blk_item", fblk.item);
    keep("face_blk_cell", fblk.cell);
    keep("face_ucell", fblk.cells);
    // per-entry tables in the plain k-major layout (the device holds them block by block)
    keep("face_local", fblk.unblocked(fblk.local, 1, S));
    keep("cell_blk_item", cblk.item);
    keep("cell_blk_cell", cblk.cell);
    keep("cell_ucell", cblk.cells);
    keep("cell_local", cblk.unblocked(cblk.local, 1, S));
    keep("face_coef", fblk.unblocked(fcoef, ncoef, S));
    keep("cell_extrap", cblk.unblocked(cext, NSI, S));
    keep("face_own", fown);
    keep("face_nei", fnei);
    keep("face_area_vec", fsv);
    keep("face_stab", fstab);
    keep("cell_faces", cfaces);
    keep("cell_src", src);
    keep("pc_perm", perm);
    keep("pc_dinv", pdinv);
    keep("pc_a", pa);
    keep("pc_nbr", pnbr);
    keep("centroids", c->cen);
    keep("face_centre", pts);
    keep("nn_nbr", gnbr);
    keep("nn_wf", gwf);
    keep("nn_wb", gwb);
    keep("nn_bflag", gbf);
    c->dev.S = S;
    c->dev.nq = nq;
    c->dev.nf = nf;
    c->dev.nfi = nfi;
  }
  // byte model (algorithmic HBM bytes per launch): coefficient streams and
  // 2-byte local indices per stencil entry, per-item data, the block cell
  // lists, u counted once per cell (the staging gathers of a cell shared by
  // several blocks hit in L2)
  const double ub = (double)D * 8 * nc;
  const double face_b = (double)nf * S * (ncoef * 8.0 + 2.0) + (double)nf * (4 * 3 + 8 + 8.0 * (fold ? D : nq * D)) +
                        (nh ? (double)nq * D * D * 8 * nfd : 0.0) + 4.0 * fblk.cells.size() + ub +
                        2.0 * D * 8 * nf + (double)D * 8 * nf;
  const double ext_b = (double)ni * S * (NSI * 8.0 + 2.0) + 4.0 * cblk.cells.size() + 4.0 * ni + ub +
                       (double)NSI * D * 8 * ni;
  const double sum_b = (double)nc * (NS * 4.0 + 2 * D * 8.0) + 2.0 * D * 8 * nf;
  c->kernel_bytes[nh ? "k_face_nh" : (fold ? "k_face_le" : "k_face_q")] = face_b;
  c->kernel_bytes["k_extrap"] = ext_b;
  c->kernel_bytes["k_cell_sum"] = sum_b;
  c->report.stencil_size = S;
  c->report.n_grown_stencils = n_grown;
  c->report.n_colours = ncol;
  c->report.n_internal_faces = nfi;
  c->report.n_disp_faces = nfd;
  c->report.n_trac_faces = (int64_t)trac.size();
  c->report.max_cond = max_cond;
  c->report.residual_bytes = face_b + ext_b + sum_b;
  if (c->prm.host_only) {
    c->report.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return HOFV_OK;
  }

  // upload
  DeviceTables& t = c->dev;
  t.S = S;
  t.nq = nq;
  t.nf = nf;
  t.nfi = nfi;
  hofv_status st;
#define UP(ptr, vec) \
  if ((st = upload(c, &ptr, vec))) return st;
  t.nfb = (int32_t)fblk.item.size() - 1;
  t.ncb = (int32_t)cblk.item.size() - 1;
  UP(t.f_blk_item, fblk.item);
  UP(t.f_blk_cell, fblk.cell);
  UP(t.f_ucell, fblk.cells);
  UP(t.f_local, fblk.local);
  UP(t.c_blk_item, cblk.item);
  UP(t.c_blk_cell, cblk.cell);
  UP(t.c_ucell, cblk.cells);
  UP(t.c_local, cblk.local);
  UP(t.c_cell, ccell);
  UP(t.f_coef, fcoef);
  UP(t.f_own, fown_item);
  UP(t.f_nei, fnei_item);
  UP(t.f_slots, fslots_item);
  UP(t.f_area_vec, fsv);
  UP(t.f_stab, fstab);
  if (nh) UP(t.f_ghost, fghost);
  UP(t.c_extrap, cext);
  UP(t.c_faces, cfaces);
  UP(t.c_src, src);
  UP(t.p_perm, perm);
  UP(t.p_nbr, pnbr);
  if (NS > 2 * D) {
    std::vector<int32_t> order;
    std::vector<uint8_t> pbig(nc, 0);
    for (int pass = 1; pass >= 0; --pass)
      for (int64_t P = 0; P < nc; ++P)
        if (big[P] == pass) order.push_back((int32_t)P);
    for (int64_t i = 0; i < nc; ++i) pbig[i] = big[perm[i]];
    t.colour_big_end.assign(ncol, 0);
    for (int k = 0; k < ncol; ++k) {
      int64_t e = t.colour_start[k];
      while (e < t.colour_start[k + 1] && pbig[e]) ++e;
      t.colour_big_end[k] = e;
    }
    t.n_big = 0;
    for (int64_t P = 0; P < nc; ++P) t.n_big += big[P];
    t.grp = 1;
    while (t.grp * 2 * D < NS && t.grp < 64) t.grp *= 2;
    UP(t.c_order, order);
    UP(t.p_big, pbig);
  }
  UP(t.p_a, pa);
  UP(t.p_dinv, pdinv);
  UP(t.p_diag, pdiag);
  UP(t.g_nbr, gnbr);
  UP(t.g_wf, gwf);
  UP(t.g_wb, gwb);
  UP(t.g_bflag, gbf);
  t.sym_nf = nfs;
  t.sym_S = Sh;
  if (nfs) {
    UP(t.sym_st, sst_t);
    if (nh) {
      UP(t.sym_C, sC);
      UP(t.sym_sv, ssv);
      UP(t.sym_n, sn);
    } else {
      UP(t.sym_T, sT);
    }
    if ((st = dev_alloc(c, &t.sym_flux, (size_t)D * nfs))) return st;
  }
#undef UP
  t.nsi = NSI;
  t.ns = NS;
  t.n_items = ni;
  if ((st = dev_alloc(c, &t.ustar, (size_t)NSI * D * ni))) return st;
  if ((st = dev_alloc(c, &t.flux, (size_t)D * nf))) return st;
  if ((st = dev_alloc(c, &t.w, (size_t)(D == 3 ? 4 : 2) * nc))) return st;  // padded gather copy
  if ((st = dev_alloc(c, &t.scratch, 16384))) return st;  // >= 2 x 512 partials of the J.v norms
  if ((st = dev_alloc(c, &t.part, (size_t)3 * kGsChunk * kRedParts))) return st;
  if ((st = dev_alloc(c, &t.eps, 8))) return st;
  if ((st = dev_alloc(c, &t.flag, 8))) return st;
  if ((st = dev_alloc(c, &t.p_r, (size_t)D * nc))) return st;
  if ((st = dev_alloc(c, &t.p_z, (size_t)D * nc))) return st;
  HOFV_HIP(c, hipMemset(t.flag, 0, 8 * sizeof(int32_t)));

  c->report.device_bytes = (double)c->device_bytes;
  c->report.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return HOFV_OK;
}

}  // namespace hofv
