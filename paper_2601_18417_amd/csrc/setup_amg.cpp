// Smoothed-aggregation multigrid hierarchy of the compact approximate Jacobian.
//
// "A few sweeps" of the approximate Jacobian (Sec. 4.1) leave its
// long-wavelength error untouched; on slender parts with free sides this
// stalls the Krylov solver.  The multilevel application keeps the paper's
// matrix, uses its FP32 sweeps as the finest smoother and adds coarse-grid
// corrections.  Rules (levels l = 0, 1, ...; A_0 = the approximate Jacobian):
//  * j != i is a strong neighbour of i on level l when |a_ij| >= theta_l
//    sqrt(a_ii a_jj), theta_l = theta / 2^l (coarse operators spread their
//    couplings over more neighbours);
//  * aggregation in index order: (1) an unassigned node whose strong
//    neighbours are all unassigned opens an aggregate with them; (2) a node
//    left over joins the pass-1 aggregate of its strongest strong neighbour
//    (strengths within a relative 1e-10 tie, the lowest index wins: a uniform
//    mesh's equal couplings must not be ordered by rounding); (3) a node
//    still left over opens an aggregate with
//    its unassigned strong neighbours; aggregates are numbered as created;
//  * tentative prolongation T[i, agg(i)] = 1 smoothed by one damped Jacobi
//    step, P = (I - omega / rho D^-1 A_l) T, rho = max_i sum_j |a_ij| / |a_ii|
//    (a Gershgorin bound of the spectral radius of D^-1 A_l);
//  * A_{l+1} = P^T A_l P; levels are added while the level has more than
//    kCoarseSize nodes, up to the requested count, and while a coarsening
//    keeps at most 80 % of the nodes; the last level is inverted densely.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "common.h"

namespace hofv {

namespace {

constexpr double kTheta = 0.08;
constexpr double kOmega = 4.0 / 3.0;
constexpr int64_t kCoarseSize = 256;
constexpr int64_t kMaxDense = 2048;

struct Csr {  // sorted columns per row, diagonal included
  int64_t n = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  double diag(int64_t i) const {
    for (int64_t t = ptr[i]; t < ptr[i + 1]; ++t)
      if (col[t] == i) return val[t];
    return 0.0;
  }
};

std::vector<int32_t> aggregate(const Csr& A, double theta, int32_t* n_agg) {
  const int64_t n = A.n;
  std::vector<double> d(n);
  for (int64_t i = 0; i < n; ++i) d[i] = A.diag(i);
  auto strong = [&](int64_t i, int64_t t) {
    const int32_t j = A.col[t];
    return j != i && std::fabs(A.val[t]) >= theta * std::sqrt(d[i] * d[j]);
  };
  std::vector<int32_t> agg(n, -1);
  int32_t k = 0;
  for (int64_t i = 0; i < n; ++i) {  // pass 1
    if (agg[i] >= 0) continue;
    bool free = true;
    for (int64_t t = A.ptr[i]; t < A.ptr[i + 1] && free; ++t)
      if (strong(i, t) && agg[A.col[t]] >= 0) free = false;
    if (!free) continue;
    agg[i] = k;
    for (int64_t t = A.ptr[i]; t < A.ptr[i + 1]; ++t)
      if (strong(i, t)) agg[A.col[t]] = k;
    ++k;
  }
  const std::vector<int32_t> first = agg;
  for (int64_t i = 0; i < n; ++i) {  // pass 2
    if (agg[i] >= 0) continue;
    int32_t best = -1;
    double best_v = -1.0;
    for (int64_t t = A.ptr[i]; t < A.ptr[i + 1]; ++t)
      if (strong(i, t) && first[A.col[t]] >= 0 && std::fabs(A.val[t]) > best_v * (1.0 + 1e-10)) {
        best = A.col[t];
        best_v = std::fabs(A.val[t]);
      }
    if (best >= 0) agg[i] = first[best];
  }
  for (int64_t i = 0; i < n; ++i) {  // pass 3
    if (agg[i] >= 0) continue;
    agg[i] = k;
    for (int64_t t = A.ptr[i]; t < A.ptr[i + 1]; ++t)
      if (strong(i, t) && agg[A.col[t]] < 0) agg[A.col[t]] = k;
    ++k;
  }
  *n_agg = k;
  return agg;
}

// sparse product C = A B (Gustavson), rows of C with sorted columns
Csr multiply(const Csr& A, const Csr& B, int64_t ncols) {
  Csr C;
  C.n = A.n;
  C.ptr.assign(A.n + 1, 0);
  std::vector<int64_t> mark(ncols, -1);
  std::vector<double> acc(ncols, 0.0);
  std::vector<int32_t> cols;
  for (int64_t i = 0; i < A.n; ++i) {
    cols.clear();
    for (int64_t t = A.ptr[i]; t < A.ptr[i + 1]; ++t) {
      const int32_t j = A.col[t];
      const double a = A.val[t];
      for (int64_t u = B.ptr[j]; u < B.ptr[j + 1]; ++u) {
        const int32_t k = B.col[u];
        if (mark[k] != i) {
          mark[k] = i;
          acc[k] = 0.0;
          cols.push_back(k);
        }
        acc[k] += a * B.val[u];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t k : cols) {
      C.col.push_back(k);
      C.val.push_back(acc[k]);
    }
    C.ptr[i + 1] = (int64_t)C.col.size();
  }
  return C;
}

Csr transpose(const Csr& A, int64_t ncols) {
  Csr T;
  T.n = ncols;
  T.ptr.assign(ncols + 1, 0);
  for (int32_t c : A.col) T.ptr[c + 1]++;
  for (int64_t k = 0; k < ncols; ++k) T.ptr[k + 1] += T.ptr[k];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int64_t> fill(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t i = 0; i < A.n; ++i)  // rows in increasing order: T's columns come out sorted
    for (int64_t t = A.ptr[i]; t < A.ptr[i + 1]; ++t) {
      const int64_t o = fill[A.col[t]]++;
      T.col[o] = (int32_t)i;
      T.val[o] = A.val[t];
    }
  return T;
}

// dense inverse by Gauss-Jordan elimination with partial pivoting
bool invert(std::vector<double>& a, int64_t n) {
  std::vector<double> inv(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int64_t c = 0; c < n; ++c) {
    int64_t piv = c;
    for (int64_t r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
    if (!(std::fabs(a[piv * n + c]) > 0.0)) return false;
    if (piv != c)
      for (int64_t k = 0; k < n; ++k) {
        std::swap(a[piv * n + k], a[c * n + k]);
        std::swap(inv[piv * n + k], inv[c * n + k]);
      }
    const double s = 1.0 / a[c * n + c];
    for (int64_t k = 0; k < n; ++k) {
      a[c * n + k] *= s;
      inv[c * n + k] *= s;
    }
    for (int64_t r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int64_t k = 0; k < n; ++k) {
        a[r * n + k] -= f * a[c * n + k];
        inv[r * n + k] -= f * inv[c * n + k];
      }
    }
  }
  a.swap(inv);
  return true;
}

// lanes per CSR row in the kernels: the power of two nearest above the average row length
int lanes(size_t nnz, int64_t rows) {
  const double avg = rows > 0 ? (double)nnz / (double)rows : 1.0;
  int g = 1;
  while (g < 64 && g < avg) g <<= 1;
  return g;
}

template <class T, class U>
std::vector<T> cast(const std::vector<U>& v) {
  return std::vector<T>(v.begin(), v.end());
}

}  // namespace

hofv_status build_multigrid(hofv_ctx* c, const std::vector<int64_t>& ptr, const std::vector<int32_t>& col,
                            const std::vector<double>& val, const std::vector<int32_t>& pos, int max_levels) {
  DeviceTables& t = c->dev;
  const int D = c->D;
  Csr A;
  A.n = (int64_t)ptr.size() - 1;
  A.ptr = ptr;
  A.col = col;
  A.val = val;
  std::vector<Csr> levels{A};
  std::vector<Csr> prolong;
  std::vector<double> rho;
  std::vector<std::vector<int32_t>> aggs;
  while ((int)levels.size() < max_levels && levels.back().n > kCoarseSize) {
    const Csr& L = levels.back();
    int32_t nagg = 0;
    const std::vector<int32_t> agg = aggregate(L, kTheta / std::ldexp(1.0, (int)levels.size() - 1), &nagg);
    if (nagg > 0.8 * L.n) break;
    double r = 0.0;
    for (int64_t i = 0; i < L.n; ++i) {
      double s = 0.0;
      for (int64_t u = L.ptr[i]; u < L.ptr[i + 1]; ++u) s += std::fabs(L.val[u]);
      r = std::max(r, s / std::fabs(L.diag(i)));
    }
    // P = T - (omega / rho) D^-1 (A T): row i has agg(i) and the aggregates of its neighbours
    Csr T;
    T.n = L.n;
    T.ptr.resize(L.n + 1);
    for (int64_t i = 0; i <= L.n; ++i) T.ptr[i] = i;
    T.col = agg;
    T.val.assign(L.n, 1.0);
    Csr P = multiply(L, T, nagg);
    for (int64_t i = 0; i < L.n; ++i) {
      const double f = (kOmega / r) / L.diag(i);
      for (int64_t u = P.ptr[i]; u < P.ptr[i + 1]; ++u) P.val[u] = (P.col[u] == agg[i] ? 1.0 : 0.0) - f * P.val[u];
    }
    const Csr Pt = transpose(P, nagg);
    const Csr AP = multiply(L, P, nagg);
    levels.push_back(multiply(Pt, AP, nagg));
    prolong.push_back(P);
    rho.push_back(r);
    aggs.push_back(agg);
  }
  const int nl = (int)levels.size();
  if (c->prm.host_only) {  // aggregates and level sizes for inspection
    std::vector<int32_t> sizes;
    for (const Csr& L : levels) sizes.push_back((int32_t)L.n);
    auto keep = [&](const std::string& name, const std::vector<int32_t>& v) {
      hofv_ctx::HostTable& h = c->host_tables[name];
      h.elem = 4;
      h.bytes.resize(v.size() * 4);
      if (!v.empty()) std::memcpy(h.bytes.data(), v.data(), h.bytes.size());
    };
    keep("mg_sizes", sizes);
    for (size_t l = 0; l < aggs.size(); ++l) keep("mg_agg" + std::to_string(l), aggs[l]);
    return HOFV_OK;
  }
  if (nl < 2) return HOFV_OK;
  if (levels.back().n > kMaxDense) return fail(c, HOFV_EINVAL, "multigrid coarsest level too large for a dense solve");
  hofv_status s;
#define UPV(ptr, vec) \
  if ((s = upload(c, &ptr, vec))) return s;
  t.mg.assign(nl, DeviceTables::MgLevel{});
  for (int l = 0; l < nl; ++l) {
    DeviceTables::MgLevel& m = t.mg[l];
    const Csr& L = levels[l];
    m.n = L.n;
    if (l > 0) {  // off-diagonal CSR, diagonal, damped inverse diagonal (Jacobi smoother)
      std::vector<int32_t> op(L.n + 1, 0), oc;
      std::vector<float> ov, dg(L.n), wd(L.n);
      for (int64_t i = 0; i < L.n; ++i) {
        for (int64_t u = L.ptr[i]; u < L.ptr[i + 1]; ++u)
          if (L.col[u] != i) {
            oc.push_back(L.col[u]);
            ov.push_back((float)L.val[u]);
          }
        op[i + 1] = (int32_t)oc.size();
        dg[i] = (float)L.diag(i);
        wd[i] = l < nl - 1 ? (float)((kOmega / rho[l]) / L.diag(i)) : 0.0f;
      }
      m.g_a = lanes(oc.size(), L.n);
      UPV(m.ptr, op);
      UPV(m.col, oc);
      UPV(m.val, ov);
      UPV(m.diag, dg);
      UPV(m.wdinv, wd);
      if ((s = dev_alloc(c, &m.r, (size_t)D * L.n))) return s;
      if ((s = dev_alloc(c, &m.z, (size_t)D * L.n))) return s;
      if (l < nl - 1 && (s = dev_alloc(c, &m.z2, (size_t)D * L.n))) return s;
    }
    if ((s = dev_alloc(c, &m.t, (size_t)D * L.n))) return s;
    if (l < nl - 1) {  // P with rows in this level's vector order (level 0: colour-major)
      const Csr& P = prolong[l];
      std::vector<int32_t> pp(L.n + 1, 0), pc;
      std::vector<float> pv;
      std::vector<int64_t> row_of(L.n);
      for (int64_t i = 0; i < L.n; ++i) row_of[l == 0 ? pos[i] : i] = i;
      for (int64_t k = 0; k < L.n; ++k) {
        const int64_t i = row_of[k];
        for (int64_t u = P.ptr[i]; u < P.ptr[i + 1]; ++u) {
          pc.push_back(P.col[u]);
          pv.push_back((float)P.val[u]);
        }
        pp[k + 1] = (int32_t)pc.size();
      }
      const Csr Pt = transpose(P, levels[l + 1].n);
      std::vector<int32_t> rp(Pt.ptr.size()), rc(Pt.col.size());
      for (size_t k = 0; k < Pt.ptr.size(); ++k) rp[k] = (int32_t)Pt.ptr[k];
      for (size_t k = 0; k < Pt.col.size(); ++k) rc[k] = l == 0 ? pos[Pt.col[k]] : Pt.col[k];
      m.g_p = lanes(pc.size(), L.n);
      m.g_r = lanes(rc.size(), levels[l + 1].n);
      UPV(m.p_ptr, pp);
      UPV(m.p_col, pc);
      UPV(m.p_val, pv);
      UPV(m.r_ptr, rp);
      UPV(m.r_col, rc);
      std::vector<float> rv = cast<float>(Pt.val);
      UPV(m.r_val, rv);
    } else {  // coarsest: dense inverse, stored column-major
      const int64_t n = L.n;
      std::vector<double> a(n * n, 0.0);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t u = L.ptr[i]; u < L.ptr[i + 1]; ++u) a[i * n + L.col[u]] = L.val[u];
      if (!invert(a, n)) return fail(c, HOFV_ESINGULAR, "singular coarsest multigrid level");
      std::vector<float> ci(n * n);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) ci[j * n + i] = (float)a[i * n + j];
      UPV(m.cinv, ci);
    }
  }
#undef UPV
  return HOFV_OK;
}

}  // namespace hofv
