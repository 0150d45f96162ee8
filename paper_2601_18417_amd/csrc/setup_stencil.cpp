// Nearest-neighbour interpolation stencils (paper Sec. 3.5.2) by a uniform
// bin grid over the cell centroids.
//
// For a reference point x the stencil is the S cells of smallest
// key = (rint(d^2 / quantum), cell id), d^2 = ((dx*dx + dy*dy) + dz*dz).  The
// search grows a radius r until at least S centroids lie within r, gathering
// every centroid with d^2 <= r^2 + 2 quantum so that any cell tied (after
// quantisation) with the S-th one is among the candidates.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "common.h"

namespace hofv {

namespace {

struct Grid {
  int D;
  double lo[3], inv[3];
  int64_t n[3];
  std::vector<int64_t> start;  // bin -> first entry in ids
  std::vector<int32_t> ids;
};

Grid make_grid(const std::vector<double>& cen, int D, int64_t nc) {
  Grid g;
  g.D = D;
  double hi[3];
  for (int d = 0; d < D; ++d) {
    g.lo[d] = INFINITY;
    hi[d] = -INFINITY;
  }
  for (int64_t i = 0; i < nc; ++i)
    for (int d = 0; d < D; ++d) {
      g.lo[d] = std::min(g.lo[d], cen[i * D + d]);
      hi[d] = std::max(hi[d], cen[i * D + d]);
    }
  double vol = 1.0;
  for (int d = 0; d < D; ++d) vol *= std::max(hi[d] - g.lo[d], 1e-300);
  double cell = std::pow(vol / (double)nc, 1.0 / D);  // ~one centroid per bin
  int64_t total = 1;
  for (int d = 0; d < 3; ++d) {
    if (d < D) {
      g.n[d] = std::max<int64_t>(1, (int64_t)std::floor((hi[d] - g.lo[d]) / cell) + 1);
      g.inv[d] = g.n[d] / std::max(hi[d] - g.lo[d], 1e-300) * (1.0 - 1e-12);
    } else {
      g.n[d] = 1;
      g.inv[d] = 0;
      g.lo[d] = 0;
    }
    total *= g.n[d];
  }
  std::vector<int64_t> bin(nc);
  std::vector<int64_t> count(total + 1, 0);
  for (int64_t i = 0; i < nc; ++i) {
    int64_t b = 0;
    for (int d = D - 1; d >= 0; --d) {
      int64_t k = (int64_t)((cen[i * D + d] - g.lo[d]) * g.inv[d]);
      k = std::min<int64_t>(std::max<int64_t>(k, 0), g.n[d] - 1);
      b = b * g.n[d] + k;
    }
    bin[i] = b;
    count[b + 1]++;
  }
  for (int64_t b = 0; b < total; ++b) count[b + 1] += count[b];
  g.start = count;
  g.ids.resize(nc);
  std::vector<int64_t> fill(count.begin(), count.end() - 1);
  for (int64_t i = 0; i < nc; ++i) g.ids[fill[bin[i]]++] = (int32_t)i;  // ids ascending per bin
  return g;
}

}  // namespace

void nearest_cells(const std::vector<double>& cen, int D, int64_t nc, const double* pts, int64_t npts,
                   int S, double quantum, int32_t* out) {
  Grid g = make_grid(cen, D, nc);
  double binw = 0;
  for (int d = 0; d < D; ++d) binw = std::max(binw, 1.0 / g.inv[d]);
  double r0 = binw * std::pow((double)S, 1.0 / D) * 0.6;
#pragma omp parallel
  {
    struct Cand {
      double key;
      int32_t id;
      double d2;
    };
    std::vector<Cand> cand;
#pragma omp for schedule(dynamic, 256)
    for (int64_t q = 0; q < npts; ++q) {
      const double* x = pts + q * D;
      double r = r0;
      for (;;) {
        cand.clear();
        double r2 = r * r, rr = std::sqrt(r2 + 2.0 * quantum);
        int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int d = 0; d < D; ++d) {
          lo[d] = std::max<int64_t>(0, (int64_t)std::floor((x[d] - rr - g.lo[d]) * g.inv[d]));
          hi[d] = std::min<int64_t>(g.n[d] - 1, (int64_t)std::floor((x[d] + rr - g.lo[d]) * g.inv[d]));
        }
        int64_t inside = 0;
        for (int64_t k2 = lo[2]; k2 <= hi[2]; ++k2)
          for (int64_t k1 = lo[1]; k1 <= hi[1]; ++k1)
            for (int64_t k0 = lo[0]; k0 <= hi[0]; ++k0) {
              int64_t b = (k2 * g.n[1] + k1) * g.n[0] + k0;
              for (int64_t t = g.start[b]; t < g.start[b + 1]; ++t) {
                int32_t id = g.ids[t];
                const double* y = &cen[(size_t)id * D];
                double d2 = 0.0;
                for (int d = 0; d < D; ++d) {
                  double dd = y[d] - x[d];
                  d2 = d2 + dd * dd;
                }
                if (d2 <= r2 + 2.0 * quantum) {
                  cand.push_back({std::nearbyint(d2 / quantum), id, d2});
                  if (d2 <= r2) ++inside;
                }
              }
            }
        if (inside >= S || (int64_t)cand.size() >= nc) break;
        r *= 1.25;
      }
      std::sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
        return a.key != b.key ? a.key < b.key : a.id < b.id;
      });
      for (int k = 0; k < S; ++k) out[q * S + k] = cand[k].id;
    }
  }
}

}  // namespace hofv
