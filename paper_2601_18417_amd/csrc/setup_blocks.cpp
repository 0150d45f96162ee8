// Item blocks for LDS-staged stencil gathers.
//
// The stencil kernels (face gradients, cell extrapolation) run one workgroup
// per block of consecutive items.  A workgroup first copies the union of its
// items' stencils (the block's cell list) from the gather copy of u into LDS,
// then reads every stencil value from LDS through a 16-bit position in that
// list.  Items are ordered along a Morton curve so that a block covers a
// compact patch of the mesh and its union stays small (each cell of it is
// used by many items of the block); a block is closed when it holds
// max_items items or when one more item would push its union past max_cells.
#include <algorithm>
#include <numeric>

#include "common.h"

namespace hofv {

namespace {

// spread the low 21 bits of x so that bit i lands on bit 3 i
uint64_t spread3(uint64_t x) {
  x &= 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffULL;
  x = (x | x << 16) & 0x1f0000ff0000ffULL;
  x = (x | x << 8) & 0x100f00f00f00f00fULL;
  x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
  x = (x | x << 2) & 0x1249249249249249ULL;
  return x;
}

// spread the low 31 bits of x so that bit i lands on bit 2 i
uint64_t spread2(uint64_t x) {
  x &= 0x7fffffff;
  x = (x | x << 16) & 0x0000ffff0000ffffULL;
  x = (x | x << 8) & 0x00ff00ff00ff00ffULL;
  x = (x | x << 4) & 0x0f0f0f0f0f0f0f0fULL;
  x = (x | x << 2) & 0x3333333333333333ULL;
  x = (x | x << 1) & 0x5555555555555555ULL;
  return x;
}

}  // namespace

std::vector<int64_t> morton_order(const double* pts, int D, int64_t n) {
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < D; ++d) {
    lo[d] = hi[d] = n ? pts[d] : 0.0;
    for (int64_t i = 1; i < n; ++i) {
      lo[d] = std::min(lo[d], pts[i * D + d]);
      hi[d] = std::max(hi[d], pts[i * D + d]);
    }
  }
  // one scale for every axis keeps the curve's cells cubic on stretched boxes
  double ext = 0;
  for (int d = 0; d < D; ++d) ext = std::max(ext, hi[d] - lo[d]);
  const double top = D == 3 ? 2097151.0 : 2147483647.0;
  const double sc = ext > 0 ? top / ext : 0.0;
  std::vector<uint64_t> key(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint64_t k = 0;
    for (int d = 0; d < D; ++d) {
      const uint64_t q = (uint64_t)std::min(top, std::max(0.0, (pts[i * D + d] - lo[d]) * sc));
      k |= (D == 3 ? spread3(q) : spread2(q)) << d;
    }
    key[i] = k;
  }
  std::vector<int64_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
  return order;
}

StencilBlocks make_blocks(const int32_t* st, int64_t n, int S, int64_t nc, int max_items, int max_cells) {
  StencilBlocks B;
  B.item.push_back(0);
  std::vector<int32_t> mark(nc, -1);
  int32_t blk = 0, count = 0, items = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* s = st + i * S;
    int fresh = 0;
    for (int k = 0; k < S; ++k) fresh += mark[s[k]] != blk;
    if (items > 0 && (items == max_items || count + fresh > max_cells)) {
      B.item.push_back((int32_t)i);
      ++blk;
      count = 0;
      items = 0;
    }
    for (int k = 0; k < S; ++k)
      if (mark[s[k]] != blk) {
        mark[s[k]] = blk;
        ++count;
      }
    ++items;
  }
  if (n > 0) B.item.push_back((int32_t)n);
  const int64_t nb = (int64_t)B.item.size() - 1;
  B.block_of.assign(n, 0);
  for (int64_t b = 0; b < nb; ++b)
    for (int64_t i = B.item[b]; i < B.item[b + 1]; ++i) B.block_of[i] = (int32_t)b;
  // per block: sorted union and the position of every stencil entry in it
  B.cell.assign(nb + 1, 0);
  B.local.assign((size_t)S * n, 0);
  std::vector<int32_t> pos(nc, -1);
  std::vector<int32_t> u;
  for (int64_t b = 0; b < nb; ++b) {
    u.clear();
    for (int64_t i = B.item[b]; i < B.item[b + 1]; ++i)
      for (int k = 0; k < S; ++k) {
        const int32_t cell = st[i * S + k];
        if (pos[cell] != -2) {
          pos[cell] = -2;
          u.push_back(cell);
        }
      }
    std::sort(u.begin(), u.end());
    for (size_t r = 0; r < u.size(); ++r) pos[u[r]] = (int32_t)r;
    for (int64_t i = B.item[b]; i < B.item[b + 1]; ++i)
      for (int k = 0; k < S; ++k) B.local[B.at(i, k, 0, 1, S)] = (uint16_t)pos[st[i * S + k]];
    for (int32_t cell : u) pos[cell] = -1;
    B.cells.insert(B.cells.end(), u.begin(), u.end());
    B.cell[b + 1] = (int32_t)B.cells.size();
    B.max_cells = std::max<int32_t>(B.max_cells, (int32_t)u.size());
  }
  return B;
}

}  // namespace hofv
