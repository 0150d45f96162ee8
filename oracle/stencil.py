"""Nearest-neighbour interpolation stencils (paper Sec. 3.5.2).

Test infrastructure (see package docstring).  The stencil of a reference point
(a face centre x_f, or a cell centroid x_P) is the |S| = N_t + n+ cells whose
centroids are closest to it.  The paper does not say how equal distances are
ordered; on uniform meshes the cut-off almost always splits an equidistant
shell, so the order must be exact.  Reading used here: the sort key is
(rint(d^2 / quantum), cell id) with d^2 = dx*dx + dy*dy (+ dz*dz), i.e. squared
distances closer than about one quantum count as equal and the lower cell id
wins.  The quantum is a problem input (1e-6 h_min^2 for the named problems).
"""
from __future__ import annotations

import numpy as np


def n_terms(dim: int, p: int) -> int:
    """N_t = (d+p)! / (d! p!), the size of the Taylor basis (Sec. 3.5.2)."""
    return (p + 1) * (p + 2) // 2 if dim == 2 else (p + 1) * (p + 2) * (p + 3) // 6


def nearest(points: np.ndarray, centroids: np.ndarray, size: int, quantum: float,
            chunk: int | None = None) -> np.ndarray:
    """Stencil (m, size) of cell ids for every reference point (m, D), brute force
    (in chunks of points whose distance rows take about 400 MB)."""
    m = points.shape[0]
    n = centroids.shape[0]
    if chunk is None:
        chunk = max(1, min(256, 50_000_000 // max(n, 1)))
    if size > n:
        raise ValueError(f"stencil size {size} exceeds the number of cells {n}")
    ids = np.arange(n, dtype=np.int64)
    out = np.empty((m, size), np.int64)
    for s in range(0, m, chunk):
        p = points[s:s + chunk]
        d2 = np.zeros((p.shape[0], n))
        for a in range(p.shape[1]):
            diff = centroids[None, :, a] - p[:, a, None]
            d2 = d2 + diff * diff
        key = np.rint(d2 / quantum)
        for r in range(p.shape[0]):
            # every cell with a key below the size-th smallest key is in; the
            # cells tied at that key are taken in increasing id order
            kth = np.partition(key[r], size - 1)[size - 1]
            cand = np.nonzero(key[r] <= kth)[0]
            order = cand[np.lexsort((ids[cand], key[r][cand]))]
            out[s + r] = order[:size]
    return out
