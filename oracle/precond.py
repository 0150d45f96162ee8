"""Compact-stencil approximate Jacobian (AJ) and its sweeps (paper Sec. 4.1).

Test infrastructure (see package docstring).

The AJ of cell P is the central-difference diffusion operator

    P_P(u) = sum_{f int} Kbar |Delta_f| (u_N - u_P) / |d_PN| Gamma_f
           + sum_{b disp} Kbar |Delta_b| (ubar_b - u_P) / |d_Pb| Gamma_b,
    Delta_f = d_PN / (d_PN . n_f),  Kbar = 2 mu + lambda,

without non-orthogonal correction.  |Delta_f| / |d_PN| = 1 / |d_PN . n_f|, and
every block is a multiple of the identity, so the matrix acts on each
displacement component with the same scalar matrix A:

    A_PN = Kbar Gamma_f / |d_PN . n_f|,   A_PP = -sum of those over internal
    faces - sum_{b disp} Kbar Gamma_b / |d_Pb . n_b|.

The boundary value ubar_b is a constant and drops out of the Jacobian.

Application: "a few sweeps" is read as s symmetric multicolour Gauss-Seidel
sweeps on A z = r from z = 0: colours in increasing order, then decreasing,
each cell set z_P = (r_P - sum_N A_PN z_N) / A_PP.  Colours are greedy in cell
id order (smallest colour not used by a lower-id neighbour).  ``dtype`` selects
the arithmetic (float64, or float32 to emulate the FP32 sweeps).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def assemble(disc_full):
    """Sparse A (n_c x n_c) from a full (all-cells) discretisation."""
    d = disc_full
    n = d.n_cells
    dPN = d.cen[d.f_nei] - d.cen[d.f_own]
    a = d.kbar * d.f_area / np.abs(np.sum(dPN * d.f_n, axis=1))
    dPb = d.d_x - d.cen[d.d_own]
    ab = d.kbar * d.d_area / np.abs(np.sum(dPb * d.d_n, axis=1))
    rows = np.concatenate([d.f_own, d.f_nei])
    cols = np.concatenate([d.f_nei, d.f_own])
    vals = np.concatenate([a, a])
    diag = np.zeros(n)
    np.add.at(diag, d.f_own, -a)
    np.add.at(diag, d.f_nei, -a)
    np.add.at(diag, d.d_own, -ab)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A = A + sp.diags(diag)
    return A.tocsr()


def greedy_colours(A):
    n = A.shape[0]
    col = np.full(n, -1, np.int64)
    indptr, indices = A.indptr, A.indices
    for P in range(n):
        used = {col[N] for N in indices[indptr[P]:indptr[P + 1]] if N != P and col[N] >= 0}
        c = 0
        while c in used:
            c += 1
        col[P] = c
    return col


def sgs(A, colours, r, sweeps, dtype=np.float64):
    """s symmetric multicolour Gauss-Seidel sweeps for A z = r, z0 = 0.

    r is (n, D); the same scalar matrix acts on every column.  Cells of one
    colour are not coupled, so each colour is updated as one block.
    """
    A = A.tocsr()
    diag = A.diagonal().astype(dtype)
    off = (A - sp.diags(A.diagonal())).tocsr().astype(dtype)
    r = np.asarray(r).astype(dtype)
    z = np.zeros_like(r)
    n_col = int(colours.max()) + 1
    groups = [np.nonzero(colours == c)[0] for c in range(n_col)]
    rows = [off[g] for g in groups]
    order = list(range(n_col)) + list(range(n_col - 1, -1, -1))
    for _ in range(sweeps):
        for c in order:
            g = groups[c]
            z[g] = ((r[g] - rows[c] @ z) / diag[g][:, None]).astype(dtype)
    return z
