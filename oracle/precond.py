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


def assemble(disc_full, mass=None):
    """Sparse A (n_c x n_c) from a full (all-cells) discretisation; with the
    BDF2 inertia's m (oracle.dynamics) the diagonal gains -m_P, the Jacobian of
    its -m_P u_P."""
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
    if d.s_own is not None:
        # symmetry faces: the paper's term a_b (R_b - I) u_P = -2 a_b n n^T u_P acts
        # on the normal component only; one scalar matrix for every component
        # takes its isotropic average, -(2/3) a_b on the diagonal
        dPs = d.s_x - d.cen[d.s_own]
        a_s = d.kbar * d.s_area / np.abs(np.sum(dPs * d.s_n, axis=1))
        np.add.at(diag, d.s_own, -(2.0 / 3.0) * a_s)
    if mass is not None:
        diag = diag - mass
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


# ---- aggregation multigrid V-cycle on A -------------------------------------
# "A few sweeps" leaves the long-wavelength error of A untouched, which on a
# slender beam with free sides stalls the Krylov solver.  The multilevel
# application keeps the paper's matrix and its FP32 sweeps as the smoother
# and adds coarse corrections.  Definitions (the library implements the same
# rules independently):
#
# * strong neighbours of i on level l: j != i with |a_ij| >= theta_l sqrt(a_ii a_jj),
#   theta_l = THETA / 2^l (coarse operators spread their couplings over more
#   neighbours);
# * aggregation, nodes visited in index order:
#   1. i unassigned and all its strong neighbours unassigned -> new aggregate
#      {i} + strong(i);
#   2. i still unassigned -> joins the pass-1 aggregate of its strong
#      neighbour with the largest |a_ij| (values within a relative 1e-10 of
#      each other count as equal, and the smallest j wins), if any;
#   3. i still unassigned -> new aggregate {i} + its unassigned strong
#      neighbours;
#   aggregates are numbered in creation order;
# * tentative prolongation T[i, agg(i)] = 1, smoothed by one damped Jacobi
#   step, P = (I - OMEGA / rho D^-1 A_l) T with rho = max_i sum_j |a_ij| / |a_ii|
#   (a Gershgorin bound of the spectral radius of D^-1 A_l), A_{l+1} = P^T A_l P;
# * levels are added while the level has more than COARSE_SIZE nodes, at most
#   MAX_LEVELS, and while a coarsening keeps at most 80 % of the nodes;
# * smoother S_l: on the cell level s symmetric multicolour Gauss-Seidel sweeps
#   (the preconditioner's own sweeps); on coarser levels s damped Jacobi steps
#   z <- z + (OMEGA / rho_l) D^-1 (r - A_l z), rho_l the Gershgorin bound above;
# * V-cycle on level l < L-1: z = S_l(r) from 0, z += P V(P^T (r - A z)), then
#   S_l again from z; the last level is solved exactly.
THETA = 0.08
OMEGA = 4.0 / 3.0
COARSE_SIZE = 256
MAX_LEVELS = 8


def strong_neighbours(A, theta=THETA):
    A = A.tocsr()
    d = A.diagonal()
    out = []
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        keep = [(j, abs(v)) for j, v in zip(cols, vals)
                if j != i and abs(v) >= theta * np.sqrt(d[i] * d[j])]
        out.append(sorted(keep))
    return out


def aggregate(A, theta=THETA):
    """Aggregate index of every node (np.int64 array) and the number of aggregates."""
    n = A.shape[0]
    strong = strong_neighbours(A, theta)
    agg = np.full(n, -1, np.int64)
    k = 0
    for i in range(n):  # pass 1
        if agg[i] < 0 and all(agg[j] < 0 for j, _ in strong[i]):
            agg[i] = k
            for j, _ in strong[i]:
                agg[j] = k
            k += 1
    first = agg.copy()
    for i in range(n):  # pass 2
        if agg[i] >= 0:
            continue
        best, best_v = -1, -1.0
        for j, v in strong[i]:
            if first[j] >= 0 and v > best_v * (1.0 + 1e-10):
                best, best_v = j, v
        if best >= 0:
            agg[i] = first[best]
    for i in range(n):  # pass 3
        if agg[i] >= 0:
            continue
        agg[i] = k
        for j, _ in strong[i]:
            if agg[j] < 0:
                agg[j] = k
        k += 1
    return agg, k


def hierarchy(A):
    """List of levels: dicts with A, colours, and (except the last) agg, P."""
    levels = []
    A = A.tocsr()
    while True:
        lev = {"A": A, "colours": greedy_colours(A)}
        levels.append(lev)
        n = A.shape[0]
        if n <= COARSE_SIZE or len(levels) == MAX_LEVELS:
            break
        agg, nc = aggregate(A, THETA / 2 ** (len(levels) - 1))
        if nc > 0.8 * n:
            break
        T = sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nc))
        d = A.diagonal()
        rho = np.max(np.asarray(abs(A).sum(axis=1)).ravel() / np.abs(d))
        P = (T - (OMEGA / rho) * (sp.diags(1.0 / d) @ (A @ T))).tocsr()
        lev["agg"], lev["P"], lev["rho"] = agg, P, rho
        A = (P.T @ A @ P).tocsr()
    return levels


def _sweeps(A, colours, r, z, sweeps, dtype):
    diag = A.diagonal().astype(dtype)
    off = (A - sp.diags(A.diagonal())).tocsr().astype(dtype)
    n_col = int(colours.max()) + 1
    groups = [np.nonzero(colours == c)[0] for c in range(n_col)]
    rows = [off[g] for g in groups]
    order = list(range(n_col)) + list(range(n_col - 1, -1, -1))
    for _ in range(sweeps):
        for c in order:
            g = groups[c]
            z[g] = ((r[g] - rows[c] @ z) / diag[g][:, None]).astype(dtype)
    return z


def _jacobi(A, rho, r, z, steps, dtype):
    Ad = A.astype(dtype)
    wd = ((OMEGA / rho) / A.diagonal()).astype(dtype)
    for _ in range(steps):
        z = (z + wd[:, None] * (r - Ad @ z)).astype(dtype)
    return z


def _smooth(levels, level, r, z, sweeps, dtype):
    lev = levels[level]
    if level == 0:
        return _sweeps(lev["A"], lev["colours"], r, z, sweeps, dtype)
    return _jacobi(lev["A"], lev["rho"], r, z, sweeps, dtype)


def vcycle(levels, r, sweeps, dtype=np.float64, level=0):
    lev = levels[level]
    A = lev["A"]
    r = np.asarray(r).astype(dtype)
    if level == len(levels) - 1:
        return np.linalg.solve(A.toarray(), r.astype(np.float64)).astype(dtype)
    z = _smooth(levels, level, r, np.zeros_like(r), sweeps, dtype)
    res = (r - (A.astype(dtype) @ z)).astype(dtype)
    zc = vcycle(levels, (lev["P"].T.astype(dtype) @ res).astype(dtype), sweeps, dtype, level + 1)
    z = (z + lev["P"].astype(dtype) @ zc).astype(dtype)
    return _smooth(levels, level, r, z, sweeps, dtype)
