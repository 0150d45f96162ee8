"""Weighted least-squares Taylor reconstruction, "LRE" (paper Sec. 3.5.1, App. B).

Test infrastructure (see package docstring).

For an expansion point x~ and its stencil S the truncated Taylor expansion of
order p (eq. te) is written with the scaled basis of App. B,

    q(x - x~) = [ prod_d ((x_d - x~_d)/h)^{e_d} / e_d! ]  over |e| <= p,

h = 2 r_s with r_s the largest |x_N - x~| in S.  Minimising the weighted sum of
squares (eq. ls) with the weight function of eq. weightFunc (shape k) gives
a~ = A~ u with A~ = M^{-1} Q W (eqs. maQw, lsA).  It is not formed from the normal
equations: B = diag(sqrt(w)) Q^T is factorised by Householder QR (numpy's
LAPACK geqrf), B = Q_h R, and A~ = R^{-1} Q_h^T diag(sqrt(w)).  Row e of A~ then
gives h^{|e|} d^e u(x~); it is divided by h^{|e|} to return physical
derivatives.

A displacement-boundary quadrature point adds one ghost node co-located with
x~: basis row [1, 0, ..., 0] and weight ``ghost_weight`` (Sec. 3.5.3); it does
not change r_s.
"""
from __future__ import annotations

import math

import numpy as np


def exponents(dim: int, p: int):
    """Multi-indices of the Taylor basis, by degree, then x-power, then y-power
    descending: 3D degree 3 gives xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz
    (the order of the third-order coefficient vector of App. B)."""
    out = []
    for deg in range(p + 1):
        if dim == 2:
            for a in range(deg, -1, -1):
                out.append((a, deg - a))
        else:
            for a in range(deg, -1, -1):
                for b in range(deg - a, -1, -1):
                    out.append((a, b, deg - a - b))
    return out


def weight(dt: np.ndarray, k: float) -> np.ndarray:
    """Eq. weightFunc: w = (exp(-dt^2 k^2) - exp(-k^2)) / (1 - exp(-k^2))."""
    return (np.exp(-(dt ** 2) * k * k) - math.exp(-k * k)) / (1.0 - math.exp(-k * k))


class SingularStencil(ValueError):
    pass


def _weighted_qr(xt, Xs, p, k, ghost_weight):
    """QR of the weighted scaled-Taylor system W^(1/2) Q (eqs. maQw, weightFunc)."""
    m, S, D = Xs.shape
    E = exponents(D, p)
    dx = Xs - xt[:, None, :]
    dist = np.sqrt(np.sum(dx * dx, axis=2))
    r_s = dist.max(axis=1)
    h = 2.0 * r_s
    w = weight(dist / h[:, None], k)
    Q = np.empty((m, S, len(E)))
    for c, e in enumerate(E):
        col = np.ones((m, S))
        for d in range(D):
            col = col * (dx[:, :, d] / h[:, None]) ** e[d] / math.factorial(e[d])
        Q[:, :, c] = col
    if ghost_weight is not None:
        g = np.zeros((m, 1, len(E)))
        g[:, 0, 0] = 1.0
        Q = np.concatenate([Q, g], axis=1)
        w = np.concatenate([w, np.full((m, 1), float(ghost_weight))], axis=1)
    sw = np.sqrt(w)
    Qh, R = np.linalg.qr(sw[:, :, None] * Q, mode="reduced")
    return Qh, R, sw, h, E


def pivot_ok(xt: np.ndarray, Xs: np.ndarray, p: int, k: float, ghost_weight: float | None = None,
             pivot_tol: float = 1e-14) -> np.ndarray:
    """Per point: does the stencil pass the pivot test min|R_ii| > tol max|R_ii|?"""
    _, R, _, _, _ = _weighted_qr(xt, Xs, p, k, ghost_weight)
    diag = np.abs(np.diagonal(R, axis1=1, axis2=2))
    return diag.min(axis=1) > pivot_tol * diag.max(axis=1)


def reconstruction(xt: np.ndarray, Xs: np.ndarray, p: int, k: float,
                   ghost_weight: float | None = None, pivot_tol: float = 1e-14):
    """Batched LS reconstruction.

    xt: (m, D) expansion points; Xs: (m, S, D) stencil centroids.
    Returns (A, cond): A is (m, N_t, S [+1 ghost column]) with row e giving the
    physical derivative d^e u(x~) as a combination of the stencil values (and the
    ghost value last); cond = max|R_ii| / min|R_ii| per point.
    """
    Qh, R, sw, h, E = _weighted_qr(xt, Xs, p, k, ghost_weight)
    diag = np.abs(np.diagonal(R, axis1=1, axis2=2))
    if np.any(diag.min(axis=1) <= pivot_tol * diag.max(axis=1)):
        raise SingularStencil("rank-deficient least-squares stencil")
    cond = diag.max(axis=1) / diag.min(axis=1)
    A = np.linalg.solve(R, np.swapaxes(Qh, 1, 2)) * sw[:, None, :]
    for c, e in enumerate(E):
        A[:, c, :] /= h[:, None] ** sum(e)
    return A, cond


def row_index(dim: int, p: int):
    """Map multi-index -> row of A."""
    return {e: i for i, e in enumerate(exponents(dim, p))}
