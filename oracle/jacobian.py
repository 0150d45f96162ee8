"""Jacobian-vector products and brute-force Jacobians (paper Sec. 4.1).

Test infrastructure (see package docstring).

* J v ~ (R(u + eps v) - R(u)) / eps with the perturbation
  eps = sqrt((1 + ||u||_2) eps_mach) / ||v||_2 (the paper only calls eps a small
  scalar; this is the rule of the JFNK survey it cites) and J v = 0 for v = 0.
* Brute force: linear elasticity is affine in u, so column j of J is
  R(e_j) - R(0) exactly; the neo-Hookean residual is analytic in u, so column j
  is Im R(u + i h e_j) / h with h = 1e-30 (complex step).
"""
from __future__ import annotations

import numpy as np

from .residual import residual

EPS_MACH = np.finfo(np.float64).eps


def default_eps(u, v):
    nv = float(np.linalg.norm(np.ravel(v)))
    if nv == 0.0:
        return 0.0
    return float(np.sqrt((1.0 + np.linalg.norm(np.ravel(u))) * EPS_MACH) / nv)


def jvp(disc, u, v, Ru=None, eps=None, load=1.0):
    if eps is None:
        eps = default_eps(u, v)
    if eps == 0.0:
        return np.zeros_like(np.asarray(v, float))
    if Ru is None:
        Ru = residual(disc, u, load)
    return (residual(disc, u + eps * v, load) - Ru) / eps


def jacobian_affine(disc, load=1.0):
    """Dense J of an affine residual, columns R(e_j) - R(0), unknowns cell-major."""
    n, D = disc.n_cells, disc.dim
    R0 = residual(disc, np.zeros((n, D)), load)
    J = np.empty((n * D, n * D))
    for j in range(n * D):
        e = np.zeros(n * D)
        e[j] = 1.0
        J[:, j] = (residual(disc, e.reshape(n, D), load) - R0).ravel()
    return J


def jacobian_complex_step(disc, u, load=1.0, h=1e-30):
    """Dense J of an analytic residual at u by the complex step."""
    n, D = disc.n_cells, disc.dim
    J = np.empty((n * D, n * D))
    base = np.asarray(u, float).astype(np.complex128).ravel()
    for j in range(n * D):
        x = base.copy()
        x[j] += 1j * h
        J[:, j] = residual(disc, x.reshape(n, D), load).imag.ravel() / h
    return J
