"""Near-exact Jacobian (NEJ) preconditioner (paper App. C; its use in Sec. 5,
the comparison with the compact approximate Jacobian, Tables 1-2).

Test infrastructure (see package docstring).

For the linear elastic law the NEJ is the derivative of the discrete momentum
equations with the alpha-stabilisation term (Sec. 3.4) left out: the
face-point tractions of internal and displacement faces through the full face
stencils (a displacement face's ghost values are constants and go to the
right-hand side), the mirrored half stencils of symmetry faces with the
reflection R = I - 2 n n^T, and nothing from traction faces, whose loads are
constants too.  The residual is affine in u, so the NEJ is the Jacobian of the
residual built with alpha = 0, column j being R_0(e_j) - R_0(0).  With BDF2
dynamics the step's Jacobian adds -m_P on the diagonal.

Application: the paper assembles the NEJ and solves with it.  Here it is
applied by k iterations of GMRES from zero on A, right-preconditioned by a
fixed operator M (the compact approximate Jacobian's sweeps):
z = M(V_k y) with y minimising ||beta e_1 - H_k y||, V_k and H_k the Arnoldi
basis and Hessenberg matrix of A M from r.  The map r -> z is not linear, so
the outer solver must be the flexible one.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .jacobian import jacobian_affine


def discretisation(disc):
    """The discretisation without the stabilisation term (alpha = 0)."""
    return dataclasses.replace(disc, alpha=0.0)


def operator(disc, mass=None):
    """Dense NEJ, unknowns cell-major (index P * D + d); mass: m_P of BDF2."""
    A = jacobian_affine(discretisation(disc))
    if mass is not None:
        A -= np.diag(np.repeat(np.asarray(mass, float), disc.dim))
    return A


def gmres_fixed(A, r, k, M):
    """k GMRES iterations from zero on A z = r, right-preconditioned by M
    (callables on flat vectors); fewer if the Krylov space closes."""
    r = np.asarray(r, float).ravel()
    beta = np.linalg.norm(r)
    if beta == 0.0:
        return np.zeros_like(r)
    V = np.zeros((k + 1, r.size))
    H = np.zeros((k + 1, k))
    V[0] = r / beta
    kk = k
    for j in range(k):
        w = A(M(V[j]))
        for i in range(j + 1):  # Arnoldi, modified Gram-Schmidt
            H[i, j] = V[i] @ w
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:
            kk = j + 1
            break
        V[j + 1] = w / H[j + 1, j]
    e1 = np.zeros(kk + 1)
    e1[0] = beta
    y = np.linalg.lstsq(H[:kk + 1, :kk], e1, rcond=None)[0]
    return M(V[:kk].T @ y)
