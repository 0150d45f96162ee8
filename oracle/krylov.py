"""Right-preconditioned flexible GMRES(m) (Saad 1993) with classical Gram-Schmidt
applied twice, or once (passes = 1: the orthogonalisation PETSc's GMRES uses
unless told otherwise, the library the paper's solver runs on).

Test infrastructure (see package docstring).  The paper solves J du = -R with
GMRES and a left preconditioner (eq. jfnk); right preconditioning in the
flexible variant is used here so that a preconditioner that changes between
iterations (FP32 sweeps, a learned correction) is admissible.  Stops when the
true residual ||b - A x|| <= rtol ||b|| (checked at every restart) or the
Arnoldi estimate of it is, or after ``maxit`` iterations.
"""
from __future__ import annotations

import numpy as np


STALL = 0.99  # a cycle that keeps more than this fraction of the residual ends the solve


def fgmres(A, b, M=None, x0=None, m=30, rtol=1e-8, maxit=1000, callback=None, stall=STALL, passes=2):
    """A, M: callables on flat float64 vectors.  Returns (x, info dict).

    The solve also ends (info["stalled"]) when a full cycle reduced the true
    residual, recomputed at the restart, by less than 1 % (stall = 0.99): a
    finite-difference product is linear only to its precision, and past the
    residual that precision allows more cycles change nothing."""
    b = np.asarray(b, float).ravel()
    n = b.size
    x = np.zeros(n) if x0 is None else np.asarray(x0, float).ravel().copy()
    M = M or (lambda v: v)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), {"iters": 0, "converged": True, "rel": 0.0}
    its = 0
    r = b - A(x)
    beta = np.linalg.norm(r)
    hist = [beta / bnorm]
    beta_prev = None
    while True:
        stalled = beta_prev is not None and beta > stall * beta_prev
        if beta <= rtol * bnorm or its >= maxit or stalled:
            return x, {"iters": its, "converged": beta <= rtol * bnorm, "rel": beta / bnorm,
                       "hist": hist, "stalled": bool(stalled and beta > rtol * bnorm)}
        beta_prev = beta
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = A(Z[j])
            h = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h
            if passes == 2:
                h2 = V[: j + 1] @ w
                w = w - V[: j + 1].T @ h2
                h = h + h2
            H[: j + 1, j] = h
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if callback:
                callback(its, abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= rtol * bnorm or its >= maxit:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        r = b - A(x)
        beta = np.linalg.norm(r)


def gmres_left(A, b, M, x0=None, m=30, rtol=1e-8, maxit=1000, stall=STALL, passes=2):
    """Left-preconditioned GMRES(m) (eq. jfnk as printed): minimises
    ||M (b - A x)|| over x0 + K_k(M A, M r0), classical Gram-Schmidt twice; stops
    when ||M (b - A x)|| <= rtol ||M b|| (recomputed at every restart), after
    ``maxit`` iterations, or when a cycle keeps more than ``stall`` of that
    residual.  M must be a fixed linear operator.  Returns (x, info dict)."""
    b = np.asarray(b, float).ravel()
    n = b.size
    x = np.zeros(n) if x0 is None else np.asarray(x0, float).ravel().copy()
    bnorm = np.linalg.norm(M(b))
    if bnorm == 0.0:
        return np.zeros(n), {"iters": 0, "converged": True, "rel": 0.0, "hist": [0.0], "stalled": False}
    its, beta_prev, hist = 0, None, []
    while True:
        r = M(b - A(x))
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        stalled = beta_prev is not None and beta > stall * beta_prev
        if beta <= rtol * bnorm or its >= maxit or stalled:
            return x, {"iters": its, "converged": beta <= rtol * bnorm, "rel": beta / bnorm, "hist": hist,
                       "stalled": bool(stalled and beta > rtol * bnorm)}
        beta_prev = beta
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = M(A(V[j]))
            for _ in range(passes):
                h = V[: j + 1] @ w
                w = w - V[: j + 1].T @ h
                H[: j + 1, j] += h
            H[j + 1, j] = np.linalg.norm(w)
            its += 1
            k = j + 1
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            # least-squares residual of this Krylov space
            e1 = np.zeros(k + 1)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[: k + 1, :k], e1, rcond=None)
            res = np.linalg.norm(e1 - H[: k + 1, :k] @ y)
            if res <= rtol * bnorm or its >= maxit or H[j + 1, j] == 0.0:
                break
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[: k + 1, :k], e1, rcond=None)
        x = x + V[:k].T @ y
