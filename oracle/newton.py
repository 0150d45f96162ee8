"""Jacobian-free Newton-Krylov driver (paper Sec. 4.1, Sec. 5 solver settings).

Test infrastructure (see package docstring).

For every load increment i = 1..n (load factor i/n):
    R0 = R(u);  repeat  J(u) du = -R(u) by FGMRES with J v from finite
    differences and the AJ sweeps as right preconditioner;  backtracking line
    search lam = 1, 1/2, 1/4, ... (at most ``ls_max`` halvings) accepting the
    first ||R(u + lam du)|| <= (1 - 1e-4 lam) ||R(u)|| (or the last trial);
    until ||R|| <= tol ||R0||.  The Krylov tolerance is ``eta`` (forcing 0) or
    the Eisenstat-Walker term of ``forcing_term`` starting from ``eta``
    (forcing 1).  ``inertia`` = (m, s) adds a BDF2 time step's inertia to R
    and -m to the approximate Jacobian's diagonal (oracle.dynamics).  side 1
    solves each Newton system by left-preconditioned GMRES (eq. jfnk as
    printed) instead of right-preconditioned FGMRES.
    predictor 1 starts increment i+1 from u_i + (u_i - u_{i-1})
    (a secant in the load factor; not in the paper) when R there is finite,
    R0 staying that of u_i at the new load.  ls_max < 0: full steps, lam halved (at most
    10 times) only while R(u + lam du) is not finite (an inverted cell makes
    the neo-Hookean ln J undefined).
The paper defers its line search to the authors' earlier work without
details and reduces the residual by six orders; the Armijo backtracking, the
full-step mode and the tolerances here are readings (tolerance per problem,
Krylov rtol ``eta``).
"""
from __future__ import annotations

import numpy as np

from . import precond
from .jacobian import default_eps
from .krylov import fgmres, gmres_left
from .residual import residual


def forcing_term(rn, rprev, eta_prev, eta_max, tol, r0):
    """Eisenstat & Walker (1996), choice 2 with gamma = 0.9, alpha = 2: the
    Krylov tolerance follows the observed reduction of ||R||, raised to
    gamma eta_prev^alpha when that exceeds 0.1 (their safeguard), capped at
    eta_max, and not below 0.5 tol ||R0|| / ||R|| (no more than the
    increment's tolerance needs)."""
    e = 0.9 * (rn / rprev) ** 2
    if 0.9 * eta_prev ** 2 > 0.1:
        e = max(e, 0.9 * eta_prev ** 2)
    return max(min(e, eta_max), 0.5 * tol * r0 / rn)


def newton(disc, u0, A=None, colours=None, sweeps=2, tol=1e-8, eta=1e-4, m=30,
           maxit_newton=50, maxit_krylov=2000, n_increments=1, ls_max=10, precond_fn=None,
           log=None, forcing=0, predictor=0, inertia=None, load_scale=1.0, side=0, passes=2):
    n, D = disc.n_cells, disc.dim
    if A is None:
        A = precond.assemble(disc, None if inertia is None else inertia[0])
    if colours is None:
        colours = precond.greedy_colours(A)
    u = np.asarray(u0, float).copy()
    stats = {"newton": 0, "krylov": 0, "increments": []}

    def M(v):
        if precond_fn is not None:
            return precond_fn(v.reshape(n, D)).ravel()
        return precond.sgs(A, colours, v.reshape(n, D), sweeps).ravel()

    u_prev = u.copy()
    for inc in range(1, n_increments + 1):
        load = load_scale * inc / n_increments
        R = residual(disc, u, load, inertia)
        r0 = np.linalg.norm(R)
        rn = r0
        if predictor == 1 and inc > 1:
            u_pred = u + (u - u_prev)
            u_prev = u
            with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
                R_pred = residual(disc, u_pred, load, inertia)
            if np.all(np.isfinite(R_pred)):
                u, R, rn = u_pred, R_pred, np.linalg.norm(R_pred)
        elif predictor == 1:
            u_prev = u.copy()
        it = 0
        eta_k, rprev = eta, r0
        while rn > tol * r0 and it < maxit_newton:
            if forcing == 1 and it > 0:
                eta_k = forcing_term(rn, rprev, eta_k, eta, tol, r0)
            rprev = rn
            Ru = R
            uu = u

            def J(v):
                vv = v.reshape(n, D)
                eps = default_eps(uu, vv)
                if eps == 0.0:
                    return np.zeros_like(v)
                return ((residual(disc, uu + eps * vv, load, inertia) - Ru) / eps).ravel()

            if side == 1:
                du, info = gmres_left(J, -R.ravel(), M, m=m, rtol=eta_k, maxit=maxit_krylov, passes=passes)
            else:
                du, info = fgmres(J, -R.ravel(), M, m=m, rtol=eta_k, maxit=maxit_krylov, passes=passes)
            stats["krylov"] += info["iters"]
            du = du.reshape(n, D)
            lam = 1.0
            full = ls_max < 0
            for _ in range((10 if full else ls_max) + 1):
                ut = u + lam * du
                with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
                    Rt = residual(disc, ut, load, inertia)
                finite = bool(np.all(np.isfinite(Rt)))
                if finite and (full or np.linalg.norm(Rt) <= (1.0 - 1e-4 * lam) * rn):
                    break
                lam *= 0.5
            u, R = ut, Rt
            rn = np.linalg.norm(R)
            it += 1
            stats["newton"] += 1
            if log:
                log(inc, it, rn / r0, info["iters"], lam)
        stats["increments"].append({"load": load, "newton": it, "rel": rn / r0 if r0 else 0.0, "r0": r0})
    return u, stats
