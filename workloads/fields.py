"""Manufactured displacement fields and the loads that go with them (inputs only).

A field gives u(x) and its exact partial derivatives.  The loads a problem
needs are evaluated from the exact field:

* body force of linear elasticity, f_b = -div(sigma(u)), with
  sigma = mu (grad u + grad u^T) + lambda (div u) I;
* traction on a boundary with outward normal n, t_j = sum_i n_i sigma_ij.

These are the manufactured-solution inputs of a problem, not part of the
finite-volume method, and are shared by the CPU oracle and the GPU library.
Derivative multi-indices are tuples (a, b[, c]).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np


def lame_from_young(E: float, nu: float):
    """Lame parameters (mu, lambda) from Young's modulus and Poisson's ratio."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


class Field:
    dim: int

    def deriv(self, x: np.ndarray, alpha) -> np.ndarray:
        """d^alpha u at points x (m, dim) -> (m, dim) (component-minor)."""
        raise NotImplementedError

    def value(self, x):
        return self.deriv(x, (0,) * self.dim)

    def grad(self, x):
        """G[m, i, j] = d u_j / d x_i."""
        out = np.empty((x.shape[0], self.dim, self.dim))
        for i in range(self.dim):
            a = [0] * self.dim
            a[i] = 1
            out[:, i, :] = self.deriv(x, tuple(a))
        return out

    def second(self, x, i, j):
        a = [0] * self.dim
        a[i] += 1
        a[j] += 1
        return self.deriv(x, tuple(a))


@dataclass
class TrigField(Field):
    """u_j = sum_t coef[t, j] * prod_d sin(k[t, d] x_d + phase[t, d])."""
    dim: int
    coef: np.ndarray   # (terms, dim)
    k: np.ndarray      # (terms, dim)
    phase: np.ndarray  # (terms, dim)

    def deriv(self, x, alpha):
        x = np.atleast_2d(np.asarray(x, float))
        out = np.zeros((x.shape[0], self.dim))
        for t in range(self.coef.shape[0]):
            prod = np.ones(x.shape[0])
            for d in range(self.dim):
                n = alpha[d]
                kk = self.k[t, d]
                prod = prod * (kk ** n) * np.sin(kk * x[:, d] + self.phase[t, d] + n * (math.pi / 2))
            out += prod[:, None] * self.coef[t][None, :]
        return out


    def lap_and_graddiv(self, x):
        """(lap u, grad div u) at x (m, dim), from each term's sin S_d and cos C_d
        of each coordinate: with P = prod_d S_d, d^2 P / dx_d^2 = -k_d^2 P and, for
        i != d, d^2 P / dx_i dx_d = k_i k_d C_i C_d prod_{e != i, d} S_e."""
        x = np.atleast_2d(np.asarray(x, float))
        D = self.dim
        lap = np.zeros((x.shape[0], D))
        gd = np.zeros((x.shape[0], D))
        for t in range(self.coef.shape[0]):
            k, a = self.k[t], self.coef[t]
            S, C = [], []
            for d in range(D):
                arg = k[d] * x[:, d] + self.phase[t, d]
                S.append(np.sin(arg))
                C.append(np.cos(arg))
            P = S[0]
            for d in range(1, D):
                P = P * S[d]
            lap -= float(np.sum(k * k)) * P[:, None] * a[None, :]
            for j in range(D):
                g = -(k[j] ** 2) * a[j] * P
                for d in range(D):
                    if d == j:
                        continue
                    term = (k[j] * k[d] * a[d]) * C[j] * C[d]
                    for e in range(D):
                        if e != j and e != d:
                            term = term * S[e]
                    g = g + term
                gd[:, j] += g
        return lap, gd


@dataclass
class PolyField(Field):
    """u_j = sum_m coef[m, j] * x^e[m, 0] * y^e[m, 1] (* z^e[m, 2])."""
    dim: int
    expo: np.ndarray  # (monomials, dim) int
    coef: np.ndarray  # (monomials, dim)

    def deriv(self, x, alpha):
        x = np.atleast_2d(np.asarray(x, float))
        out = np.zeros((x.shape[0], self.dim))
        for m in range(self.expo.shape[0]):
            prod = np.ones(x.shape[0])
            ok = True
            for d in range(self.dim):
                e, n = int(self.expo[m, d]), int(alpha[d])
                if n > e:
                    ok = False
                    break
                c = math.factorial(e) // math.factorial(e - n)
                prod = prod * c * x[:, d] ** (e - n)
            if ok:
                out += prod[:, None] * self.coef[m][None, :]
        return out


def symmetric_poly_field(dim: int, degree: int, seed: int, scale: float = 1.0) -> PolyField:
    """A random polynomial field symmetric about the plane x = 0: u_x odd in x,
    the other components even in x (its mirror image is itself)."""
    f = random_poly_field(dim, degree, seed, scale)
    odd = f.expo[:, 0] % 2 == 1
    coef = f.coef.copy()
    coef[~odd, 0] = 0.0
    coef[odd, 1:] = 0.0
    return PolyField(dim, f.expo, coef)


def random_poly_field(dim: int, degree: int, seed: int, scale: float = 1.0) -> PolyField:
    """All monomials of total degree <= degree, seeded N(0,1)*scale coefficients."""
    expo = [e for e in np.ndindex(*([degree + 1] * dim)) if sum(e) <= degree]
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal((len(expo), dim)) * scale
    return PolyField(dim, np.asarray(expo, int), coef)


@dataclass
class ZeroField(Field):
    dim: int

    def deriv(self, x, alpha):
        return np.zeros((np.atleast_2d(x).shape[0], self.dim))


def stress_le(G: np.ndarray, mu: float, lam: float) -> np.ndarray:
    """Small-strain stress from G[m, i, j] = du_j/dx_i (input helper for loads)."""
    dim = G.shape[-1]
    tr = np.trace(G, axis1=-2, axis2=-1)
    return mu * (G + np.swapaxes(G, -1, -2)) + lam * tr[..., None, None] * np.eye(dim)


def body_force_le(fld: Field, mu: float, lam: float, x: np.ndarray) -> np.ndarray:
    """f_b = -(mu lap u + (mu + lambda) grad div u) at x (m, dim)."""
    dim = fld.dim
    x = np.atleast_2d(x)
    if isinstance(fld, TrigField):  # the two contractions directly, chunks of points on threads
        f = np.empty((x.shape[0], dim))
        step = 1 << 20

        def chunk(a):
            lap, graddiv = fld.lap_and_graddiv(x[a:a + step])
            f[a:a + step] = -(mu * lap + (mu + lam) * graddiv)

        starts = range(0, x.shape[0], step)
        if len(starts) > 1:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
                list(ex.map(chunk, starts))
        else:
            for a in starts:
                chunk(a)
        return f
    f = np.zeros((x.shape[0], dim))
    for d in range(dim):
        f -= mu * fld.second(x, d, d)
    for j in range(dim):
        s = np.zeros(x.shape[0])
        for d in range(dim):
            s += fld.second(x, j, d)[:, d]
        f[:, j] -= (mu + lam) * s
    return f


def traction_le(fld: Field, mu: float, lam: float, x: np.ndarray, n: np.ndarray) -> np.ndarray:
    """t_j = sum_i n_i sigma_ij of the exact field."""
    sig = stress_le(fld.grad(np.atleast_2d(x)), mu, lam)
    return np.einsum("mi,mij->mj", np.atleast_2d(n), sig)


def mms_2d_unit() -> TrigField:
    """u = (sin(pi x) sin(pi y), cos(pi x) sin(pi y)) on the unit square."""
    pi = math.pi
    coef = np.array([[1.0, 0.0], [0.0, 1.0]])
    k = np.array([[pi, pi], [pi, pi]])
    phase = np.array([[0.0, 0.0], [pi / 2, 0.0]])
    return TrigField(2, coef, k, phase)


def mms_3d_trig(a=(2e-6, 4e-6, 6e-6)) -> TrigField:
    """u_i = a_i sin(4 pi x) sin(2 pi y) sin(pi z) (the 3D manufactured field)."""
    pi = math.pi
    coef = np.array([list(a)], float)
    k = np.array([[4 * pi, 2 * pi, pi]])
    phase = np.zeros((1, 3))
    return TrigField(3, coef, k, phase)


@dataclass
class Loads:
    """Everything a problem prescribes, as point functions.

    bc_type(xc, n) -> int array (0 = displacement, 1 = traction, 2 = symmetry plane)
    per boundary face.
    u_b(x) -> prescribed displacement; traction(x, n) -> prescribed traction;
    body(x) -> body force.  All take/return (m, dim) arrays.
    """
    dim: int
    bc_type: object
    u_b: object
    traction: object
    body: object
    exact: Field | None = None
    meta: dict = field(default_factory=dict)


DISP, TRAC, SYMM = 0, 1, 2


def mms_loads(fld: Field, mu: float, lam: float, traction_faces=None, symmetry_faces=None) -> Loads:
    """Manufactured problem: displacement BC everywhere except faces selected by
    ``traction_faces(xc, n) -> bool`` which get the exact traction, and faces
    selected by ``symmetry_faces`` (symmetry planes; the field must be symmetric
    about them)."""
    def bc_type(xc, n):
        t = np.full(xc.shape[0], DISP, np.int32)
        if traction_faces is not None:
            t[traction_faces(xc, n)] = TRAC
        if symmetry_faces is not None:
            t[symmetry_faces(xc, n)] = SYMM
        return t
    return Loads(fld.dim, bc_type, fld.value,
                 lambda x, n: traction_le(fld, mu, lam, x, n),
                 lambda x: body_force_le(fld, mu, lam, x), exact=fld)


def cantilever_loads(length: float, tip_traction) -> Loads:
    """Clamped at x = 0 (u = 0), dead-load traction on x = length, free elsewhere."""
    tip = np.asarray(tip_traction, float)
    dim = tip.shape[0]
    tol = 1e-9 * length

    def bc_type(xc, n):
        t = np.full(xc.shape[0], TRAC, np.int32)
        t[np.abs(xc[:, 0]) < tol] = DISP
        return t

    def traction(x, n):
        out = np.zeros((x.shape[0], dim))
        out[np.abs(x[:, 0] - length) < tol] = tip
        return out

    return Loads(dim, bc_type, lambda x: np.zeros((x.shape[0], dim)), traction,
                 lambda x: np.zeros((x.shape[0], dim)), exact=None,
                 meta={"tip_traction": tip.tolist()})
