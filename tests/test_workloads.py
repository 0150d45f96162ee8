"""Checks of the shared input generators (meshes, manufactured loads)."""
import numpy as np
import pytest

import workloads as w


def test_perturbation_bounds_and_fixed_boundary():
    m = w.box_mesh((6, 5, 4), perturb=0.2, seed=0)
    u = w.box_mesh((6, 5, 4))
    d = m.verts - u.verts
    h = np.asarray(u.spacing())
    assert np.all(np.abs(d) <= 0.2 * h + 1e-15)
    on_bnd = np.any(np.isclose(u.verts, 0) | np.isclose(u.verts, 1), axis=1)
    assert not np.any(d[on_bnd]) and np.all(np.abs(d[~on_bnd]).max(axis=1) > 0)
    again = w.box_mesh((6, 5, 4), perturb=0.2, seed=0)
    assert np.array_equal(m.verts, again.verts)


def _sympy_body_force(expr_u, mu, lam, pts):
    sp = pytest.importorskip("sympy")
    xs = sp.symbols("x0:%d" % len(expr_u))
    U = [e(xs, sp) for e in expr_u]
    D = len(U)
    G = [[sp.diff(U[j], xs[i]) for j in range(D)] for i in range(D)]
    div = sum(G[i][i] for i in range(D))
    sig = [[mu * (G[i][j] + G[j][i]) + (lam * div if i == j else 0) for j in range(D)] for i in range(D)]
    f = [-sum(sp.diff(sig[i][j], xs[i]) for i in range(D)) for j in range(D)]
    fn = sp.lambdify(xs, f, "numpy")
    return np.array([fn(*p) for p in pts], float)


def test_body_force_2d_matches_symbolic():
    mu, lam = w.lame_from_young(1.0, 0.3)
    fld = w.mms_2d_unit()
    pts = np.random.default_rng(0).uniform(0, 1, (7, 2))
    exprs = [lambda x, sp: sp.sin(sp.pi * x[0]) * sp.sin(sp.pi * x[1]),
             lambda x, sp: sp.cos(sp.pi * x[0]) * sp.sin(sp.pi * x[1])]
    ref = _sympy_body_force(exprs, mu, lam, pts)
    assert np.allclose(w.body_force_le(fld, mu, lam, pts), ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(fld.value(pts), np.stack([np.sin(np.pi * pts[:, 0]) * np.sin(np.pi * pts[:, 1]),
                                                 np.cos(np.pi * pts[:, 0]) * np.sin(np.pi * pts[:, 1])], 1))


def test_body_force_3d_matches_symbolic():
    mu, lam = w.lame_from_young(1.0, 0.3)
    a = (2e-6, 4e-6, 6e-6)
    fld = w.mms_3d_trig(a)
    pts = np.random.default_rng(1).uniform(0, 1, (5, 3))
    mk = lambda ai: (lambda x, sp: ai * sp.sin(4 * sp.pi * x[0]) * sp.sin(2 * sp.pi * x[1]) * sp.sin(sp.pi * x[2]))
    ref = _sympy_body_force([mk(ai) for ai in a], mu, lam, pts)
    got = w.body_force_le(fld, mu, lam, pts)
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_lame_parameters():
    mu, lam = w.lame_from_young(1.0, 0.3)
    assert mu == pytest.approx(1 / 2.6) and lam == pytest.approx(0.3 / (1.3 * 0.4))
