"""Pins of the oracle's geometry, stencils and least-squares reconstruction.

Each check is against something the mathematics fixes (exact volumes of boxes,
closed surfaces, exact polynomial reproduction, brute-force sorting), not
against the oracle's own formulas.
"""
import math

import numpy as np
import pytest

import workloads as w
from oracle import geometry as geo
from oracle import lsq
from oracle.stencil import n_terms, nearest


@pytest.mark.parametrize("shape", [(4, 3), (3, 4, 2)])
def test_uniform_cells_are_boxes(shape):
    mesh = w.box_mesh(shape, lengths=(2.0,) * len(shape))
    vol, cen = geo.cell_volume_centroid(mesh.verts[mesh.cells])
    h = np.asarray(mesh.spacing())
    assert np.allclose(vol, np.prod(h), rtol=1e-14)
    ijk = w.cell_ijk(mesh)
    assert np.allclose(cen, (ijk + 0.5) * h, atol=1e-14)


@pytest.mark.parametrize("shape", [(5, 4), (4, 3, 5)])
def test_perturbed_mesh_volume_and_closed_cells(shape):
    mesh = w.box_mesh(shape, perturb=0.2, seed=7)
    X = mesh.verts[mesh.cells]
    vol, cen = geo.cell_volume_centroid(X)
    assert abs(vol.sum() - 1.0) < 1e-13          # boundary vertices are fixed
    faces = geo.enumerate_faces(mesh.cells, mesh.dim)
    fg = geo.face_geometry(mesh.verts, faces.verts, 2)
    Sv = fg.area[:, None] * fg.normal
    closure = np.zeros((mesh.n_cells, mesh.dim))
    np.add.at(closure, faces.owner, Sv)
    inner = faces.neigh >= 0
    np.add.at(closure, faces.neigh[inner], -Sv[inner])
    assert np.abs(closure).max() < 1e-14        # sum of outward vector areas = 0
    # divergence theorem: sum_f S_f . x_f over a cell = D * volume for planar
    # faces; for bilinear faces use the exact first moment via quadrature
    assert np.allclose(fg.qw.sum(axis=1), 1.0)
    # every owner normal points away from the owner centroid
    assert np.all(np.sum((fg.centre - cen[faces.owner]) * fg.normal, axis=1) > 0)
    n_int = np.count_nonzero(inner)
    nx = shape
    if mesh.dim == 2:
        expect = (nx[0] - 1) * nx[1] + nx[0] * (nx[1] - 1)
    else:
        expect = ((nx[0] - 1) * nx[1] * nx[2] + nx[0] * (nx[1] - 1) * nx[2]
                  + nx[0] * nx[1] * (nx[2] - 1))
    assert n_int == expect


def test_gauss_rule_exactness():
    for n in (1, 2, 3, 5):
        t, wt = geo.gauss_01(n)
        for deg in range(2 * n):
            assert abs(np.sum(wt * t ** deg) - 1.0 / (deg + 1)) < 1e-15


def test_planar_face_centre_is_polygon_centroid():
    # a planar non-parallelogram quad in the z=0 plane
    verts = np.array([[0, 0, 0], [2, 0, 0], [1.5, 1, 0], [0.2, 1.3, 0]], float)
    fg = geo.face_geometry(verts, np.array([[0, 1, 2, 3]]), 2)
    x, y = verts[:, 0], verts[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cr = x * yn - xn * y
    A = cr.sum() / 2
    cx = ((x + xn) * cr).sum() / (6 * A)
    cy = ((y + yn) * cr).sum() / (6 * A)
    assert abs(fg.area[0] - A) < 1e-14
    assert np.allclose(fg.centre[0], [cx, cy, 0.0], atol=1e-14)
    assert np.allclose(fg.normal[0], [0, 0, 1])


def test_stencil_matches_brute_force_sort():
    mesh = w.box_mesh((7, 6, 5), perturb=0.2, seed=3)
    _, cen = geo.cell_volume_centroid(mesh.verts[mesh.cells])
    rng = np.random.default_rng(0)
    pts = rng.uniform(0, 1, (20, 3))
    st = nearest(pts, cen, 30, 1e-12)
    for r in range(pts.shape[0]):
        d2 = np.sum((cen - pts[r]) ** 2, axis=1)
        assert set(st[r]) == set(np.argsort(d2)[:30])


def test_stencil_ties_break_by_cell_id():
    mesh = w.box_mesh((7, 7, 7))
    _, cen = geo.cell_volume_centroid(mesh.verts[mesh.cells])
    P = 3 + 7 * 3 + 49 * 3  # centre cell
    st = nearest(cen[[P]], cen, 49, 1e-6 / 49)[0]
    h2 = 1.0 / 49
    d2 = np.rint(np.sum((cen[st] - cen[P]) ** 2, axis=1) / h2).astype(int)
    # shells d^2 = 0,1,2,3,4 hold 1+6+12+8+6 = 33 cells; 16 of the 24 at d^2 = 5
    assert [np.count_nonzero(d2 == s) for s in range(6)] == [1, 6, 12, 8, 6, 16]
    shell5 = np.nonzero(np.rint(np.sum((cen - cen[P]) ** 2, axis=1) / h2) == 5)[0]
    assert sorted(st[d2 == 5]) == sorted(shell5)[:16]


def test_weight_function_values():
    assert lsq.weight(np.array([0.0]), 6.0)[0] == pytest.approx(1.0, rel=1e-15, abs=0)
    # at the stencil radius (d~ = 1/2) the weight is (e^-9 - e^-36)/(1 - e^-36),
    # 1.2340980408644762e-4 (e^-9 = 1.2340980408667956e-4, e^-36 = 2.3195228e-16)
    assert lsq.weight(np.array([0.5]), 6.0)[0] == pytest.approx(1.2340980408644762e-4, rel=1e-14, abs=0)
    assert lsq.weight(np.array([1.0]), 6.0)[0] == pytest.approx(0.0, abs=1e-16)


def test_basis_order_matches_paper_listing():
    e3 = lsq.exponents(3, 3)
    names = ["".join("x" * a + "y" * b + "z" * c) for a, b, c in e3 if a + b + c == 3]
    assert names == ["xxx", "xxy", "xxz", "xyy", "xyz", "xzz", "yyy", "yyz", "yzz", "zzz"]
    assert len(lsq.exponents(2, 3)) == n_terms(2, 3) == 10
    assert len(lsq.exponents(3, 2)) == n_terms(3, 2) == 10


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
@pytest.mark.parametrize("ghost", [False, True])
def test_reconstruction_reproduces_polynomials(dim, p, ghost):
    """Derivatives of any polynomial of degree <= p are exact (LS exactness)."""
    shape = (9, 9) if dim == 2 else (6, 6, 6)
    mesh = w.box_mesh(shape, perturb=0.2, seed=11)
    _, cen = geo.cell_volume_centroid(mesh.verts[mesh.cells])
    S = n_terms(dim, p) + (10 if dim == 2 else {1: 45, 2: 55, 3: 65}[p])
    rng = np.random.default_rng(5)
    xt = rng.uniform(0.3, 0.7, (6, dim))
    st = nearest(xt, cen, S, 1e-9)
    fld = w.random_poly_field(dim, p, seed=2)
    A, cond = lsq.reconstruction(xt, cen[st], p, 6.0, 1.0 if ghost else None)
    vals = fld.value(cen[st].reshape(-1, dim)).reshape(6, S, dim)
    if ghost:
        vals = np.concatenate([vals, fld.value(xt)[:, None, :]], axis=1)
    for r, e in enumerate(lsq.exponents(dim, p)):
        got = np.einsum("ms,msj->mj", A[:, r, :], vals)
        exact = fld.deriv(xt, e)
        assert np.allclose(got, exact, rtol=1e-9, atol=1e-9 * (1 + np.abs(exact).max())), e


def test_reconstruction_invariances():
    rng = np.random.default_rng(1)
    Xs = rng.uniform(-1, 1, (1, 30, 3))
    xt = np.zeros((1, 3))
    A, _ = lsq.reconstruction(xt, Xs, 2, 6.0)
    perm = rng.permutation(30)
    Ap, _ = lsq.reconstruction(xt, Xs[:, perm], 2, 6.0)
    assert np.allclose(Ap, A[:, :, perm], rtol=1e-11, atol=1e-12)
    s = 0.01
    As, _ = lsq.reconstruction(xt, s * Xs, 2, 6.0)
    for r, e in enumerate(lsq.exponents(3, 2)):
        assert np.allclose(As[0, r], A[0, r] / s ** sum(e), rtol=1e-10, atol=1e-10 * np.abs(A[0, r]).max() / s ** sum(e))


def test_rank_deficient_stencil_raises():
    xs = np.stack([np.linspace(-1, 1, 12), np.zeros(12)], axis=1)[None]  # collinear
    with pytest.raises(lsq.SingularStencil):
        lsq.reconstruction(np.zeros((1, 2)), xs, 2, 6.0)


def test_reconstruction_equals_normal_equations():
    """A~ = M^{-1} Q W with M = Q W Q^T (eq. maQw) built directly from the
    paper's definitions of the scaled basis and the weights, by a dense solve."""
    rng = np.random.default_rng(4)
    Xs = rng.uniform(-1, 1, (1, 25, 2))
    xt = np.array([[0.1, -0.2]])
    p, k = 3, 6.0
    A, _ = lsq.reconstruction(xt, Xs, p, k)
    dx = Xs[0] - xt[0]
    d = np.hypot(dx[:, 0], dx[:, 1])
    h = 2 * d.max()
    wts = (np.exp(-(d / h) ** 2 * k * k) - np.exp(-k * k)) / (1 - np.exp(-k * k))
    basis = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]
    Q = np.array([[(x / h) ** a * (y / h) ** b / (math.factorial(a) * math.factorial(b))
                   for (x, y) in dx] for (a, b) in basis])
    W = np.diag(wts)
    Abar = np.linalg.solve(Q @ W @ Q.T, Q @ W)
    for r, (a, b) in enumerate(basis):
        assert np.allclose(A[0, r], Abar[r] / h ** (a + b), rtol=1e-7, atol=1e-7 * np.abs(Abar[r]).max() / h ** (a + b))
