"""Pins of the oracle on triangular and tetrahedral meshes (Sec. 3.1 geometry
and quadrature on simplices; the paper's triangular and tetrahedral cases of
Sec. 5)."""
import math

import numpy as np
import pytest

import workloads as w
from oracle import geometry as geo
from oracle import jacobian as jc
from oracle import residual as rs


def _simplex_moment(e):
    """Integral of prod x_i^e_i over the unit simplex: prod e_i! / (sum e + D)!."""
    return math.prod(math.factorial(k) for k in e) / math.factorial(sum(e) + len(e))


@pytest.mark.parametrize("n", [1, 2, 3])
def test_triangle_rule_degree(n):
    """The n x n conical product on the triangle (0,0,0), (1,0,0), (0,1,0) is
    exact for every monomial x^a y^b of degree <= 2n - 1 and not for all of
    degree 2n."""
    tri = np.array([[[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0]]])
    g = geo.face_geometry(tri[0], np.array([[0, 1, 2]]), n)
    assert g.area[0] == pytest.approx(0.5)
    assert np.allclose(g.normal[0], [0, 0, 1])
    x, y = g.qpts[0, :, 0], g.qpts[0, :, 1]
    for deg in range(2 * n + 1):
        errs = []
        for a in range(deg + 1):
            q = g.area[0] * np.sum(g.qw[0] * x ** a * y ** (deg - a))
            errs.append(abs(q - _simplex_moment((a, deg - a))))
        if deg <= 2 * n - 1:
            assert max(errs) <= 1e-15
        else:
            assert max(errs) > 1e-8


@pytest.mark.parametrize("n", [2, 3, 4])
def test_triangle_cell_rule_degree(n):
    """The 2D cell rule on the unit triangle is exact to degree 2n - 1 and not
    beyond; a sheared triangle gets its determinant area and vertex-mean
    centroid."""
    X = np.array([[[0.0, 0], [1.0, 0], [0.0, 1]]])
    pts, W = geo.cell_quadrature(X, n)
    for deg in range(2 * n + 1):
        errs = [abs(np.sum(W[0] * pts[0, :, 0] ** a * pts[0, :, 1] ** (deg - a)) - _simplex_moment((a, deg - a)))
                for a in range(deg + 1)]
        if deg <= 2 * n - 1:
            assert max(errs) <= 1e-15
        else:
            assert max(errs) > 1e-9
    Y = np.array([[[0.3, 0.1], [2.0, 0.4], [0.5, 1.7]]])
    vol, cen = geo.cell_volume_centroid(Y)
    pts, W = geo.cell_quadrature(Y, n)
    assert vol[0] == pytest.approx(0.5 * np.linalg.det(np.stack([Y[0, 1] - Y[0, 0], Y[0, 2] - Y[0, 0]])), rel=1e-14)
    assert W.sum() == pytest.approx(vol[0], rel=1e-14)
    assert np.allclose(np.einsum("q,qd->d", W[0], pts[0]) / W.sum(), cen[0], rtol=1e-14)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_tet_rule_degree(n):
    """The cell rule on the unit tetrahedron is exact to degree 2n - 1 and not
    beyond; on a sheared tetrahedron it integrates 1 and x to volume and
    volume times centroid."""
    X = np.array([[[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0], [0.0, 0, 1]]])
    pts, W = geo.cell_quadrature(X, n)
    for deg in range(2 * n + 1):
        errs = []
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                c = deg - a - b
                q = np.sum(W[0] * pts[0, :, 0] ** a * pts[0, :, 1] ** b * pts[0, :, 2] ** c)
                errs.append(abs(q - _simplex_moment((a, b, c))))
        if deg <= 2 * n - 1:
            assert max(errs) <= 1e-15
        else:
            assert max(errs) > 1e-9
    Y = np.array([[[0.3, 0.1, 0], [2.0, 0.4, 0.2], [0.5, 1.7, 0.1], [0.2, 0.6, 1.4]]])
    vol, cen = geo.cell_volume_centroid(Y)
    pts, W = geo.cell_quadrature(Y, n)
    det = np.linalg.det(np.stack([Y[0, 1] - Y[0, 0], Y[0, 2] - Y[0, 0], Y[0, 3] - Y[0, 0]]))
    assert vol[0] == pytest.approx(det / 6.0, rel=1e-14)
    assert W.sum() == pytest.approx(vol[0], rel=1e-14)
    assert np.allclose(np.einsum("q,qd->d", W[0], pts[0]) / W.sum(), cen[0], rtol=1e-14)


def test_tet_mesh_invariants():
    """Kuhn split of a perturbed box: positive volumes summing to the box, each
    cell's outward vector areas summing to zero, every interior triangle shared
    by exactly two tetrahedra and the boundary made of 2 triangles per square."""
    mesh = w.tet_mesh((4, 3, 5), lengths=(2.0, 1.0, 1.5), perturb=0.2, seed=7)
    X = mesh.verts[mesh.cells]
    vol, _ = geo.cell_volume_centroid(X)
    assert vol.min() > 0 and vol.sum() == pytest.approx(3.0, rel=1e-13)
    faces = geo.enumerate_faces(mesh.cells, 3)
    g = geo.face_geometry(mesh.verts, faces.verts, 1)
    S = g.normal * g.area[:, None]
    net = np.zeros((mesh.n_cells, 3))
    np.add.at(net, faces.owner, S)
    inner = faces.neigh >= 0
    np.add.at(net, faces.neigh[inner], -S[inner])
    assert np.abs(net).max() <= 1e-14
    assert np.count_nonzero(~inner) == 2 * 2 * (4 * 3 + 3 * 5 + 4 * 5)
    assert mesh.n_cells == 6 * 60


def test_tri_mesh_invariants():
    mesh = w.tri_mesh((5, 4), lengths=(2.0, 1.0), perturb=0.2, seed=7)
    X = mesh.verts[mesh.cells]
    vol, _ = geo.cell_volume_centroid(X)
    assert vol.min() > 0 and vol.sum() == pytest.approx(2.0, rel=1e-13)
    faces = geo.enumerate_faces(mesh.cells, 2)
    g = geo.face_geometry(mesh.verts, faces.verts, 1)
    S = g.normal * g.area[:, None]
    net = np.zeros((mesh.n_cells, 2))
    np.add.at(net, faces.owner, S)
    inner = faces.neigh >= 0
    np.add.at(net, faces.neigh[inner], -S[inner])
    assert np.abs(net).max() <= 1e-14
    assert np.count_nonzero(~inner) == 2 * (5 + 4)
    assert mesh.n_cells == 2 * 20


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("perturb", [0.0, 0.2])
def test_polynomial_fields_give_zero_residual_on_triangles(p, perturb):
    prob = w.poly_patch(w.tri_mesh((8, 8), perturb=perturb, seed=3), p, p, seed=5)
    disc = rs.build(prob)
    R = rs.residual(disc, prob.loads.exact.value(disc.cen))
    Ff, Fd = rs.face_fluxes(disc, prob.loads.exact.value(disc.cen))
    assert np.abs(R).max() <= 1e-12 * max(np.abs(Ff).max(), np.abs(Fd).max())


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("perturb", [0.0, 0.2])
def test_polynomial_fields_give_zero_residual_on_tets(p, perturb):
    """Flat faces: the reconstruction reproduces degree-p fields and the face
    and volume rules integrate their stress and body force exactly, so the
    residual of the exact field vanishes on regular and irregular tetrahedra."""
    prob = w.poly_patch(w.tet_mesh((4, 4, 4), perturb=perturb, seed=3), p, p, seed=5)
    disc = rs.build(prob)
    R = rs.residual(disc, prob.loads.exact.value(disc.cen))
    Ff, Fd = rs.face_fluxes(disc, prob.loads.exact.value(disc.cen))
    scale = max(np.abs(Ff).max(), np.abs(Fd).max())
    assert np.abs(R).max() <= 1e-12 * scale


def test_degree_above_p_leaves_a_residual_on_tets():
    prob = w.poly_patch(w.tet_mesh((4, 4, 4), perturb=0.2, seed=3), 1, 2, seed=5)
    disc = rs.build(prob)
    R = rs.residual(disc, prob.loads.exact.value(disc.cen))
    Ff, _ = rs.face_fluxes(disc, prob.loads.exact.value(disc.cen))
    assert np.abs(R).max() > 1e-4 * np.abs(Ff).max()


@pytest.mark.parametrize("n", [1, 2])
def test_fan_rule_on_a_planar_quadrilateral(n):
    """Fan rule (the paper's face subdivision): on a planar trapezoid it
    integrates every monomial of degree <= 2n - 1 exactly, whichever vertex
    carries the lowest id, and the points do not depend on where the cyclic
    vertex list starts."""
    verts = np.array([[0.0, 0, 0], [2.0, 0, 0], [1.5, 1, 0], [0.5, 1, 0]])
    exact = lambda a, b: sum(((2.0 - 0.5 * y) ** (a + 1) - (0.5 * y) ** (a + 1)) / (a + 1) * y ** b * wy
                             for y, wy in zip(*geo.gauss_01(8)))
    for ids in ([0, 1, 2, 3], [2, 3, 0, 1]):
        g = geo.face_geometry(verts, np.array([ids]), n, fan=True)
        assert g.area[0] == pytest.approx(1.5)
        x, y = g.qpts[0, :, 0], g.qpts[0, :, 1]
        for deg in range(2 * n):
            for a in range(deg + 1):
                q = g.area[0] * np.sum(g.qw[0] * x ** a * y ** (deg - a))
                assert q == pytest.approx(exact(a, deg - a), rel=1e-13, abs=1e-14)
    g0 = geo.face_geometry(verts, np.array([[0, 1, 2, 3]]), 2, fan=True)
    g1 = geo.face_geometry(verts, np.array([[1, 2, 3, 0]]), 2, fan=True)
    assert np.allclose(g0.qpts, g1.qpts) and np.allclose(g0.qw, g1.qw)


@pytest.mark.parametrize("order", [[0, 1, 2, 3], [1, 2, 3, 0], [3, 2, 1, 0]])
def test_fan_rule_area_of_a_warped_quadrilateral(order):
    """Sec. 3.1 takes the face area as the sum of its sub-triangle areas.  The
    face (0,0,0), (1,0,0), (1,1,z), (0,1,0) is cut from vertex 0 into two
    triangles of area sqrt(1+z^2)/2 each, so Gamma = sqrt(1+z^2), while its
    vector area (-z, -z, 2)/2 has length sqrt(1+z^2/2); the normal stays
    that vector's direction."""
    z = 0.5
    verts = np.array([[0.0, 0, 0], [1.0, 0, 0], [1.0, 1, z], [0.0, 1, 0]])
    g = geo.face_geometry(verts, np.array([order]), 2, fan=True)
    assert g.area[0] == pytest.approx(np.sqrt(1 + z * z), rel=1e-14)
    sgn = 1.0 if order[1] == (order[0] + 1) % 4 else -1.0
    assert np.allclose(g.normal[0], sgn * np.array([-z, -z, 2.0]) / np.sqrt(2 * z * z + 4), rtol=1e-14)
    assert g.qw[0].sum() == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_polynomial_fields_give_zero_residual_with_the_fan_rule(p):
    prob = w.poly_patch(w.box_mesh((5, 5, 5), perturb=0.2, seed=3, mode="tensor"), p, p, seed=5)
    prob.face_rule = 1
    disc = rs.build(prob)
    assert disc.f_qw.shape[1] == 2 * prob.n_gauss ** 2
    u = prob.loads.exact.value(disc.cen)
    R = rs.residual(disc, u)
    Ff, Fd = rs.face_fluxes(disc, u)
    assert np.abs(R).max() <= 1e-12 * max(np.abs(Ff).max(), np.abs(Fd).max())


@pytest.mark.parametrize("p,min_slope", [(1, 1.9), (2, 1.5), (3, 3.5)])
def test_oracle_converges_on_regular_triangles(p, min_slope):
    """The 2D manufactured problem on 8^2 and 16^2 quads split into triangles,
    solved exactly (the linear law's residual is affine): the centroid RMS
    error against the manufactured field falls at the scheme's rate (observed
    2.11, 1.66 and 4.08 at p = 1, 2, 3)."""
    errs = []
    for n in (8, 16):
        prob = w.tri_mms(n, p, perturb=0.0)
        disc = rs.build(prob)
        J = jc.jacobian_affine(disc)
        R0 = rs.residual(disc, np.zeros((disc.n_cells, 2)))
        u = -np.linalg.solve(J, R0.ravel()).reshape(-1, 2)
        ue = prob.loads.exact.value(disc.cen)
        errs.append(np.sqrt(np.mean(np.sum((u - ue) ** 2, axis=1))))
    assert np.log(errs[0] / errs[1]) / np.log(2.0) >= min_slope
