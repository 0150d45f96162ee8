"""Oracle pins on polygonal (2D) and polyhedral (3D) face-list meshes (Sec. 3.1:
faces cut into triangles by a fan, cells into simplices from an apex).

The meshes merge 2^dim fine cells of every other coarse block of a box into
one cell with 8 edges or 24 quadrilateral faces and hanging vertices."""
import numpy as np
import pytest

import workloads as w
from oracle import geometry as geo
from oracle import residual as rs
from workloads.meshes import split_block_mesh

CASES = [((4, 4), "random", 1), ((4, 4), "random", 2), ((5, 5), "random", 3),
         ((3, 3, 3), "tensor", 1), ((3, 3, 3), "tensor", 2), ((3, 3, 3), "tensor", 3)]


@pytest.mark.parametrize("cs,mode,p", CASES)
def test_polynomial_fields_give_zero_residual_on_polyhedra(cs, mode, p):
    """Degree <= p fields with their exact loads give R = 0 on planar-faced
    polygons and polyhedra (every 2D mesh; tensor-perturbed 3D); degree p + 1
    does not."""
    m = split_block_mesh(cs, perturb=0.2, seed=2, mode=mode)
    prob = w.poly_patch(m, p, p, seed=5)
    disc = rs.build(prob)
    u = prob.loads.exact.value(disc.cen)
    R = rs.residual(disc, u)
    Ff, Fd = rs.face_fluxes(disc, u)
    scale = max(np.abs(Ff).max(), np.abs(Fd).max())
    assert np.abs(R).max() <= 1e-12 * scale
    prob1 = w.poly_patch(m, p, p + 1, seed=6)
    disc1 = rs.build(prob1)
    R1 = rs.residual(disc1, prob1.loads.exact.value(disc1.cen))
    Ff1, _ = rs.face_fluxes(disc1, prob1.loads.exact.value(disc1.cen))
    assert np.abs(R1).max() > 1e-6 * np.abs(Ff1).max()


def test_merged_cells_have_their_faces_and_volumes():
    """Each merged 3D block is one cell of 24 faces; cells tile the box; on a
    tensor-perturbed grid a merged block is an axis-aligned box, so its
    centroid is the box centre although the mean of its 26 surface vertices is
    not, and every cell's vector areas sum to zero."""
    m = split_block_mesh((3, 3, 2), lengths=(1.0, 0.8, 0.6), perturb=0.2, seed=4, mode="tensor")
    own, nei, loops = geo.poly_faces(m)
    fg = geo.polygon_face_geometry(m.verts, loops, 2)
    vol, cen, pts, W, cof = geo.poly_cells(m, own, nei, loops, 3)
    deg = np.bincount(own, minlength=m.n_cells) + np.bincount(nei[nei >= 0], minlength=m.n_cells)
    assert set(np.unique(deg)) == {6, 24}
    assert vol.sum() == pytest.approx(0.48, rel=1e-14) and vol.min() > 0
    Wc = np.zeros(m.n_cells)
    np.add.at(Wc, cof, W)
    assert np.allclose(Wc, vol, rtol=1e-13)
    S = np.zeros((m.n_cells, 3))
    np.add.at(S, own, fg.area[:, None] * fg.normal)
    np.add.at(S, nei[nei >= 0], -(fg.area[:, None] * fg.normal)[nei >= 0])
    assert np.abs(S).max() <= 1e-14
    for c in np.nonzero(deg == 24)[0]:
        ids = np.unique(np.concatenate([loops[f] for f in np.nonzero((own == c) | (nei == c))[0]]))
        X = m.verts[ids]
        lo, hi = X.min(axis=0), X.max(axis=0)
        assert np.allclose(cen[c], 0.5 * (lo + hi), rtol=0, atol=1e-14)
        assert vol[c] == pytest.approx(np.prod(hi - lo), rel=1e-13)
    # the vertex mean differs from the centroid somewhere (the pin above can tell them apart)
    c = np.nonzero(deg == 24)[0][0]
    ids = np.unique(np.concatenate([loops[f] for f in np.nonzero((own == c) | (nei == c))[0]]))
    assert np.abs(m.verts[ids].mean(axis=0) - cen[c]).max() > 1e-3


def test_polygon_face_rule_integrates_exactly_and_orients_outward():
    """A pentagonal planar face: the fan rule integrates degree <= 2n - 1
    monomials exactly, its area is the polygon's, and reversing the loop
    reverses the normal while keeping points and weights."""
    th = np.linspace(0, 2 * np.pi, 6)[:-1]
    P = np.stack([np.cos(th) + 0.1 * np.sin(2 * th), np.sin(th), np.zeros(5)], axis=1)
    A = 0.5 * np.sum(P[:, 0] * np.roll(P[:, 1], -1) - np.roll(P[:, 0], -1) * P[:, 1])
    for n in (1, 2):
        g = geo.polygon_face_geometry(P, [np.arange(5)], n)
        assert g.area[0] == pytest.approx(A, rel=1e-14)
        assert np.allclose(g.normal[0], [0, 0, 1])
        g2 = geo.polygon_face_geometry(P, [np.arange(5)[::-1].copy()], n)
        assert np.allclose(g2.normal[0], [0, 0, -1])
        assert np.allclose(np.sort(g2.qw[0]), np.sort(g.qw[0]))
        # exact integrals of x^a y^b over the pentagon by its own fine triangulation
        ref = geo.polygon_face_geometry(P, [np.arange(5)], 6)
        for deg in range(2 * n):
            for a in range(deg + 1):
                f = lambda x: x[:, 0] ** a * x[:, 1] ** (deg - a)
                assert g.area[0] * np.sum(g.qw[0] * f(g.qpts[0])) == pytest.approx(
                    ref.area[0] * np.sum(ref.qw[0] * f(ref.qpts[0])), rel=1e-12, abs=1e-14)


def test_face_list_mesh_reproduces_the_hex_discretisation():
    """A face-list copy of a plain hex mesh (no block merged) gives the same
    residual as the hexahedral path with the fan face rule."""
    base = w.box_mesh((5, 5, 5), perturb=0.2, seed=7, mode="tensor")
    import workloads.meshes as wm
    own_fine = np.arange(base.n_cells)
    loops = wm._HEX_LOOPS
    fv = base.cells[:, loops].reshape(-1, 4)
    keys = np.sort(fv, axis=1)
    _, inv, cnt = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    first = np.full(cnt.size, -1)
    second = np.full(cnt.size, -1)
    for r in range(fv.shape[0]):
        if first[inv[r]] < 0:
            first[inv[r]] = r
        else:
            second[inv[r]] = r
    fc = np.stack([own_fine[first // 6], np.where(second >= 0, second // 6, -1)], axis=1)
    pm = wm.PolyMesh(3, base.verts, np.arange(first.size + 1) * 4, fv[first].reshape(-1), fc, base.n_cells,
                     base.shape, base.lengths, base.origin, own_fine)
    for p in (1, 2):
        ph = w.poly_patch(base, p, p + 1, seed=3)
        ph.face_rule = 1
        pp = w.poly_patch(pm, p, p + 1, seed=3)
        dh, dp = rs.build(ph), rs.build(pp)
        u = w.random_state(base.n_cells, 3, seed=8)
        Rh, Rp = rs.residual(dh, u), rs.residual(dp, u)
        assert np.abs(Rh - Rp).max() <= 1e-12 * np.abs(Rh).max()


@pytest.mark.parametrize("kind,p", [("tris", 1), ("tris", 2), ("tris", 3), ("tets", 1)])
def test_face_list_copy_of_simplices_reproduces_the_simplex_discretisation(kind, p):
    """Triangles and tetrahedra given as face lists match the simplex path to
    rounding where the face rules coincide: Gauss-Legendre edge rules are
    symmetric, and at p = 1 a triangle face has one point, its centroid.  (With
    more points a triangle face's conical-product rule depends on the vertex it
    starts from, which differs between the two paths: an equally exact rule,
    but the boundary constraints sit at its points.)"""
    base = (w.tri_mesh((5, 4), perturb=0.2, seed=2) if kind == "tris"
            else w.tet_mesh((3, 3, 3), perturb=0.15, seed=2))
    a = w.poly_patch(base, p, p + 1, seed=3)
    b = w.poly_patch(w.face_list_mesh(base), p, p + 1, seed=3)
    u = w.random_state(base.n_cells, base.dim, seed=8)
    Ra, Rb = rs.residual(rs.build(a), u), rs.residual(rs.build(b), u)
    assert np.abs(Ra - Rb).max() <= 1e-12 * np.abs(Ra).max()


@pytest.mark.parametrize("dim,p", [(3, 1), (3, 2), (2, 2), (2, 3)])
def test_polynomial_fields_give_zero_residual_around_a_cell_of_many_faces(dim, p):
    """A 3 x 3 x 3 block merged into one cell of 54 faces (tensor-perturbed, so
    its faces stay planar), or a 5 x 5 block into one of 20 edges: degree <= p
    fields still give R = 0, and the merged cell's volume is the block's."""
    if dim == 3:
        base = w.box_mesh((7, 7, 7), perturb=0.15, seed=5, mode="tensor")
        m = w.merged_block_mesh(base, (2, 2, 2), (5, 5, 5))
    else:
        base = w.box_mesh((9, 9), perturb=0.2, seed=5)
        m = w.merged_block_mesh(base, (2, 2), (7, 7))
    fc = m.face_cells
    nfaces = np.bincount(fc[fc >= 0], minlength=m.n_cells)
    assert nfaces.max() == (54 if dim == 3 else 20)
    prob = w.poly_patch(m, p, p, seed=5)
    disc = rs.build(prob)
    big = int(np.argmax(nfaces))
    vb, _ = geo.cell_volume_centroid(base.verts[base.cells])
    assert abs(disc.vol[big] - vb[m.fine_cell_of == big].sum()) <= 1e-13
    u = prob.loads.exact.value(disc.cen)
    R = rs.residual(disc, u)
    Ff, Fd = rs.face_fluxes(disc, u)
    assert np.abs(R).max() <= 1e-12 * max(np.abs(Ff).max(), np.abs(Fd).max())
