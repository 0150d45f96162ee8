"""Stencil growth (Sec. 5's ill-conditioning study: a larger n+ restores the
least-squares systems that a structured node layout makes singular), applied
to the stencils that fail the pivot test.

A tensor-perturbed 12^3 grid (seed 7) at p = 3 has face stencils of 85 cells
whose centroids span too few distinct planes for the cubic terms."""
import numpy as np
import pytest

import workloads as w
from oracle import geometry as geo
from oracle import residual as rs
from oracle.lsq import SingularStencil, pivot_ok
from oracle.stencil import nearest

GROW = 10


def _mesh():
    return w.box_mesh((12, 12, 12), perturb=0.2, seed=7, mode="tensor")


@pytest.fixture(scope="module")
def grown():
    prob = w.poly_patch(_mesh(), 3, 3, seed=2)
    prob.stencil_grow = GROW
    return prob, rs.build(prob)


def test_the_mesh_fails_the_pivot_test_without_growth():
    with pytest.raises(SingularStencil):
        rs.build(w.poly_patch(_mesh(), 3, 3, seed=2))


def test_exactly_the_failing_stencils_grow_to_the_first_size_that_passes(grown):
    """Every internal-face stencil is the S nearest cells if those pass at all
    its points, else the S + k g nearest for the smallest k that passes."""
    prob, d = grown
    S = prob.stencil_size
    mesh = prob.mesh
    vol, cen = geo.cell_volume_centroid(mesh.verts[mesh.cells])
    faces = geo.enumerate_faces(mesh.cells, 3)
    fg = geo.face_geometry(mesh.verts, faces.verts, prob.n_gauss)
    fi = np.nonzero(faces.neigh >= 0)[0]
    nq = fg.qpts.shape[1]
    size = np.array([np.unique(r).size for r in d.f_st])
    assert set(np.unique(size)) <= {S + k * GROW for k in range(5)} and size.max() > S

    def passes(faces_idx, st):
        ok = pivot_ok(fg.qpts[fi[faces_idx]].reshape(-1, 3), np.repeat(cen[st], nq, axis=0), 3, prob.k_weight)
        return ok.reshape(len(faces_idx), nq).all(axis=1)

    base = nearest(fg.centre[fi], cen, S, prob.stencil_quantum)
    ok0 = passes(np.arange(fi.size), base)
    assert np.array_equal(ok0, size == S)  # grown iff the S-cell stencil fails
    same = size == S
    assert np.array_equal(np.sort(d.f_st[same][:, :S], axis=1), np.sort(base[same], axis=1))
    for s in np.unique(size[~same]):
        idx = np.nonzero(size == s)[0]
        st = nearest(fg.centre[fi[idx]], cen, s, prob.stencil_quantum)
        assert passes(idx, st).all()
        assert np.array_equal(np.sort(d.f_st[idx][:, :s], axis=1), np.sort(st, axis=1))
        prev = nearest(fg.centre[fi[idx]], cen, s - GROW, prob.stencil_quantum)
        assert not passes(idx, prev).any()  # one size smaller still fails


def test_padded_entries_carry_zero_coefficients(grown):
    prob, d = grown
    for st, C in ((d.f_st, d.f_C), (d.d_st, d.d_C)):
        size = np.array([np.unique(r).size for r in st])
        for i in np.nonzero(size < st.shape[1])[0][:50]:
            assert np.all(C[i, ..., size[i]:] == 0.0)
            assert np.all(st[i, size[i]:] == st[i, size[i] - 1])


def test_grown_stencils_reproduce_cubics(grown):
    """A full-rank stencil of any size reproduces polynomials of degree <= p,
    so R(u_exact) = 0 also where stencils grew (a nonzero padded coefficient or
    a misplaced ghost column would break it)."""
    prob, d = grown
    u = prob.loads.exact.value(d.cen)
    R = rs.residual(d, u)
    Ff, Fd = rs.face_fluxes(d, u)
    assert np.abs(R).max() <= 1e-11 * max(np.abs(Ff).max(), np.abs(Fd).max())
