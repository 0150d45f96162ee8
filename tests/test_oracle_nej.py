"""Pins of the oracle's near-exact Jacobian (App. C) and its inner GMRES."""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as w
from oracle import jacobian as jc
from oracle import krylov as kr
from oracle import nej
from oracle import precond as pc
from oracle import residual as rs


def _div_stress(fld, mu, lam, x):
    """div sigma of the linear elastic law from the field's second derivatives:
    (div sigma)_i = mu sum_j (u_i,jj + u_j,ij) + lam sum_k u_k,ki."""
    D = fld.dim
    d2 = {}
    for a, b in itertools.product(range(D), repeat=2):
        alpha = [0] * D
        alpha[a] += 1
        alpha[b] += 1
        d2[a, b] = fld.deriv(x, alpha)  # (n, D): d^2 u / dx_a dx_b
    out = np.zeros((x.shape[0], D))
    for i in range(D):
        for j in range(D):
            out[:, i] += mu * (d2[j, j][:, i] + d2[i, j][:, j]) + lam * d2[j, i][:, j]
    return out


def _interior(disc):
    cnt = np.bincount(np.concatenate([disc.f_own, disc.f_nei]), minlength=disc.n_cells)
    return np.nonzero(cnt == 2 * disc.dim)[0]


@pytest.mark.parametrize("mesh", [lambda: w.box_mesh((7, 7), perturb=0.2, seed=3),
                                  lambda: w.box_mesh((5, 5, 5), perturb=0.2, seed=3, mode="tensor")])
def test_nej_of_a_quadratic_field_is_the_divergence_of_its_stress(mesh):
    """A p = 2 reconstruction is exact for quadratic fields and the face Gauss
    rule for their linear stress, so on a cell with only internal faces the
    NEJ row is the closed-face integral of sigma . n, i.e. Omega_P div sigma
    (divergence theorem), with no stabilisation contribution."""
    prob = w.poly_patch(mesh(), 2, 2, seed=5)
    disc = rs.build(prob)
    A = nej.operator(disc)
    fld = w.random_poly_field(disc.dim, 2, seed=11)
    u = fld.value(disc.cen)
    Au = (A @ u.ravel()).reshape(disc.n_cells, disc.dim)
    ref = disc.vol[:, None] * _div_stress(fld, disc.mu, disc.lam, disc.cen)
    cells = _interior(disc)
    assert cells.size >= 8
    assert np.abs(Au[cells] - ref[cells]).max() <= 1e-9 * np.abs(ref[cells]).max()


def test_nej_differs_from_the_jacobian_by_the_stabilisation_only():
    """J(alpha) = NEJ + alpha S with S independent of alpha and non-zero; S
    vanishes on degree-p polynomials at cells with only internal faces (the
    two reconstructions at a face agree for them)."""
    prob = w.cube_mms(5, 2, perturb=0.2)
    disc = rs.build(prob)
    A = nej.operator(disc)
    a = disc.alpha
    assert a > 0
    J1 = jc.jacobian_affine(disc)
    J2 = jc.jacobian_affine(nej.dataclasses.replace(disc, alpha=2 * a))
    S1, S2 = (J1 - A) / a, (J2 - A) / (2 * a)
    assert np.abs(S1).max() > 1e-3 * np.abs(A).max()
    assert np.abs(S1 - S2).max() <= 1e-10 * np.abs(S1).max()
    fld = w.random_poly_field(3, 2, seed=12)
    Su = (S1 @ fld.value(disc.cen).ravel()).reshape(disc.n_cells, 3)
    cells = _interior(disc)
    assert cells.size >= 1
    assert np.abs(Su[cells]).max() <= 1e-9 * np.abs(S1).max() * np.abs(fld.value(disc.cen)).max()


def test_nej_rows_couple_the_union_of_the_face_stencils():
    """Row P of the NEJ couples only the cells of the stencils of P's faces (the
    "substantially larger stencil" of App. C), many more than the compact
    approximate Jacobian's face neighbours."""
    prob = w.cube_mms(5, 2, perturb=0.2)
    disc = rs.build(prob)
    A = nej.operator(disc)
    n, D = disc.n_cells, disc.dim
    blocks = np.abs(A).reshape(n, D, n, D).max(axis=(1, 3)) > 0
    union = [set() for _ in range(n)]
    for f in range(disc.f_own.size):
        s = set(disc.f_st[f][disc.f_st[f] >= 0].tolist())
        union[disc.f_own[f]] |= s
        union[disc.f_nei[f]] |= s
    for f in range(disc.d_own.size):
        union[disc.d_own[f]] |= set(disc.d_st[f][disc.d_st[f] >= 0].tolist())
    AJ = pc.assemble(disc)
    for P in range(n):
        cols = set(np.nonzero(blocks[P])[0].tolist())
        assert cols <= union[P]
        assert len(cols) >= 3 * AJ[P].nnz


def test_gmres_fixed_closed_forms():
    """One iteration with M = I is the minimal-residual step z = (r.Ar / |Ar|^2) r;
    n iterations solve an n x n system exactly; r = 0 gives 0."""
    rng = np.random.default_rng(4)
    n = 12
    A = rng.standard_normal((n, n)) + 6 * np.eye(n)
    r = rng.standard_normal(n)
    I = lambda v: v
    Ar = A @ r
    z1 = nej.gmres_fixed(lambda v: A @ v, r, 1, I)
    assert np.allclose(z1, (r @ Ar) / (Ar @ Ar) * r, rtol=1e-13, atol=0)
    zn = nej.gmres_fixed(lambda v: A @ v, r, n, I)
    assert np.allclose(zn, np.linalg.solve(A, r), rtol=1e-9, atol=1e-12)
    Dg = np.diag(A).copy()
    zp = nej.gmres_fixed(lambda v: A @ v, r, n, lambda v: v / Dg)
    assert np.allclose(zp, np.linalg.solve(A, r), rtol=1e-9, atol=1e-12)
    assert not np.any(nej.gmres_fixed(lambda v: A @ v, np.zeros(n), 3, I))


def test_nej_preconditioner_needs_fewer_iterations_than_the_compact_one():
    """The direction of Table 1 at p = 3 on regular hexahedra: with the NEJ
    solved exactly, FGMRES on the full J converges in fewer iterations than
    with the compact approximate Jacobian's sweeps."""
    prob = w.cube_mms(5, 3, perturb=0.0)
    disc = rs.build(prob)
    J = jc.jacobian_affine(disc)
    lu = sla.lu_factor(nej.operator(disc))
    n = disc.n_cells
    AJ = pc.assemble(disc)
    col = pc.greedy_colours(AJ)
    b = w.random_state(n, 3, seed=9, scale=1.0).ravel()
    Jm = lambda v: J @ v
    _, i_nej = kr.fgmres(Jm, b, lambda v: sla.lu_solve(lu, v), rtol=1e-8, maxit=400)
    _, i_aj = kr.fgmres(Jm, b, lambda v: pc.sgs(AJ, col, v.reshape(n, 3), 2).ravel(), rtol=1e-8, maxit=400)
    assert i_nej["converged"] and i_aj["converged"]
    assert i_nej["iters"] < i_aj["iters"]


def test_nej_preconditioner_loses_on_irregular_tetrahedra():
    """The direction of Table 2: on irregular tetrahedra the exactly solved NEJ
    needs more FGMRES iterations than the compact approximate Jacobian's
    sweeps (without the alpha-term the operator keeps the poorly damped modes
    that irregular cells excite)."""
    prob = w.tet_mms(3, 2, perturb=0.2)
    disc = rs.build(prob)
    J = jc.jacobian_affine(disc)
    lu = sla.lu_factor(nej.operator(disc))
    n = disc.n_cells
    AJ = pc.assemble(disc)
    col = pc.greedy_colours(AJ)
    b = w.random_state(n, 3, seed=9, scale=1.0).ravel()
    Jm = lambda v: J @ v
    _, i_nej = kr.fgmres(Jm, b, lambda v: sla.lu_solve(lu, v), rtol=1e-8, maxit=600)
    _, i_aj = kr.fgmres(Jm, b, lambda v: pc.sgs(AJ, col, v.reshape(n, 3), 2).ravel(), rtol=1e-8, maxit=600)
    assert i_nej["converged"] and i_aj["converged"]
    assert i_nej["iters"] > 2 * i_aj["iters"]


def test_nej_on_symmetry_plane_cells_is_the_divergence_of_the_stress():
    """App. C's symmetry-face part: the mirrored half stencil reproduces a
    quadratic field symmetric about the plane, so cells whose faces are all
    internal or on the plane also get Omega_P div sigma."""
    mesh = w.box_mesh((6, 5, 5), perturb=0.2, seed=4, mode="tensor")
    prob = w.poly_patch(mesh, 2, 2, seed=6, symmetric=True)
    disc = rs.build(prob)
    assert disc.s_own is not None and disc.s_own.size > 0
    A = nej.operator(disc)
    fld = w.fields.symmetric_poly_field(3, 2, seed=13)
    u = fld.value(disc.cen)
    Au = (A @ u.ravel()).reshape(disc.n_cells, 3)
    ref = disc.vol[:, None] * _div_stress(fld, disc.mu, disc.lam, disc.cen)
    cnt = np.bincount(np.concatenate([disc.f_own, disc.f_nei, disc.s_own]), minlength=disc.n_cells)
    cells = np.intersect1d(np.nonzero(cnt == 6)[0], disc.s_own)
    assert cells.size >= 4
    assert np.abs(Au[cells] - ref[cells]).max() <= 1e-9 * np.abs(ref[cells]).max()


@pytest.mark.parametrize("mk", [lambda: w.cube_mms(5, 2, perturb=0.0), lambda: w.tet_mms(3, 2, perturb=0.2)])
def test_nej_weakest_mode_is_a_checkerboard(mk):
    """Without the alpha-term the weakest mode of the operator alternates in
    sign across most faces and is much weaker than the full Jacobian's, whose
    weakest mode is smooth: the stabilisation exists to damp such modes."""
    disc = rs.build(mk())
    J = jc.jacobian_affine(disc)
    A = nej.operator(disc)

    def weakest(M):
        _, s, vt = np.linalg.svd(M)
        v = vt[-1].reshape(-1, 3)
        x = v[:, np.argmax(np.abs(v).sum(axis=0))]
        return s[-1] / s[0], np.mean(np.sign(x[disc.f_own]) != np.sign(x[disc.f_nei]))

    rel_a, flips_a = weakest(A)
    rel_j, flips_j = weakest(J)
    assert rel_a < 0.2 * rel_j
    assert flips_a > 0.8 and flips_j < 0.3
