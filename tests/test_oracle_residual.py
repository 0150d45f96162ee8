"""Pins of the oracle residual R(u) against what the mathematics fixes."""
import numpy as np
import pytest

import workloads as w
from oracle import residual as rs


def _rel_zero(disc, u, load=1.0):
    R = rs.residual(disc, u, load)
    Ff, Fd = rs.face_fluxes(disc, u, load)
    scale = max(np.abs(Ff).max(), np.abs(Fd).max() if Fd.size else 0.0)
    return np.abs(R).max() / scale


CASES = [(2, (7, 6), 0.0, "random"), (2, (7, 6), 0.2, "random"),
         (3, (5, 5, 5), 0.0, "random"), (3, (5, 5, 5), 0.2, "tensor")]


@pytest.mark.parametrize("dim,shape,pert,mode", CASES)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_polynomial_fields_give_zero_residual(dim, shape, pert, mode, p):
    """A polynomial of degree <= p with its exact body force and boundary values
    is reproduced exactly: gradients, face integrals and u* jumps are exact."""
    mesh = w.box_mesh(shape, perturb=pert, seed=3, mode=mode)
    prob = w.poly_patch(mesh, p, p, seed=p)
    disc = rs.build(prob)
    u = prob.loads.exact.value(disc.cen)
    assert _rel_zero(disc, u) < 1e-12


def test_linear_field_zero_residual_on_nonplanar_faces():
    mesh = w.box_mesh((5, 5, 5), perturb=0.2, seed=9)
    prob = w.poly_patch(mesh, 3, 1, seed=1)
    disc = rs.build(prob)
    assert _rel_zero(disc, prob.loads.exact.value(disc.cen)) < 1e-12


def test_quadratic_field_not_exact_on_nonplanar_faces():
    """The single-normal face rule is only exact on planar faces (Sec. 3.2)."""
    mesh = w.box_mesh((5, 5, 5), perturb=0.2, seed=9)
    prob = w.poly_patch(mesh, 2, 2, seed=1)
    disc = rs.build(prob)
    assert _rel_zero(disc, prob.loads.exact.value(disc.cen)) > 1e-6


@pytest.mark.parametrize("dim,shape", [(2, (6, 6)), (3, (5, 5, 5))])
def test_traction_faces_with_exact_traction(dim, shape):
    mesh = w.box_mesh(shape, perturb=0.15, seed=2, mode="tensor")
    prob = w.poly_patch(mesh, 2, 2, seed=4, traction_faces=lambda xc, n: xc[:, 0] > 1 - 1e-9)
    disc = rs.build(prob)
    assert np.abs(prob.loads.bc_type(disc.d_x, disc.d_n)).max() == 0
    assert disc.b_trac.any()
    assert _rel_zero(disc, prob.loads.exact.value(disc.cen)) < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_symmetric_polynomial_fields_give_zero_residual_with_symmetry_faces(p):
    """Faces on x = 0 are symmetry planes (Sec. 3.5: half stencil plus its mirror
    image, ghosts carrying R_b u).  A polynomial of degree <= p that is
    symmetric about x = 0 (u_x odd in x, u_y and u_z even) is its own mirror
    image, so the reconstruction reproduces it and R = 0."""
    mesh = w.box_mesh((5, 5, 5), perturb=0.2, seed=3, mode="tensor")
    prob = w.poly_patch(mesh, p, p, seed=p, symmetric=True)
    disc = rs.build(prob)
    assert disc.s_own.size == 25 and disc.s_st.shape[1] == (prob.stencil_size + 1) // 2
    assert _rel_zero(disc, prob.loads.exact.value(disc.cen)) < 1e-12


def test_symmetry_faces_see_an_asymmetric_field():
    """The same faces with a field that is not symmetric about x = 0: the mirror
    images contradict it and the cells on the plane keep a residual."""
    mesh = w.box_mesh((5, 5, 5), perturb=0.2, seed=3, mode="tensor")
    prob = w.poly_patch(mesh, 2, 2, seed=2)
    fld = prob.loads.exact
    prob.loads = w.fields.mms_loads(fld, prob.mu, prob.lam, symmetry_faces=lambda xc, n: np.abs(xc[:, 0]) < 1e-9)
    disc = rs.build(prob)
    u = fld.value(disc.cen)
    R = rs.residual(disc, u)
    on_plane = np.unique(disc.s_own)
    assert np.abs(R[on_plane]).max() > 1e-3 * np.abs(rs.symmetry_fluxes(disc, u)).max()


def _nh_problem(shape=(5, 4, 4), p=2, pert=0.15, loads=None):
    mesh = w.box_mesh(shape, perturb=pert, seed=5, mode="tensor")
    zero = lambda x: np.zeros_like(x)
    if loads is None:
        loads = w.Loads(3, lambda xc, n: np.zeros(xc.shape[0], np.int32), zero,
                        lambda x, n: np.zeros_like(x), zero)
    return w.Problem("nh", mesh, p, 55, 2, w.NEO_HOOKEAN, 1.0, 10.0, loads,
                     stencil_quantum=1e-6 / 16)


def test_neo_hookean_rigid_rotation_is_stress_free():
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    c = np.array([0.1, -0.2, 0.3])
    ub = lambda x: x @ (Q - np.eye(3)).T + c
    loads = w.Loads(3, lambda xc, n: np.zeros(xc.shape[0], np.int32), ub,
                    lambda x, n: np.zeros_like(x), lambda x: np.zeros_like(x))
    disc = rs.build(_nh_problem(loads=loads))
    u = ub(disc.cen)
    R = rs.residual(disc, u)
    assert np.abs(R).max() < 1e-12


def test_neo_hookean_homogeneous_deformation_balances():
    F = np.eye(3) + np.array([[0.2, 0.05, -0.1], [0.0, -0.1, 0.07], [0.03, 0.0, 0.15]])
    ub = lambda x: x @ (F - np.eye(3)).T
    loads = w.Loads(3, lambda xc, n: np.zeros(xc.shape[0], np.int32), ub,
                    lambda x, n: np.zeros_like(x), lambda x: np.zeros_like(x))
    disc = rs.build(_nh_problem(loads=loads))
    u = ub(disc.cen)
    R = rs.residual(disc, u)
    Ff, Fd = rs.face_fluxes(disc, u)
    assert np.abs(R).max() < 1e-12 * np.abs(Ff).max()
    assert np.abs(Ff).max() > 1e-3  # the stress is not zero


def test_neo_hookean_reduces_to_linear_elasticity():
    """NH -> LE as |grad u| -> 0 (App. A): the difference is O(delta^2)."""
    disc_nh = rs.build(_nh_problem())
    disc_le = rs.build(_nh_problem())
    disc_le.material = w.LINEAR_ELASTIC
    v = w.random_state(disc_nh.n_cells, 3, seed=1, scale=1.0)
    errs = []
    for d in (1e-2, 1e-3, 1e-4):
        Rn = rs.residual(disc_nh, d * v)
        Rl = rs.residual(disc_le, d * v)
        errs.append(np.linalg.norm(Rn - Rl) / np.linalg.norm(Rl))
    slope = np.log10(errs[0] / errs[2]) / 2
    assert 0.9 < slope < 1.1 and errs[-1] < 1e-3


def test_neo_hookean_small_strain_keeps_its_digits():
    """P(G) - sigma_LE(G) = O(|G|^2) (the law linearises to eq. linearElastic
    at G = 0, App. A), so the relative gap to the linear stress shrinks with
    |G| down to round-off: at |G| ~ 1e-12 it is ~1e-12.  A form that builds
    J - 1 or dev(bbar) by subtracting O(1) numbers fails here (its error is
    ~1e-16 / |G|), and that error is what a finite-difference J.v sees."""
    G = np.random.default_rng(4).standard_normal((200, 3, 3))
    for s in (1e-6, 1e-9, 1e-12):
        P = rs.piola_neo_hookean(s * G, 1.0, 10.0)
        L = np.swapaxes(rs.stress_linear(s * G, 1.0, 10.0), -1, -2)
        assert np.abs(P - L).max() <= 50.0 * s * np.abs(L).max()


def _fd_grad(f, X, h=1e-6):
    g = np.zeros_like(X)
    for idx in np.ndindex(*X.shape):
        e = np.zeros_like(X)
        e[idx] = h
        g[idx] = (f(X + e) - f(X - e)) / (2 * h)
    return g


def test_linear_stress_is_strain_energy_derivative():
    mu, lam = 0.7, 1.3
    rng = np.random.default_rng(0)
    for D in (2, 3):
        G = rng.standard_normal((D, D)) * 0.1

        def psi(G):
            eps = 0.5 * (G + G.T)
            return mu * np.sum(eps * eps) + 0.5 * lam * np.trace(eps) ** 2
        assert np.allclose(rs.stress_linear(G[None], mu, lam)[0], _fd_grad(psi, G), atol=1e-8)


def test_neo_hookean_piola_is_strain_energy_derivative():
    """P = dPsi/dF for Psi = mu/2 (J^{-2/3} tr(F F^T) - 3) + kappa/4 (J^2 - 1 - 2 ln J),
    the energy whose Cauchy stress is eq. neoHook."""
    mu, lam = 1.0, 10.0
    kappa = lam + 2 * mu / 3
    rng = np.random.default_rng(1)
    G = rng.standard_normal((3, 3)) * 0.2

    def psi(F):
        J = np.linalg.det(F)
        return mu / 2 * (J ** (-2 / 3) * np.trace(F @ F.T) - 3) + kappa / 4 * (J * J - 1 - 2 * np.log(J))
    F = np.eye(3) + G.T
    P_fd = _fd_grad(psi, F)
    P = rs.piola_neo_hookean(G[None], mu, lam)[0]
    assert np.allclose(P, P_fd, atol=1e-7)


@pytest.mark.parametrize("dim,shape", [(2, (6, 5)), (3, (4, 4, 4))])
def test_conservation(dim, shape):
    """Internal fluxes and stabilisation cancel pairwise: sum_P R_P equals the
    boundary fluxes plus the sources."""
    prob = w.square_mms(6, 2, perturb=0.2) if dim == 2 else w.cube_mms(4, 1, perturb=0.2)
    disc = rs.build(prob)
    u = w.random_state(disc.n_cells, dim, seed=3)
    R = rs.residual(disc, u)
    Ff, Fd = rs.face_fluxes(disc, u)
    total = Fd.sum(axis=0) + (disc.b_body + disc.b_trac).sum(axis=0)
    assert np.allclose(R.sum(axis=0), total, rtol=1e-12, atol=1e-13 * np.abs(Ff).max())


def test_linearity_of_linear_elastic_residual():
    prob = w.cube_mms(4, 1, perturb=0.2)
    disc = rs.build(prob)
    n = disc.n_cells
    u, v = w.random_state(n, 3, 1), w.random_state(n, 3, 2)
    R0 = rs.residual(disc, np.zeros((n, 3)))
    lhs = rs.residual(disc, 2.0 * u - 3.0 * v) - R0
    rhs = 2.0 * (rs.residual(disc, u) - R0) - 3.0 * (rs.residual(disc, v) - R0)
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(lhs)


def test_stabilisation_checkerboard_closed_form():
    """2D uniform mesh, p = 1: the 13-cell cell stencil is symmetric, so a
    checkerboard has zero reconstructed gradient, u* = u_P, and every internal
    face adds alpha Kbar (u_N - u_P) (|d . n| = Gamma = h): interior cells get
    the stabilisation part -8 alpha Kbar u_P."""
    prob = w.square_mms(10, 1)
    disc = rs.build(prob)
    ijk = w.cell_ijk(prob.mesh)
    sgn = (-1.0) ** (ijk[:, 0] + ijk[:, 1])
    u = np.stack([sgn, 0.5 * sgn], axis=1)
    d0 = rs.build(prob)
    d0.alpha = 0.0
    Rs = rs.residual(disc, u) - rs.residual(d0, u)
    interior = np.all((ijk >= 3) & (ijk <= 6), axis=1)  # neighbours have full stencils
    assert np.allclose(Rs[interior], -8 * prob.alpha * disc.kbar * u[interior], rtol=1e-12)


def test_stabilisation_is_dissipative():
    """v^T (R_alpha(v) - R_0(v)) = -sum_f alpha Kbar Gamma_f / |d.n| |u*_N - u*_P|^2 < 0."""
    prob = w.cube_mms(5, 2, perturb=0.2)
    disc = rs.build(prob)
    d0 = rs.build(prob)
    d0.alpha = 0.0
    v = w.random_state(disc.n_cells, 3, 6)
    zero = np.zeros_like(v)
    Rs = (rs.residual(disc, v) - rs.residual(disc, zero)) - (rs.residual(d0, v) - rs.residual(d0, zero))
    assert np.sum(v * Rs) < 0


def test_active_subset_matches_full_residual():
    prob = w.cube_mms(5, 2, perturb=0.2)
    full = rs.build(prob)
    sub = np.array([0, 17, 62, 124])
    part = rs.build(prob, active=sub)
    u = w.random_state(full.n_cells, 3, 8)
    assert np.allclose(rs.residual(part, u)[sub], rs.residual(full, u)[sub], rtol=1e-14, atol=1e-17)


# --- eq. alpha's skewness measure |d_PN . n_f| on a sheared grid --------------
#
# A uniform grid sheared by x += s y has parallelogram cells.  On the slanted
# faces (between cells i and i+1) d_PN = (h, 0), n_f = (1, -s)/sqrt(1+s^2) and
# Gamma_f = h sqrt(1+s^2), so Gamma_f / |d_PN . n_f| = 1 + s^2 while
# Gamma_f / |d_PN| = sqrt(1+s^2); on the horizontal faces d_PN = (s h, h),
# n_f = (0, 1), Gamma_f = h: the two ratios are 1 and 1/sqrt(1+s^2).  The
# shear s = 0.6 keeps every squared lattice distance within the 13-cell p = 1
# stencil distinct except for the pairs +-delta, so interior stencils are
# point-symmetric.

SHEAR = 0.6


def sheared_square(n, p=1, s=SHEAR, zero_loads=False):
    prob = w.square_mms(n, p)
    v = prob.mesh.verts.copy()
    v[:, 0] += s * v[:, 1]
    prob.mesh.verts = v
    if zero_loads:
        zero = lambda x: np.zeros((x.shape[0], 2))
        prob.loads = w.fields.Loads(2, lambda xc, nrm: np.full(xc.shape[0], w.fields.DISP, np.int32), zero,
                                    lambda x, nrm: zero(x), zero)
    return prob


def _symmetric_stencil(disc, ijk, n, P):
    """Whether P's cell stencil is invariant under the point reflection about P."""
    st = {tuple(ijk[c]) for c in disc.c_st[P]}
    return all((2 * ijk[P][0] - a, 2 * ijk[P][1] - b) in st for a, b in st)


def test_stabilisation_skewness_checkerboard_on_sheared_grid():
    """p = 1, checkerboard u: on cells whose stencil (and whose face neighbours'
    stencils) are point-symmetric the reconstructed gradient is zero, u* = u_P,
    and each face adds alpha Kbar Gamma_f / |d_PN . n_f| (u_N - u_P) with
    u_N = -u_P: the stabilisation part of R_P is -4 alpha Kbar (2 + s^2) u_P.
    With |d_PN| in place of |d_PN . n_f| it would be
    -4 alpha Kbar (sqrt(1+s^2) + 1/sqrt(1+s^2)) u_P."""
    n = 12
    prob = sheared_square(n)
    disc = rs.build(prob)
    d0 = rs.build(prob)
    d0.alpha = 0.0
    ijk = w.cell_ijk(prob.mesh)
    sgn = (-1.0) ** (ijk[:, 0] + ijk[:, 1])
    u = np.stack([sgn, -0.7 * sgn], axis=1)
    Rs = rs.residual(disc, u) - rs.residual(d0, u)
    sym = np.array([_symmetric_stencil(disc, ijk, n, P) for P in range(disc.n_cells)])
    good = np.array([sym[P] and all(sym[Q] for Q in range(disc.n_cells)
                                    if np.abs(ijk[Q] - ijk[P]).sum() == 1) for P in range(disc.n_cells)])
    assert good.sum() >= 25
    s2 = SHEAR ** 2
    expect = -4.0 * prob.alpha * disc.kbar * (2.0 + s2) * u[good]
    assert np.allclose(Rs[good], expect, rtol=1e-12, atol=0)
    wrong = -4.0 * prob.alpha * disc.kbar * (np.sqrt(1 + s2) + 1 / np.sqrt(1 + s2)) * u[good]
    assert np.abs(Rs[good] - wrong).max() > 0.05 * np.abs(wrong).max()


def test_stabilisation_skewness_on_sheared_displacement_faces():
    """A constant field c with u_b = 0: the reconstruction of a constant is
    exact on any stencil, so u* = c and internal faces add nothing; each
    displacement face adds alpha Kbar Gamma_b / |d_Pb . n_b| (0 - c).  Bottom and
    top faces: Gamma_b / |d_Pb . n_b| = h / (h/2) = 2; left and right (slanted)
    faces: h sqrt(1+s^2) / (h / (2 sqrt(1+s^2))) = 2 (1 + s^2)."""
    n = 8
    prob = sheared_square(n, zero_loads=True)
    disc = rs.build(prob)
    d0 = rs.build(prob)
    d0.alpha = 0.0
    c = np.array([0.3, -1.1])
    u = np.tile(c, (disc.n_cells, 1))
    Rs = rs.residual(disc, u) - rs.residual(d0, u)
    ijk = w.cell_ijk(prob.mesh)
    n_flat = (ijk[:, 1] == 0).astype(float) + (ijk[:, 1] == n - 1)
    n_slant = (ijk[:, 0] == 0).astype(float) + (ijk[:, 0] == n - 1)
    coef = 2.0 * n_flat + 2.0 * (1 + SHEAR ** 2) * n_slant
    expect = -prob.alpha * disc.kbar * coef[:, None] * c[None, :]
    assert np.allclose(Rs, expect, rtol=1e-12, atol=1e-14)
