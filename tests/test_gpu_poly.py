"""GPU parity on polygonal and polyhedral face-list meshes (Sec. 3.1's
arbitrary cells): the doubled structured grid with every other 2^dim block
merged into one 8-edge (2D) or 24-face (3D) cell with hanging vertices.  Such
cells have more than 2 dim faces, so every face gets its own extrapolation
item; 3D faces are fan-triangulated and their quadrature is padded to the
largest face.  Residual and J.v against the oracle at p = 1-3 (folded and
per-point quadrature), the zero residual of degree-p fields, the neo-Hookean
law (2 and 8 points per face), the compact preconditioner and V-cycle, Newton,
and convergence under refinement."""
import numpy as np
import pytest

import workloads as w
from oracle import dynamics as ody
from oracle import jacobian as ojac
from oracle import nej as onej
from oracle import newton as onw
from oracle import precond as opc
from oracle import residual as ores

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _api():
    from paper_2601_18417_amd import api
    return api


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a.T), device=DEV, dtype=torch.float64)


def to_host(t):
    return t.cpu().numpy().T


def _m2(seed=2):
    return w.split_block_mesh((6, 5), perturb=0.2, seed=seed)


def _m3(mode="tensor"):
    return w.split_block_mesh((4, 4, 4), perturb=0.15, seed=4, mode=mode)


CASES = {
    "split2d_p1": lambda: w.poly_patch(_m2(), 1, 1, seed=4),
    "split2d_p2": lambda: w.poly_patch(_m2(), 2, 2, seed=4),
    "split2d_p3": lambda: w.poly_patch(_m2(), 3, 3, seed=4),
    "split2d_p2_traction": lambda: w.poly_patch(_m2(3), 2, 2, seed=5,
                                                traction_faces=lambda xc, n: xc[:, 1] > 1 - 1e-9),
    "split3d_p1": lambda: w.poly_patch(_m3(), 1, 1, seed=4),
    "split3d_p2": lambda: w.poly_patch(_m3(), 2, 2, seed=4),
    "split3d_p3": lambda: w.poly_patch(_m3(), 3, 3, seed=4),
    # randomly perturbed vertices: warped quadrilateral faces
    "split3d_warped_p2": lambda: w.poly_patch(_m3("random"), 2, 2, seed=4),
}
# planar faces: a degree-p field is reproduced exactly, so R vanishes
EXACT = {"split2d_p1", "split2d_p2", "split2d_p3", "split2d_p2_traction", "split3d_p1", "split3d_p2", "split3d_p3"}


def _flux_scale(disc, u):
    Ff, Fd = ores.face_fluxes(disc, u)
    s = np.zeros((disc.n_cells, disc.dim))
    np.add.at(s, disc.f_own, np.abs(Ff))
    np.add.at(s, disc.f_nei, np.abs(Ff))
    np.add.at(s, disc.d_own, np.abs(Fd))
    return s + np.abs(disc.b_body + disc.b_trac)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("fold", [True, False])
def test_residual_parity_on_split_meshes(name, fold):
    prob = CASES[name]()
    disc = ores.build(prob)
    ctx = _api().context_for(prob, fold_quadrature=fold)
    n, D = disc.n_cells, disc.dim
    fc = prob.mesh.face_cells
    assert np.bincount(fc[fc >= 0], minlength=n).max() > 2 * D  # merged cells present
    for seed in (11, 12):
        u = w.random_state(n, D, seed=seed)
        R = torch.empty((D, n), device=DEV, dtype=torch.float64)
        ctx.residual(to_dev(u), R)
        torch.cuda.synchronize()
        Ro = ores.residual(disc, u)
        assert np.linalg.norm(to_host(R) - Ro) <= 1e-10 * np.linalg.norm(Ro), (name, seed)
    u = prob.loads.exact.value(disc.cen)
    R = torch.empty((D, n), device=DEV, dtype=torch.float64)
    ctx.residual(to_dev(u), R)
    torch.cuda.synchronize()
    scale = _flux_scale(disc, u)
    Rg = to_host(R)
    assert np.all(np.abs(Rg - ores.residual(disc, u)) <= 1e-10 * scale)
    if name in EXACT:
        assert np.all(np.abs(Rg) <= 1e-10 * scale)


JV_CASES = {
    "split2d_mms_p3": lambda: w.split_mms((6, 5), 3, perturb=0.2, seed=2),
    "split3d_mms_p1": lambda: w.split_mms((4, 4, 4), 1, perturb=0.15, seed=4, mode="tensor"),
    "split3d_mms_p2": lambda: w.split_mms((4, 4, 4), 2, perturb=0.15, seed=4, mode="tensor"),
    "split3d_mms_p3": lambda: w.split_mms((4, 4, 4), 3, perturb=0.15, seed=4, mode="tensor"),
    "split3d_mms_warped_p2": lambda: w.split_mms((4, 4, 4), 2, perturb=0.15, seed=4, mode="random"),
    # degree-3 field of unit size: boundary constants make |R| ~ 30
    "split3d_p3": CASES["split3d_p3"],
}


@pytest.mark.parametrize("name", list(JV_CASES))
def test_jvp_parity_on_split_meshes(name):
    """J.v to 1e-6 relative, plus the rounding floor of any FP64 difference
    quotient: each side's two residuals are exact to a few ulps of the flux
    sums S_P they add up, and the difference is divided by eps (8 ulps of |S|
    over eps: 1e-8 of |J.v| on the manufactured trig problems, 6e-6 with the
    unit-size degree-3 field)."""
    prob = JV_CASES[name]()
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n, D = disc.n_cells, disc.dim
    u = w.random_state(n, D, seed=1)
    v = w.random_state(n, D, seed=2, scale=1.0)
    ud, vd = to_dev(u), to_dev(v)
    R = torch.empty_like(ud)
    Jv = torch.empty_like(ud)
    ctx.residual(ud, R)
    eps = ojac.default_eps(u, v)
    ctx.jvp(ud, R, vd, Jv, eps=eps)
    torch.cuda.synchronize()
    Jo = ojac.jvp(disc, u, v, eps=eps)
    floor = 8 * 2.0 ** -52 * np.linalg.norm(_flux_scale(disc, u)) / eps
    err = np.linalg.norm(to_host(Jv) - Jo)
    print(f"{name}: |dJv|/|Jv| {err / np.linalg.norm(Jo):.2e}, floor {floor / np.linalg.norm(Jo):.2e}")
    assert err <= 1e-6 * np.linalg.norm(Jo) + floor


@pytest.mark.parametrize("p", [1, 2])
def test_neo_hookean_parity_on_a_split_beam(p):
    """A clamped neo-Hookean beam on the split mesh of a 10 x 1 x 1 bar, in a
    strained state: per-point gradients at 2 (p = 1) and 8 (p = 2) points per
    quadrilateral face, R at two load scales and J.v."""
    prob = w.cantilever(shape=(16, 4, 4), p=p, n_plus=20, tip_traction=0.05)
    prob.mesh = w.split_block_mesh((8, 2, 2), lengths=(10.0, 1.0, 1.0), perturb=0.1, seed=2)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    u = w.random_state(n, 3, seed=5, scale=0.05)
    ud = to_dev(u)
    R = torch.empty_like(ud)
    for load in (1.0, 0.4):
        ctx.set_load_scale(load)
        ctx.residual(ud, R)
        torch.cuda.synchronize()
        Ro = ores.residual(disc, u, load)
        assert np.linalg.norm(to_host(R) - Ro) <= 1e-10 * np.linalg.norm(Ro), load
    v = w.random_state(n, 3, seed=6, scale=1.0)
    eps = ojac.default_eps(u, v)
    Jv = torch.empty_like(ud)
    ctx.jvp(ud, R, to_dev(v), Jv, eps=eps)
    torch.cuda.synchronize()
    Jo = ojac.jvp(disc, u, v, Ro, eps, load=0.4)
    assert np.linalg.norm(to_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)


@pytest.mark.parametrize("mk", [lambda: w.poly_patch(w.split_block_mesh((12, 12), perturb=0.2, seed=2), 2, 2, seed=4),
                                lambda: w.poly_patch(_m3(), 2, 2, seed=4)])
def test_preconditioners_on_split_meshes(mk):
    """Compact-Jacobian sweeps (up to 24 neighbours per merged cell) and the
    two-level V-cycle against the oracle's, FP64 and FP32."""
    prob = mk()
    disc = ores.build(prob)
    A = opc.assemble(disc)
    col = opc.greedy_colours(A)
    r = w.random_state(disc.n_cells, disc.dim, seed=3, scale=1.0)
    ctx = _api().context_for(prob, precond_levels=8)
    z = torch.empty((disc.dim, disc.n_cells), device=DEV, dtype=torch.float64)
    for mg in (False, True):
        ctx.set_multigrid(mg)
        ctx.precond_apply(to_dev(r), z, n_sweeps=2)
        torch.cuda.synchronize()
        if mg:
            lev = opc.hierarchy(A)
            z64, z32 = opc.vcycle(lev, r, 2), opc.vcycle(lev, r, 2, dtype=np.float32)
            tol = 1e-4
        else:
            z64, z32 = opc.sgs(A, col, r, 2), opc.sgs(A, col, r, 2, dtype=np.float32)
            tol = 1e-5
        zg = to_host(z)
        assert np.abs(zg - z64).max() <= tol * np.abs(z64).max(), mg
        assert np.abs(zg - z32).max() <= tol * np.abs(z64).max(), mg
    assert ctx.report["n_colours"] == col.max() + 1


@pytest.mark.parametrize("mk", [lambda: w.split_mms((6, 5), 2, perturb=0.2, seed=2),
                                lambda: w.split_mms((3, 3, 3), 1, perturb=0.15, seed=4, mode="tensor")])
def test_newton_on_split_meshes_matches_oracle(mk):
    prob = mk()
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n, D = disc.n_cells, disc.dim
    tol = 1e-10
    u = torch.zeros((D, n), device=DEV, dtype=torch.float64)
    st = ctx.newton_solve(u, tol=tol, eta=1e-8, restart=60)
    assert st["converged"]
    ug = to_host(u)
    R0 = np.linalg.norm(ores.residual(disc, np.zeros((n, D))))
    assert np.linalg.norm(ores.residual(disc, ug)) <= 1.01 * tol * R0
    uo, _ = onw.newton(disc, np.zeros((n, D)), tol=tol, eta=1e-8, m=60)
    print("solution difference", np.linalg.norm(ug - uo) / np.linalg.norm(uo))
    assert np.linalg.norm(ug - uo) <= 100 * tol * np.linalg.norm(uo)


@pytest.mark.parametrize("p,min_slope", [(1, 2.0), (2, 1.5), (3, 3.5)])
def test_mms_error_falls_on_refined_split_meshes(p, min_slope):
    """Unperturbed split grids of 4^2 and 8^2 blocks: the centroid RMS error of
    the converged solution falls at the rate the oracle's solutions show
    (2.26, 1.71 and 4.00 at p = 1, 2, 3)."""
    errs = []
    for cs in ((4, 4), (8, 8)):
        prob = w.split_mms(cs, p, perturb=0.0, mode="tensor")
        ctx = _api().context_for(prob)
        u = torch.zeros((2, prob.mesh.n_cells), device=DEV, dtype=torch.float64)
        st = ctx.newton_solve(u, tol=1e-10, eta=1e-8, restart=60)
        assert st["converged"]
        ue = prob.loads.exact.value(ctx.cell_centroids())
        errs.append(np.sqrt(np.mean(np.sum((to_host(u) - ue) ** 2, axis=1))))
    slope = np.log2(errs[0] / errs[1])
    print(f"split p={p} errors {errs} slope {slope:.2f}")
    assert slope >= min_slope


@pytest.mark.parametrize("mk", [lambda: w.poly_patch(_m2(), 2, 2, seed=4),
                                lambda: w.poly_patch(w.split_block_mesh((3, 3, 3), perturb=0.15, seed=4,
                                                                        mode="tensor"), 2, 2, seed=4)])
def test_near_exact_jacobian_on_split_meshes(mk):
    """The near-exact Jacobian's product (App. C) on face-list meshes against
    the oracle's assembled operator."""
    prob = mk()
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n, D = disc.n_cells, disc.dim
    v = w.random_state(n, D, seed=31, scale=1.0)
    out = torch.empty((D, n), device=DEV, dtype=torch.float64)
    ctx.nej_apply(to_dev(v), out)
    torch.cuda.synchronize()
    ref = (onej.operator(disc) @ v.ravel()).reshape(n, D)
    assert np.linalg.norm(to_host(out) - ref) <= 1e-10 * np.linalg.norm(ref)


def test_symmetry_planes_on_a_split_mesh():
    """x = 0 symmetry planes on a tensor-perturbed split mesh, a field
    symmetric about them: R against the oracle and R = 0 for degree p."""
    prob = w.poly_patch(w.split_block_mesh((4, 3, 3), perturb=0.15, seed=4, mode="tensor"), 2, 2, seed=6,
                        symmetric=True)
    disc = ores.build(prob)
    assert disc.s_own.size > 0
    ctx = _api().context_for(prob)
    n = disc.n_cells
    for u in (w.random_state(n, 3, seed=3), prob.loads.exact.value(disc.cen)):
        R = torch.empty((3, n), device=DEV, dtype=torch.float64)
        ctx.residual(to_dev(u), R)
        torch.cuda.synchronize()
        Ro = ores.residual(disc, u)
        Ff, Fd = ores.face_fluxes(disc, u)
        scale = max(np.abs(Ff).max(), np.abs(Fd).max())
        assert np.abs(to_host(R) - Ro).max() <= 1e-10 * scale
    assert np.abs(to_host(R)).max() <= 1e-10 * scale  # the symmetric quadratic: zero residual


def test_bdf2_steps_of_a_split_beam_match_oracle():
    """A neo-Hookean beam of merged blocks set moving from rest by a sudden end
    traction: three BDF2 steps on the GPU equal the oracle's."""
    prob = w.cantilever(shape=(12, 2, 2), p=1, n_plus=10)
    prob.mesh = w.split_block_mesh((6, 1, 1), lengths=(6.0, 1.0, 1.0))
    prob.loads = w.fields.cantilever_loads(6.0, (0.0, -0.02, 0.01))
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    rho, dt = 1.0, 0.5
    ctx.set_dynamics(rho, dt)
    zero = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    ctx.dyn_reset(zero, zero)
    u = zero.clone()
    z = np.zeros((n, 3))
    hist = (z, z, z, z)
    for k in range(3):
        st = ctx.dyn_step(u, tol=1e-10, eta=1e-8, max_line_search=-1, restart=96, max_krylov=400)
        assert st["converged"]
        uo, hist, _ = ody.step(disc, rho, dt, hist, m=96, maxit_krylov=400, ls_max=-1, tol=1e-10, eta=1e-8)
        assert np.linalg.norm(to_host(u) - uo) <= 1e-7 * np.linalg.norm(uo)


# face-list copies of ordinary cells: at most 2 dim faces per cell, so the
# slot-walking kernels take the short-table form (tetrahedra: 4 slots of 6,
# triangles: 3 of 4) or the fixed 2 dim-slot form (hexahedra, quads)
FACE_LIST = {
    "tets_p1": lambda: w.poly_patch(w.face_list_mesh(w.tet_mesh((4, 4, 4), perturb=0.15, seed=2)), 1, 2, seed=3),
    "tets_p2": lambda: w.poly_patch(w.face_list_mesh(w.tet_mesh((4, 4, 4), perturb=0.15, seed=2)), 2, 3, seed=3),
    "tris_p3": lambda: w.poly_patch(w.face_list_mesh(w.tri_mesh((12, 11), perturb=0.2, seed=2)), 3, 3, seed=3),
    "hexes_p2": lambda: w.poly_patch(w.face_list_mesh(w.box_mesh((7, 7, 7), perturb=0.2, seed=7, mode="tensor")),
                                     2, 3, seed=3),
    "quads_p2": lambda: w.poly_patch(w.face_list_mesh(w.box_mesh((17, 16), perturb=0.2, seed=7)), 2, 3, seed=3),
}
# every mesh has more than 256 cells, so that a V-cycle has a coarse level


@pytest.mark.parametrize("name", list(FACE_LIST))
def test_face_lists_of_ordinary_cells(name):
    """R, J.v and both preconditioners against the oracle's face-list build."""
    prob = FACE_LIST[name]()
    assert prob.mesh.n_cells > 256
    disc = ores.build(prob)
    ctx = _api().context_for(prob, precond_levels=8)
    n, D = disc.n_cells, disc.dim
    fc = prob.mesh.face_cells
    assert np.bincount(fc[fc >= 0], minlength=n).max() <= 2 * D
    u = w.random_state(n, D, seed=11)
    ud = to_dev(u)
    R = torch.empty_like(ud)
    ctx.residual(ud, R)
    torch.cuda.synchronize()
    Ro = ores.residual(disc, u)
    assert np.linalg.norm(to_host(R) - Ro) <= 1e-10 * np.linalg.norm(Ro)
    v = w.random_state(n, D, seed=2, scale=1.0)
    eps = ojac.default_eps(u, v)
    Jv = torch.empty_like(ud)
    ctx.jvp(ud, R, to_dev(v), Jv, eps=eps)
    torch.cuda.synchronize()
    Jo = ojac.jvp(disc, u, v, eps=eps)
    floor = 8 * 2.0 ** -52 * np.linalg.norm(_flux_scale(disc, u)) / eps
    assert np.linalg.norm(to_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo) + floor
    A = opc.assemble(disc)
    col = opc.greedy_colours(A)
    r = w.random_state(n, D, seed=3, scale=1.0)
    z = torch.empty((D, n), device=DEV, dtype=torch.float64)
    for mg in (False, True):
        ctx.set_multigrid(mg)
        ctx.precond_apply(to_dev(r), z, n_sweeps=2)
        torch.cuda.synchronize()
        z64 = opc.vcycle(opc.hierarchy(A), r, 2) if mg else opc.sgs(A, col, r, 2)
        assert np.abs(to_host(z) - z64).max() <= (1e-4 if mg else 1e-5) * np.abs(z64).max(), mg


MANY = {
    "cube_54_faces": lambda: w.poly_patch(w.merged_block_mesh(w.box_mesh((7, 7, 7), perturb=0.15, seed=5,
                                                                         mode="tensor"), (2, 2, 2), (5, 5, 5)),
                                          1, 2, seed=3),
    "square_20_edges": lambda: w.poly_patch(w.merged_block_mesh(w.box_mesh((17, 17), perturb=0.2, seed=5),
                                                                (6, 6), (11, 11)), 2, 3, seed=3),
    # the largest cells accepted: groups of 64 lanes, the whole wavefront
    "cube_216_faces": lambda: w.poly_patch(w.merged_block_mesh(w.box_mesh((8, 8, 8), perturb=0.15, seed=5,
                                                                          mode="tensor"), (1, 1, 1), (7, 7, 7)),
                                           1, 2, seed=3),
    "square_252_edges": lambda: w.poly_patch(w.merged_block_mesh(w.box_mesh((65, 65), perturb=0.2, seed=5),
                                                                 (1, 1), (64, 64)), 1, 2, seed=3),
}
NFACES = {"cube_54_faces": 54, "square_20_edges": 20, "cube_216_faces": 216, "square_252_edges": 252}


@pytest.mark.parametrize("name", list(MANY))
def test_cells_with_many_faces(name):
    """One cell with 54 faces (3D: 16 lanes of the cell sum and sweeps share
    it), 20 edges (2D: 8 lanes), or the most a cell may have short of 255
    (216 faces, 252 edges: 64 lanes) among ordinary cells: R, J.v and both
    preconditioners against the oracle."""
    prob = MANY[name]()
    disc = ores.build(prob)
    ctx = _api().context_for(prob, precond_levels=8)
    n, D = disc.n_cells, disc.dim
    fc = prob.mesh.face_cells
    assert np.bincount(fc[fc >= 0], minlength=n).max() == NFACES[name]
    u = w.random_state(n, D, seed=11)
    ud = to_dev(u)
    R = torch.empty_like(ud)
    ctx.residual(ud, R)
    torch.cuda.synchronize()
    Ro = ores.residual(disc, u)
    assert np.linalg.norm(to_host(R) - Ro) <= 1e-10 * np.linalg.norm(Ro)
    assert np.all(np.abs(to_host(R) - Ro) <= 1e-10 * _flux_scale(disc, u))
    v = w.random_state(n, D, seed=2, scale=1.0)
    eps = ojac.default_eps(u, v)
    Jv = torch.empty_like(ud)
    ctx.jvp(ud, R, to_dev(v), Jv, eps=eps)
    torch.cuda.synchronize()
    Jo = ojac.jvp(disc, u, v, eps=eps)
    floor = 8 * 2.0 ** -52 * np.linalg.norm(_flux_scale(disc, u)) / eps
    assert np.linalg.norm(to_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo) + floor
    A = opc.assemble(disc)
    col = opc.greedy_colours(A)
    r = w.random_state(n, D, seed=3, scale=1.0)
    z = torch.empty((D, n), device=DEV, dtype=torch.float64)
    for mg in (False, True):
        ctx.set_multigrid(mg)
        ctx.precond_apply(to_dev(r), z, n_sweeps=2)
        torch.cuda.synchronize()
        z64 = opc.vcycle(opc.hierarchy(A), r, 2) if mg else opc.sgs(A, col, r, 2)
        assert np.abs(to_host(z) - z64).max() <= (1e-4 if mg else 1e-5) * np.abs(z64).max(), mg
