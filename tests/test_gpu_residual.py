"""GPU parity of R(u) and J.v against the FP64 oracle, through the C ABI.

Tolerances: R to 1e-10 relative (2-norm) on seeded random states, and a
per-cell scale-aware bound (|dR_P| <= 1e-10 (sum of |face fluxes| + |sources|))
near the manufactured solution; J.v with the same eps to 1e-6 relative: both
sides difference two residuals whose constant parts (boundary sources of order
one) round at eps_mach and are divided by eps ~ 1e-10..1e-8, so the products
themselves carry ~1e-8 relative noise.
"""
import numpy as np
import pytest

import workloads as w
from oracle import jacobian as ojac
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


def _flux_scale(disc, u):
    Ff, Fd = ores.face_fluxes(disc, u)
    s = np.zeros((disc.n_cells, disc.dim))
    np.add.at(s, disc.f_own, np.abs(Ff))
    np.add.at(s, disc.f_nei, np.abs(Ff))
    np.add.at(s, disc.d_own, np.abs(Fd))
    if disc.s_own is not None:
        np.add.at(s, disc.s_own, np.abs(ores.symmetry_fluxes(disc, u)))
    return s + np.abs(disc.b_body + disc.b_trac)


CASES = {
    "square32_p2": lambda: w.square_mms(32, 2),
    "square12_p3_pert": lambda: w.square_mms(12, 3, perturb=0.2, seed=4),
    "square9_p1": lambda: w.square_mms(9, 1, perturb=0.15, seed=2),
    "cube8_p1_pert": lambda: w.cube_mms(8, 1, perturb=0.2, seed=1),
    "cube8_p2_pert": lambda: w.cube_mms(8, 2, perturb=0.2, seed=2),
    "cube9_p3_pert": lambda: w.cube_mms(9, 3, perturb=0.2, seed=3),
    "box_11x7x6_p3": lambda: w.cube_mms((11, 7, 6), 3, perturb=0.2, seed=5, lengths=(1.0, 0.6, 0.5)),
    "cube7_p2_traction": lambda: w.poly_patch(w.box_mesh((7, 7, 7), perturb=0.2, seed=8), 2, 3, seed=3,
                                              traction_faces=lambda xc, n: xc[:, 2] > 1 - 1e-9),
    # symmetry planes on x = 0 with fields symmetric about them
    "square8_p2_symmetry": lambda: w.poly_patch(w.box_mesh((8, 7), perturb=0.15, seed=4, mode="tensor"), 2, 2,
                                                seed=6, symmetric=True),
    "box_p1_symmetry": lambda: w.poly_patch(w.box_mesh((6, 5, 5), perturb=0.2, seed=4, mode="tensor"), 1, 1,
                                            seed=5, symmetric=True),
    "box_p2_symmetry": lambda: w.poly_patch(w.box_mesh((6, 5, 5), perturb=0.2, seed=4, mode="tensor"), 2, 2,
                                            seed=6, symmetric=True),
    "box_p3_symmetry": lambda: w.poly_patch(w.box_mesh((7, 6, 6), perturb=0.2, seed=4, mode="tensor"), 3, 3,
                                            seed=7, symmetric=True),
    # far from the origin (|x| / h ~ 10^3): geometry, stencils and least squares
    # start from absolute coordinates
    "square_far_p2": lambda: w.poly_patch(w.box_mesh((12, 10), lengths=(1.0, 0.8), origin=(100.0, -50.0),
                                                     perturb=0.2, seed=2), 2, 2, seed=4),
    "cube_far_p2": lambda: w.poly_patch(w.box_mesh((7, 6, 6), lengths=(1.0, 0.9, 0.8), origin=(40.0, -20.0, 10.0),
                                                   perturb=0.2, seed=3), 2, 2, seed=5),
    # very small and very large domains: nothing in the setup may assume unit size
    "cube_mm_p2": lambda: w.poly_patch(w.box_mesh((6, 6, 5), lengths=(1e-3, 1e-3, 8e-4), perturb=0.2, seed=3), 2, 2,
                                       seed=5),
    "square_km_p3": lambda: w.poly_patch(w.box_mesh((10, 9), lengths=(1e3, 9e2), perturb=0.2, seed=2), 3, 3, seed=4),
    # flat cells (aspect 10 and 30): the least squares are worse conditioned
    "box_aspect10_p3": lambda: w.cube_mms((9, 9, 9), 3, perturb=0.2, seed=4, lengths=(1.0, 1.0, 0.1)),
    "box_aspect30_p2": lambda: w.cube_mms((9, 9, 8), 2, perturb=0.2, seed=4, lengths=(1.0, 1.0, 1.0 / 30 * 8 / 9)),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("fold", [True, False])
def test_residual_parity(name, fold):
    prob = CASES[name]()
    disc = ores.build(prob)
    ctx = _api().context_for(prob, fold_quadrature=fold)
    n, D = disc.n_cells, disc.dim
    for seed in (11, 12):
        u = w.random_state(n, D, seed=seed)
        R = torch.empty((D, n), device=DEV, dtype=torch.float64)
        ctx.residual(to_dev(u), R)
        torch.cuda.synchronize()
        Ro = ores.residual(disc, u)
        Rg = to_host(R)
        rel = np.linalg.norm(Rg - Ro) / np.linalg.norm(Ro)
        assert rel <= 1e-10, (name, seed, rel)
        # and cell by cell, against the size of what the cell sums
        assert np.all(np.abs(Rg - Ro) <= 1e-10 * _flux_scale(disc, u)), (name, seed)
    # near the manufactured solution
    if prob.loads.exact is not None:
        u = prob.loads.exact.value(disc.cen)
        R = torch.empty((D, n), device=DEV, dtype=torch.float64)
        ctx.residual(to_dev(u), R)
        torch.cuda.synchronize()
        Ro = ores.residual(disc, u)
        bound = 1e-10 * _flux_scale(disc, u)
        assert np.all(np.abs(to_host(R) - Ro) <= bound), name


@pytest.mark.parametrize("name", ["square32_p2", "cube8_p2_pert", "cube9_p3_pert", "box_p3_symmetry"])
def test_jvp_parity(name):
    prob = CASES[name]()
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n, D = disc.n_cells, disc.dim
    u = w.random_state(n, D, seed=1)
    v = w.random_state(n, D, seed=2, scale=1.0)
    ud, vd = to_dev(u), to_dev(v)
    Ru = torch.empty_like(ud)
    ctx.residual(ud, Ru)
    Ro = ores.residual(disc, u)
    eps = ojac.default_eps(u, v)
    Jo = ojac.jvp(disc, u, v, Ro, eps)
    Jv = torch.empty_like(ud)
    ctx.jvp(ud, Ru, vd, Jv, eps=eps)
    torch.cuda.synchronize()
    assert np.linalg.norm(to_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)
    # device-side default eps
    ctx.jvp(ud, Ru, vd, Jv, eps=0.0)
    torch.cuda.synchronize()
    assert np.linalg.norm(to_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)
    # v = 0 gives exactly 0
    ctx.jvp(ud, Ru, torch.zeros_like(vd), Jv, eps=0.0)
    torch.cuda.synchronize()
    assert not torch.any(Jv)


def test_load_scale_scales_sources():
    prob = CASES["cube7_p2_traction"]()
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    u = w.random_state(n, 3, seed=4)
    R = torch.empty((3, n), device=DEV, dtype=torch.float64)
    ctx.set_load_scale(0.3)
    ctx.residual(to_dev(u), R)
    torch.cuda.synchronize()
    Ro = ores.residual(disc, u, load=0.3)
    assert np.linalg.norm(to_host(R) - Ro) <= 1e-10 * np.linalg.norm(Ro)


def test_residual_is_deterministic():
    prob = CASES["cube9_p3_pert"]()
    ctx = _api().context_for(prob)
    n = prob.mesh.n_cells
    ud = to_dev(w.random_state(n, 3, seed=9))
    R1 = torch.empty_like(ud)
    R2 = torch.empty_like(ud)
    ctx.residual(ud, R1)
    ctx.residual(ud, R2)
    torch.cuda.synchronize()
    assert torch.equal(R1, R2)


def test_fgmres_is_deterministic():
    """The Krylov sums are fixed-order reductions: two solves of the same
    system give identical bits."""
    prob = CASES["cube8_p2_pert"]()
    ctx = _api().context_for(prob)
    n = prob.mesh.n_cells
    ud = to_dev(w.random_state(n, 3, seed=9))
    Ru = torch.empty_like(ud)
    ctx.residual(ud, Ru)
    b = to_dev(w.random_state(n, 3, seed=10, scale=1.0))
    xs = []
    for _ in range(2):
        x = torch.zeros_like(b)
        st = ctx.fgmres_solve(ud, Ru, b, x, rtol=1e-8, max_iters=400, restart=40)
        assert st["converged"]
        xs.append(x)
    torch.cuda.synchronize()
    assert torch.equal(xs[0], xs[1])


def test_neo_hookean_residual_and_jvp_parity():
    prob = w.cantilever(shape=(12, 5, 5), p=2, tip_traction=0.05)
    prob.mesh = w.box_mesh((12, 5, 5), lengths=(10.0, 1, 1), perturb=0.15, seed=3)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    u = w.random_state(n, 3, seed=5, scale=0.05)
    for load in (1.0, 0.4):
        ctx.set_load_scale(load)
        ud = to_dev(u)
        R = torch.empty_like(ud)
        ctx.residual(ud, R)
        torch.cuda.synchronize()
        Ro = ores.residual(disc, u, load)
        assert np.linalg.norm(to_host(R) - Ro) <= 1e-10 * np.linalg.norm(Ro)
    v = w.random_state(n, 3, seed=6, scale=1.0)
    eps = ojac.default_eps(u, v)
    Jv = torch.empty_like(ud)
    ctx.jvp(ud, R, to_dev(v), Jv, eps=eps)
    torch.cuda.synchronize()
    Jo = ojac.jvp(disc, u, v, Ro, eps, load=0.4)
    assert np.linalg.norm(to_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)


@pytest.mark.parametrize("p", [1, 2])
def test_neo_hookean_symmetry_faces_parity(p):
    """Symmetry planes with the neo-Hookean law: per-point gradients from the
    cells and their mirror images, R and J.v against the oracle at a strained
    random state."""
    # a small field: its values are the displacement-face data, and O(1) data would invert cells
    prob = w.poly_patch(w.box_mesh((6, 5, 5), perturb=0.2, seed=4, mode="tensor"), p, p, seed=6, symmetric=True,
                        scale=1e-3)
    prob.material = w.NEO_HOOKEAN
    prob.mu, prob.lam = 1.0, 10.0
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    u = w.random_state(n, 3, seed=31, scale=1e-2)
    v = w.random_state(n, 3, seed=32, scale=1.0)
    R = torch.empty((3, n), device=DEV, dtype=torch.float64)
    Jv = torch.empty_like(R)
    ud = to_dev(u)
    ctx.residual(ud, R)
    eps = ojac.default_eps(u, v)
    ctx.jvp(ud, R, to_dev(v), Jv, eps=eps)
    torch.cuda.synchronize()
    Ro = ores.residual(disc, u)
    Jo = (ores.residual(disc, u + eps * v) - Ro) / eps
    assert disc.s_own.size > 0
    assert np.linalg.norm(to_host(R) - Ro) <= 1e-10 * np.linalg.norm(Ro)
    assert np.linalg.norm(to_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)


def _fan_beam(p):
    prob = w.cantilever(shape=(10, 3, 3), p=p, n_plus=20, tip_traction=0.05)
    prob.mesh = w.box_mesh((10, 3, 3), lengths=(10.0, 1.0, 1.0), perturb=0.15, seed=3)
    return prob


@pytest.mark.parametrize("case", ["le_p2_folded", "le_p3_folded", "le_p2_points", "le_p3_points", "nh_p1", "nh_p2"])
def test_residual_and_jvp_parity_with_the_fan_face_rule(case):
    """Quadrilateral faces integrated by fan triangulation (two triangles from
    the lowest-numbered vertex, area-scaled weights) on randomly perturbed
    meshes, whose faces are not planar: the linear law with the points folded
    into the coefficients or kept (8 points per face), and the neo-Hookean law
    on a strained beam (2 and 8 points per face)."""
    law, pp, form = (case.split("_") + [""])[:3]
    p = int(pp[1])
    prob = w.cube_mms(6 if p == 2 else 7, p, perturb=0.2) if law == "le" else _fan_beam(p)
    prob.face_rule = 1
    disc = ores.build(prob)
    ctx = _api().context_for(prob, fold_quadrature=form != "points")
    n = disc.n_cells
    u = w.random_state(n, 3, seed=21, scale=1e-3 if law == "le" else 0.05)
    v = w.random_state(n, 3, seed=22, scale=1.0)
    ud, vd = to_dev(u), to_dev(v)
    R = torch.empty_like(ud)
    Jv = torch.empty_like(ud)
    ctx.residual(ud, R)
    eps = ojac.default_eps(u, v)
    ctx.jvp(ud, R, vd, Jv, eps=eps)
    torch.cuda.synchronize()
    Ro = ores.residual(disc, u)
    assert np.linalg.norm(to_host(R) - Ro) <= 1e-10 * np.linalg.norm(Ro)
    Jo = ojac.jvp(disc, u, v, eps=eps)
    assert np.linalg.norm(to_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)


@pytest.mark.parametrize("name", ["cube8_p2_pert", "square9_p1", "tri8_p3"])
def test_caller_cell_numbering_is_kept(name):
    """The library orders cells and faces internally (Morton order, item
    blocks) but reads and writes vectors in the caller's cell numbering:
    renumbering the cells permutes R and J.v the same way (to rounding, as
    the sums' order changes), on perturbed meshes where no stencil ties."""
    import copy
    if name == "tri8_p3":
        prob = w.tri_mms(8, 3, perturb=0.2)
    else:
        prob = CASES[name]()
    n, D = prob.mesh.n_cells, prob.dim
    perm = np.random.default_rng(5).permutation(n)
    prob2 = copy.deepcopy(prob)
    prob2.mesh.cells = prob.mesh.cells[perm]  # cell i of prob2 is cell perm[i] of prob
    api = _api()
    c1, c2 = api.context_for(prob), api.context_for(prob2)
    u = w.random_state(n, D, seed=31)
    v = w.random_state(n, D, seed=32, scale=1.0)
    out = []
    for ctx, uu, vv in ((c1, u, v), (c2, u[perm], v[perm])):
        ud, vd = to_dev(uu), to_dev(vv)
        R = torch.empty_like(ud)
        Jv = torch.empty_like(ud)
        ctx.residual(ud, R)
        ctx.jvp(ud, R, vd, Jv, eps=1e-7)
        torch.cuda.synchronize()
        out.append((to_host(R), to_host(Jv)))
    (R1, J1), (R2, J2) = out
    assert np.abs(R2 - R1[perm]).max() <= 1e-12 * np.abs(R1).max()
    assert np.abs(J2 - J1[perm]).max() <= 1e-7 * np.abs(J1).max()
