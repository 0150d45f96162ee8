"""GPU parity of the preconditioner sweeps, FGMRES and Newton solves."""
import numpy as np
import pytest

import workloads as w
from oracle import jacobian as ojac
from oracle import krylov as okr
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


@pytest.mark.parametrize("prob_fn", [lambda: w.square_mms(16, 2, perturb=0.2),
                                     lambda: w.cube_mms(9, 2, perturb=0.2),
                                     lambda: w.cantilever(shape=(16, 4, 4), p=1, n_plus=20),
                                     lambda: w.poly_patch(w.box_mesh((8, 6, 6), perturb=0.2, seed=4, mode="tensor"),
                                                          2, 2, seed=6, symmetric=True)])
@pytest.mark.parametrize("sweeps", [1, 3])
def test_precond_parity(prob_fn, sweeps):
    prob = prob_fn()
    disc = ores.build(prob)
    A = opc.assemble(disc)
    col = opc.greedy_colours(A)
    ctx = _api().context_for(prob)
    r = w.random_state(disc.n_cells, disc.dim, seed=3, scale=1.0)
    z = torch.empty((disc.dim, disc.n_cells), device=DEV, dtype=torch.float64)
    ctx.precond_apply(to_dev(r), z, n_sweeps=sweeps)
    torch.cuda.synchronize()
    z64 = opc.sgs(A, col, r, sweeps)
    z32 = opc.sgs(A, col, r, sweeps, dtype=np.float32)
    zg = to_host(z)
    assert np.abs(zg - z64).max() <= 1e-5 * np.abs(z64).max()
    assert np.abs(zg - z32).max() <= 1e-5 * np.abs(z64).max()
    assert ctx.report["n_colours"] == col.max() + 1


def test_fgmres_parity_linear_system():
    prob = w.cube_mms(8, 2, perturb=0.2)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    u = np.zeros((n, 3))
    ud = to_dev(u)
    Ru = torch.empty_like(ud)
    ctx.residual(ud, Ru)
    b = w.random_state(n, 3, seed=7, scale=1.0)
    x = torch.zeros_like(ud)
    # the finite-difference product carries ~1e-9 relative noise, so ask 1e-7
    st = ctx.fgmres_solve(ud, Ru, to_dev(b), x, rtol=1e-7, max_iters=500, n_sweeps=2)
    assert st["converged"] and st["rel_residual"] <= 1e-7
    J = ojac.jacobian_affine(disc)
    xe = np.linalg.solve(J, b.ravel()).reshape(n, 3)
    assert np.linalg.norm(to_host(x) - xe) <= 1e-5 * np.linalg.norm(xe)


@pytest.mark.parametrize("side", [0, 1])
def test_one_pass_gram_schmidt_matches_oracle(side):
    """gs_passes = 1 (classical Gram-Schmidt once, PETSc's default): the linear
    solve reaches the dense solution, and Newton on the 8^3 p = 2 cube equals
    the oracle's Newton with one pass (100 tol), right and left preconditioned."""
    prob = w.cube_mms(8, 2, perturb=0.2)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    ud = to_dev(np.zeros((n, 3)))
    Ru = torch.empty_like(ud)
    ctx.residual(ud, Ru)
    b = w.random_state(n, 3, seed=7, scale=1.0)
    x = torch.zeros_like(ud)
    st = ctx.fgmres_solve(ud, Ru, to_dev(b), x, rtol=1e-7, max_iters=500, n_sweeps=2, side=side, gs_passes=1)
    assert st["converged"]
    xe = np.linalg.solve(ojac.jacobian_affine(disc), b.ravel()).reshape(n, 3)
    assert np.linalg.norm(to_host(x) - xe) <= 1e-5 * np.linalg.norm(xe)
    tol = 1e-9
    u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    st = ctx.newton_solve(u, tol=tol, eta=1e-6, side=side, gs_passes=1)
    assert st["converged"]
    ug = to_host(u)
    R0 = np.linalg.norm(ores.residual(disc, np.zeros((n, 3))))
    assert np.linalg.norm(ores.residual(disc, ug)) <= 1.01 * tol * R0
    uo, _ = onw.newton(disc, np.zeros((n, 3)), tol=tol, eta=1e-6, side=side, passes=1)
    assert np.linalg.norm(ug - uo) <= 100 * tol * np.linalg.norm(uo)
    bad = _api().HofvError
    with pytest.raises(bad):
        ctx.fgmres_solve(ud, Ru, to_dev(b), x, gs_passes=3)


def test_left_gmres_parity_linear_system():
    """side = 1 (eq. jfnk as printed): GMRES on M J x = M b with the FP32 sweeps
    as M; the stopping test is on the preconditioned residual, which the oracle's
    left GMRES with the FP32-emulated sweeps reproduces."""
    prob = w.cube_mms(8, 2, perturb=0.2)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    ud = to_dev(np.zeros((n, 3)))
    Ru = torch.empty_like(ud)
    ctx.residual(ud, Ru)
    b = w.random_state(n, 3, seed=7, scale=1.0)
    x = torch.zeros_like(ud)
    st = ctx.fgmres_solve(ud, Ru, to_dev(b), x, rtol=1e-7, max_iters=500, n_sweeps=2, side=1)
    assert st["converged"] and st["rel_residual"] <= 1e-7
    J = ojac.jacobian_affine(disc)
    A = opc.assemble(disc)
    col = opc.greedy_colours(A)
    M = lambda v: opc.sgs(A, col, v.reshape(n, 3), 2, dtype=np.float32).astype(float).ravel()
    xo, info = okr.gmres_left(lambda v: J @ v, b.ravel(), M, m=30, rtol=1e-7, maxit=500)
    assert info["converged"]
    xe = np.linalg.solve(J, b.ravel()).reshape(n, 3)
    assert np.linalg.norm(to_host(x) - xe) <= 1e-5 * np.linalg.norm(xe)
    assert abs(st["iters"] - info["iters"]) <= 2
    Mr = M((b.ravel() - J @ to_host(x).ravel()))
    assert np.linalg.norm(Mr) <= 1.01e-7 * np.linalg.norm(M(b.ravel()))
    with pytest.raises(_api().HofvError):
        ctx.fgmres_solve(ud, Ru, to_dev(b), x, side=2)
    with pytest.raises(_api().HofvError):
        ctx.fgmres_solve(ud, Ru, to_dev(b), x, side=1, learned=True)


def test_newton_left_gmres_matches_oracle():
    prob = w.cube_mms(6, 2, perturb=0.2)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    st = ctx.newton_solve(u, tol=1e-10, eta=1e-7, side=1)
    assert st["converged"]
    uo, _ = onw.newton(disc, np.zeros((n, 3)), tol=1e-10, eta=1e-7, side=1)
    assert np.linalg.norm(to_host(u) - uo) <= 1e-7 * np.linalg.norm(uo)


def test_newton_with_symmetry_faces_matches_oracle():
    """A symmetric quadratic field on a box whose x = 0 faces are symmetry planes
    (p = 2, exact for it): Newton on the GPU and in the oracle reach the same
    state, which is the field itself."""
    prob = w.poly_patch(w.box_mesh((6, 5, 5), perturb=0.2, seed=4, mode="tensor"), 2, 2, seed=6, symmetric=True)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    st = ctx.newton_solve(u, tol=1e-10, eta=1e-8, restart=60)
    assert st["converged"]
    uo, _ = onw.newton(disc, np.zeros((n, 3)), tol=1e-10, eta=1e-8, m=60)
    ue = prob.loads.exact.value(disc.cen)
    assert np.linalg.norm(to_host(u) - uo) <= 1e-7 * np.linalg.norm(uo)
    assert np.linalg.norm(to_host(u) - ue) <= 1e-7 * np.linalg.norm(ue)


def test_fgmres_nonzero_initial_guess_and_zero_rhs():
    prob = w.square_mms(10, 2)
    ctx = _api().context_for(prob)
    n = prob.mesh.n_cells
    ud = torch.zeros((2, n), device=DEV, dtype=torch.float64)
    Ru = torch.empty_like(ud)
    ctx.residual(ud, Ru)
    b = to_dev(w.random_state(n, 2, seed=1, scale=1.0))
    x = to_dev(w.random_state(n, 2, seed=2, scale=1.0))
    st = ctx.fgmres_solve(ud, Ru, b, x, rtol=1e-7, max_iters=300)
    assert st["converged"]
    Jx = torch.empty_like(x)
    ctx.jvp(ud, Ru, x, Jx)
    torch.cuda.synchronize()
    assert torch.linalg.norm(Jx - b) <= 2e-7 * torch.linalg.norm(b)
    x2 = torch.ones_like(x)
    st = ctx.fgmres_solve(ud, Ru, torch.zeros_like(b), x2)
    assert st["iters"] == 0 and not torch.any(x2)


def test_newton_square_mms_matches_oracle():
    """The 2D 32x32 p = 2 manufactured problem solved to 1e-10 (the config's tolerance)."""
    prob = w.square_mms(32, 2)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    u = torch.zeros((2, n), device=DEV, dtype=torch.float64)
    st = ctx.newton_solve(u, tol=1e-10, eta=1e-4)
    assert st["converged"] and st["newton_iters"] <= 4
    ug = to_host(u)
    tol = 1e-10
    R0 = np.linalg.norm(ores.residual(disc, np.zeros((n, 2))))
    assert np.linalg.norm(ores.residual(disc, ug)) <= 1.01 * tol * R0
    uo, _ = onw.newton(disc, np.zeros((n, 2)), tol=tol, eta=1e-4)
    assert np.linalg.norm(ug - uo) <= 100 * tol * np.linalg.norm(uo)
    ue = prob.loads.exact.value(disc.cen)
    assert np.sqrt(np.mean(np.sum((ug - ue) ** 2, 1))) < 2e-3


@pytest.mark.parametrize("ls_max", [10, -1])
def test_newton_neo_hookean_block_matches_oracle(ls_max):
    """A stubby neo-Hookean block clamped at x = 0 with a dead end traction,
    3 load increments, to 1e-8 per increment, with backtracking and with full
    Newton steps."""
    prob = w.cantilever(shape=(6, 4, 4), p=2, n_plus=40, n_increments=3)
    prob.mesh = w.box_mesh((6, 4, 4), lengths=(1.5, 1, 1), perturb=0.1, seed=1)
    prob.loads = w.fields.cantilever_loads(1.5, (0.0, -0.05, 0.02))
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    st = ctx.newton_solve(u, tol=1e-8, eta=1e-4, n_increments=3, max_line_search=ls_max)
    assert st["converged"]
    ug = to_host(u)
    tol = 1e-8
    uo, ost = onw.newton(disc, np.zeros((n, 3)), tol=tol, eta=1e-4, n_increments=3, ls_max=ls_max)
    assert np.linalg.norm(ug - uo) <= 100 * tol * np.linalg.norm(uo)
    # the last increment's reference: ||R|| of the previous increment's state at
    # full load (the oracle's; the GPU's agrees to the solve tolerance)
    r0_last = ost["increments"][-1]["r0"]
    assert np.linalg.norm(ores.residual(disc, ug)) <= 1.01 * tol * r0_last


MG_CASES = [lambda: w.cube_mms(12, 2, perturb=0.2),
            lambda: w.cube_mms((10, 10, 10), 1, perturb=0.2, lengths=(1.0, 1.0, 0.1)),
            lambda: w.cantilever(shape=(60, 6, 6), p=1, n_plus=20)]


@pytest.mark.parametrize("prob_fn", MG_CASES)
def test_multigrid_precond_parity(prob_fn):
    """The GPU V-cycle (FP32) against the oracle's V-cycle (FP64 and FP32)."""
    prob = prob_fn()
    disc = ores.build(prob)
    lev = opc.hierarchy(opc.assemble(disc))
    ctx = _api().context_for(prob, precond_levels=8)
    r = w.random_state(disc.n_cells, disc.dim, seed=4, scale=1.0)
    z = torch.empty((disc.dim, disc.n_cells), device=DEV, dtype=torch.float64)
    ctx.precond_apply(to_dev(r), z, n_sweeps=2)
    torch.cuda.synchronize()
    zg = to_host(z)
    z64 = opc.vcycle(lev, r, 2)
    z32 = opc.vcycle(lev, r, 2, dtype=np.float32)
    assert np.abs(zg - z64).max() <= 1e-4 * np.abs(z64).max()
    assert np.abs(zg - z32).max() <= 1e-4 * np.abs(z64).max()


def test_long_cycle_fgmres_solves_a_slender_neo_hookean_beam():
    """A clamped 60x6x6 neo-Hookean beam with free sides at load 0.1: with the
    V-cycle and a 600-vector cycle FGMRES reaches 1e-6 (the true residual,
    recomputed); the sweeps alone are far from it after as many iterations."""
    prob = w.cantilever(shape=(60, 6, 6), p=1, n_plus=20)
    rel, its = {}, {}
    for levels in (1, 8):
        ctx = _api().context_for(prob, precond_levels=levels)
        n = prob.mesh.n_cells
        u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
        R = torch.empty_like(u)
        ctx.set_load_scale(0.1)
        ctx.residual(u, R)
        x = torch.zeros_like(u)
        st = ctx.fgmres_solve(u, R, -R, x, restart=600, max_iters=600, rtol=1e-6, check=False)
        rel[levels], its[levels] = st["rel_residual"], st["iters"]
        Jx = torch.empty_like(u)
        ctx.jvp(u, R, x, Jx)
        true = float(torch.linalg.norm(Jx + R) / torch.linalg.norm(R))
        assert abs(true - rel[levels]) <= 0.05 * rel[levels] + 1e-9
    print("beam FGMRES(600) relative residual / iterations (sweeps, multigrid):", rel, its)
    assert rel[8] <= 1e-6 and its[8] < 600
    assert rel[1] > 100 * rel[8]
    # cycles are capped at 2048 vectors: a longer one is an argument error
    with pytest.raises(_api().HofvError):
        ctx.fgmres_solve(u, R, -R, x, restart=4096, max_iters=10)
    with pytest.raises(_api().HofvError):
        ctx.newton_solve(u, restart=2049, max_newton=1)


def test_newton_eisenstat_walker_forcing_matches_oracle():
    """forcing = 1 on the tip-loaded beam: the GPU reaches the oracle's state with
    fewer Krylov iterations than a constant Krylov tolerance needs."""
    prob = w.cantilever(shape=(8, 2, 2), p=1, n_plus=20, n_increments=2)
    prob.mesh = w.box_mesh((8, 2, 2), lengths=(4.0, 1, 1))
    prob.loads = w.fields.cantilever_loads(4.0, (0.0, -0.02, 0.0))
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    kw = dict(tol=1e-10, n_increments=2, max_line_search=-1, restart=96, max_krylov=200, max_newton=12)
    u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    st0 = ctx.newton_solve(u, eta=1e-7, **kw)
    u.zero_()
    st1 = ctx.newton_solve(u, eta=0.5, forcing=1, **kw)
    assert st0["converged"] and st1["converged"]
    assert st1["krylov_iters"] < 0.7 * st0["krylov_iters"]
    uo, _ = onw.newton(disc, np.zeros((n, 3)), tol=1e-10, eta=0.5, forcing=1, m=96, maxit_krylov=200,
                       n_increments=2, ls_max=-1, maxit_newton=12)
    assert np.linalg.norm(to_host(u) - uo) <= 1e-7 * np.linalg.norm(uo)
    with pytest.raises(_api().HofvError):
        ctx.newton_solve(u, forcing=2)


def test_newton_secant_predictor_matches_oracle():
    """predictor = 1 over four increments of the tip-loaded beam: fewer Newton
    steps than without it, and the oracle's state."""
    prob = w.cantilever(shape=(8, 2, 2), p=1, n_plus=20, n_increments=4)
    prob.mesh = w.box_mesh((8, 2, 2), lengths=(4.0, 1, 1))
    prob.loads = w.fields.cantilever_loads(4.0, (0.0, -0.02, 0.0))
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    kw = dict(tol=1e-10, eta=1e-7, n_increments=4, max_line_search=-1, restart=96, max_krylov=200, max_newton=12)
    u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    st0 = ctx.newton_solve(u, **kw)
    u.zero_()
    st1 = ctx.newton_solve(u, predictor=1, **kw)
    assert st0["converged"] and st1["converged"]
    assert st1["newton_iters"] < st0["newton_iters"]
    uo, _ = onw.newton(disc, np.zeros((n, 3)), tol=1e-10, eta=1e-7, m=96, maxit_krylov=200, n_increments=4,
                       ls_max=-1, maxit_newton=12, predictor=1)
    assert np.linalg.norm(to_host(u) - uo) <= 1e-7 * np.linalg.norm(uo)
    with pytest.raises(_api().HofvError):
        ctx.newton_solve(u, predictor=3)


def test_fgmres_stops_when_its_cycles_stall():
    """At a bent state (a quarter of the length of tip deflection) the
    one-sided finite-difference product is linear to ~1e-8; asked for 1e-11,
    FGMRES ends once a cycle no longer reduces the recomputed residual by 1 %,
    long before max_iters, keeping the reduction it reached."""
    prob = w.cantilever(shape=(30, 3, 3), p=1, n_plus=20, n_increments=4)
    prob.mesh = w.box_mesh((30, 3, 3), lengths=(7.5, 1, 1))
    prob.loads = w.fields.cantilever_loads(7.5, (0.0, -0.004, 0.0))
    ctx = _api().context_for(prob, precond_levels=8)
    ctx.set_multigrid(True)
    n = prob.mesh.n_cells
    u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    st = ctx.newton_solve(u, tol=1e-10, eta=0.3, forcing=1, n_increments=4, max_line_search=-1, restart=200,
                          max_krylov=400, max_newton=15)
    assert st["converged"] and float(u[1].abs().max()) > 1.0
    ctx.set_load_scale(1.25)
    R = torch.empty_like(u)
    ctx.residual(u, R)
    x = torch.zeros_like(u)
    ks = ctx.fgmres_solve(u, R, -R, x, restart=200, max_iters=4000, rtol=1e-11, check=False)
    assert ks["stalled"] == 1 and not ks["converged"] and ks["iters"] < 2000
    assert ks["rel_residual"] < 1e-2


def test_newton_full_steps_on_a_tip_loaded_beam_match_oracle():
    """A tip traction bends a neo-Hookean beam by a quarter of its length; full
    Newton steps (max_line_search < 0) converge in a few steps per increment on
    both sides, to the same state."""
    prob = w.cantilever(shape=(8, 2, 2), p=1, n_plus=20, n_increments=2)
    prob.mesh = w.box_mesh((8, 2, 2), lengths=(4.0, 1, 1))
    prob.loads = w.fields.cantilever_loads(4.0, (0.0, -0.02, 0.0))
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    st = ctx.newton_solve(u, tol=1e-10, eta=1e-7, n_increments=2, max_line_search=-1, restart=96,
                          max_krylov=200, max_newton=8)
    assert st["converged"] and st["newton_iters"] <= 14
    uo, _ = onw.newton(disc, np.zeros((n, 3)), tol=1e-10, eta=1e-7, m=96, maxit_krylov=200, n_increments=2,
                       ls_max=-1, maxit_newton=8)
    ug = to_host(u)
    assert np.abs(ug[:, 1]).max() > 0.5
    assert np.linalg.norm(ug - uo) <= 1e-7 * np.linalg.norm(uo)


@pytest.mark.parametrize("mg", [False, True])
def test_graph_replayed_arnoldi_steps_match_launched_ones(mg):
    """graphs = 1 (each Arnoldi step captured as a HIP graph the second time it
    runs, replayed after that) gives the results of graphs = 0 bit for bit: two
    FGMRES solves in a row on the 2D 32^2 problem (the first captures in its
    later cycles, the second replays every step), with the host's reads of
    Hessenberg columns and synchronisations between the replays; then Newton
    over two load increments of a small beam, whose load scale changes between
    increments, so that the captured steps are dropped and captured again (a
    step replayed with the old load would put (s_old - s) src / eps into J.v)."""
    api = _api()
    prob = w.square_mms(32, 2, perturb=0.2)
    ctx = api.context_for(prob, precond_levels=8 if mg else 1)
    ctx.set_multigrid(mg)
    n = prob.mesh.n_cells
    u = to_dev(w.random_state(n, 2, seed=3, scale=0.1))
    Ru = torch.empty_like(u)
    ctx.residual(u, Ru)
    b = to_dev(w.random_state(n, 2, seed=7, scale=1.0))
    runs = {}
    for graphs in (0, 1):
        runs[graphs] = []
        for rep in range(2):
            x = torch.zeros_like(u)
            # three full cycles (the tolerance is out of reach on purpose)
            st = ctx.fgmres_solve(u, Ru, b, x, rtol=1e-14, max_iters=90, restart=30, graphs=graphs, check=False)
            torch.cuda.synchronize()
            runs[graphs].append((x.clone(), st))
            print("graphs", graphs, "solve", rep, {k: st[k] for k in ("iters", "rel_residual", "stalled")})
    for rep in range(2):
        (x0, s0), (x1, s1) = runs[0][rep], runs[1][rep]
        assert torch.equal(x0, x1), rep
        assert (s0["iters"], s0["rel_residual"], s0["stalled"]) == (s1["iters"], s1["rel_residual"], s1["stalled"])
    assert runs[1][0][1]["iters"] > 30  # the first solve itself went past one cycle

    beam = w.cantilever(shape=(8, 2, 2), p=1, n_plus=20, n_increments=2)
    beam.mesh = w.box_mesh((8, 2, 2), lengths=(4.0, 1, 1))
    beam.loads = w.fields.cantilever_loads(4.0, (0.0, -0.02, 0.0))
    bctx = api.context_for(beam)
    kw = dict(tol=1e-10, eta=1e-7, n_increments=2, max_line_search=-1, restart=40, max_krylov=400, max_newton=12)
    res = {}
    for graphs in (0, 1):
        ub = torch.zeros((3, beam.mesh.n_cells), device=DEV, dtype=torch.float64)
        st = bctx.newton_solve(ub, graphs=graphs, check=False, **kw)
        torch.cuda.synchronize()
        res[graphs] = (ub.clone(), st)
        print("graphs", graphs, "newton", st)
    assert res[0][1]["converged"]
    assert torch.equal(res[0][0], res[1][0])
    for k in ("newton_iters", "krylov_iters", "rel_residual"):
        assert res[0][1][k] == res[1][1][k], k
    with pytest.raises(api.HofvError):
        ctx.fgmres_solve(u, Ru, b, torch.zeros_like(u), graphs=2)
