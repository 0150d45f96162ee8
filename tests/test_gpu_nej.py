"""GPU parity of the near-exact Jacobian (App. C): its matrix-free product, its
inner GMRES application and the solvers preconditioned by it."""
import numpy as np
import pytest

import workloads as w
from oracle import dynamics as ody
from oracle import jacobian as ojac
from oracle import krylov as okr
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


def _sweeps32(disc, sweeps=2):
    A = opc.assemble(disc)
    col = opc.greedy_colours(A)
    n, D = disc.n_cells, disc.dim
    return lambda v: opc.sgs(A, col, v.reshape(n, D), sweeps, dtype=np.float32).astype(float).ravel()


@pytest.mark.parametrize("prob_fn", [lambda: w.cube_mms(5, 2, perturb=0.2),
                                     lambda: w.cube_mms(5, 3, perturb=0.0),
                                     lambda: w.square_mms(8, 3, perturb=0.2),
                                     lambda: w.poly_patch(w.box_mesh((6, 5, 5), perturb=0.2, seed=4, mode="tensor"),
                                                          2, 2, seed=6, symmetric=True)])
def test_nej_apply_parity(prob_fn):
    prob = prob_fn()
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n, D = disc.n_cells, disc.dim
    A = onej.operator(disc)
    v = w.random_state(n, D, seed=31, scale=1.0)
    out = torch.empty((D, n), device=DEV, dtype=torch.float64)
    ctx.nej_apply(to_dev(v), out)
    torch.cuda.synchronize()
    ref = (A @ v.ravel()).reshape(n, D)
    assert np.linalg.norm(to_host(out) - ref) <= 1e-10 * np.linalg.norm(ref)
    ctx.nej_apply(torch.zeros((D, n), device=DEV, dtype=torch.float64), out)
    torch.cuda.synchronize()
    assert not torch.any(out)
    # the residual itself is unchanged afterwards (loads and stabilisation restored)
    R = torch.empty_like(out)
    ctx.residual(to_dev(v), R)
    torch.cuda.synchronize()
    Ro = ores.residual(disc, v)
    assert np.linalg.norm(to_host(R) - Ro) <= 1e-10 * np.linalg.norm(Ro)


def test_nej_apply_with_dynamics_includes_the_mass_term():
    prob = w.cube_mms(5, 2, perturb=0.2)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    rho, dt = 2.0, 0.05
    ctx.set_dynamics(rho, dt)
    z = to_dev(np.zeros((n, 3)))
    ctx.dyn_reset(z, z, z, z)
    A = onej.operator(disc, mass=ody.mass(disc, rho, dt))
    v = w.random_state(n, 3, seed=32, scale=1.0)
    out = torch.empty((3, n), device=DEV, dtype=torch.float64)
    ctx.nej_apply(to_dev(v), out)
    torch.cuda.synchronize()
    ref = (A @ v.ravel()).reshape(n, 3)
    assert np.linalg.norm(to_host(out) - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("k", [1, 3])
def test_nej_precond_parity(k):
    """k inner GMRES iterations on the NEJ, right-preconditioned by the FP32
    sweeps, against the oracle's with the FP32-emulated sweeps."""
    prob = w.cube_mms(6, 2, perturb=0.2)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    ctx.set_multigrid(False)
    n = disc.n_cells
    A = onej.operator(disc)
    r = w.random_state(n, 3, seed=33, scale=1.0)
    ctx.set_nej(k)
    z = torch.empty((3, n), device=DEV, dtype=torch.float64)
    ctx.precond_apply(to_dev(r), z, n_sweeps=2)
    torch.cuda.synchronize()
    zo = onej.gmres_fixed(lambda x: A @ x, r.ravel(), k, _sweeps32(disc)).reshape(n, 3)
    assert np.abs(to_host(z) - zo).max() <= 1e-4 * np.abs(zo).max()
    # switched off, the preconditioner is the sweeps again
    ctx.set_nej(0)
    ctx.precond_apply(to_dev(r), z, n_sweeps=2)
    torch.cuda.synchronize()
    z32 = _sweeps32(disc)(r.ravel()).reshape(n, 3)
    assert np.abs(to_host(z) - z32).max() <= 1e-5 * np.abs(z32).max()


def test_fgmres_with_nej_matches_oracle():
    """A linear system of the full J at p = 3 on regular hexahedra: FGMRES with
    the NEJ (4 inner iterations) solves it, in as many outer iterations as the
    oracle's and fewer than with the sweeps alone."""
    prob = w.cube_mms(6, 3, perturb=0.0)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    ctx.set_multigrid(False)
    n = disc.n_cells
    ud = to_dev(np.zeros((n, 3)))
    Ru = torch.empty_like(ud)
    ctx.residual(ud, Ru)
    b = w.random_state(n, 3, seed=7, scale=1.0)
    x = torch.zeros_like(ud)
    st_aj = ctx.fgmres_solve(ud, Ru, to_dev(b), x, rtol=1e-7, max_iters=500, n_sweeps=2)
    ctx.set_nej(4)
    x.zero_()
    st = ctx.fgmres_solve(ud, Ru, to_dev(b), x, rtol=1e-7, max_iters=500, n_sweeps=2)
    assert st["converged"] and st["rel_residual"] <= 1e-7
    J = ojac.jacobian_affine(disc)
    xe = np.linalg.solve(J, b.ravel()).reshape(n, 3)
    assert np.linalg.norm(to_host(x) - xe) <= 1e-5 * np.linalg.norm(xe)
    A = onej.operator(disc)
    M = _sweeps32(disc)
    _, info = okr.fgmres(lambda v: J @ v, b.ravel(), lambda v: onej.gmres_fixed(lambda y: A @ y, v, 4, M),
                         rtol=1e-7, maxit=500)
    assert info["converged"]
    assert abs(st["iters"] - info["iters"]) <= 2
    assert st["iters"] < st_aj["iters"]


def test_newton_with_nej_matches_oracle():
    prob = w.cube_mms(6, 2, perturb=0.2)
    disc = ores.build(prob)
    ctx = _api().context_for(prob)
    n = disc.n_cells
    ctx.set_nej(4)
    u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    st = ctx.newton_solve(u, tol=1e-10, eta=1e-8, restart=60)
    assert st["converged"]
    uo, _ = onw.newton(disc, np.zeros((n, 3)), tol=1e-10, eta=1e-8, m=60)
    assert np.linalg.norm(to_host(u) - uo) <= 1e-7 * np.linalg.norm(uo)


def test_nej_argument_errors():
    api = _api()
    prob = w.cube_mms(5, 2, perturb=0.2)
    ctx = api.context_for(prob)
    n = prob.mesh.n_cells
    ud = to_dev(np.zeros((n, 3)))
    Ru = torch.empty_like(ud)
    ctx.residual(ud, Ru)
    x = torch.zeros_like(ud)
    b = to_dev(w.random_state(n, 3, seed=1, scale=1.0))
    with pytest.raises(api.HofvError):
        ctx.set_nej(65)
    with pytest.raises(api.HofvError):
        ctx.set_nej(-1)
    with pytest.raises(api.HofvError):
        ctx.nej_apply(ud, ud)
    ctx.set_nej(2)
    with pytest.raises(api.HofvError):
        ctx.fgmres_solve(ud, Ru, b, x, side=1)
    with pytest.raises(api.HofvError):
        ctx.fgmres_solve(ud, Ru, b, x, learned=True)
    with pytest.raises(api.HofvError):
        ctx.precond_apply(b, x, learned=True)
    nh = api.context_for(w.cantilever(shape=(8, 2, 2), p=1, n_plus=20))
    with pytest.raises(api.HofvError):
        nh.set_nej(2)
    with pytest.raises(api.HofvError):
        nh.nej_apply(torch.zeros((3, 32), device=DEV, dtype=torch.float64),
                     torch.zeros((3, 32), device=DEV, dtype=torch.float64))
