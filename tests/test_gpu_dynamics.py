"""GPU parity of the BDF2 time stepping (App. D) through the C ABI."""
import numpy as np
import pytest

import workloads as w
from oracle import dynamics as ody
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


def free_block():
    mesh = w.box_mesh((4, 3, 3), lengths=(2.0, 1.0, 1.0), perturb=0.15, seed=3)
    fb = np.array([0.3, -0.2, 0.1])
    loads = w.Loads(3, lambda xc, n: np.full(xc.shape[0], w.fields.TRAC, np.int32),
                    lambda x: np.zeros_like(x), lambda x, n: np.zeros_like(x),
                    lambda x: np.tile(fb, (x.shape[0], 1)))
    return w.Problem("free", mesh, 1, 20, 2, w.LINEAR_ELASTIC, 1.0, 1.5, loads, stencil_quantum=1e-6), fb


def test_bdf2_free_body_accelerates_exactly():
    """A stress-free uniform acceleration a = f / rho is reproduced exactly from
    an exact history (BDF2 differentiates quadratics in t exactly)."""
    prob, fb = free_block()
    ctx = _api().context_for(prob)
    n = prob.mesh.n_cells
    rho, dt = 2.0, 0.05
    a = fb / rho
    U = lambda t: to_dev(np.tile(0.5 * a * t * t, (n, 1)))
    V = lambda t: to_dev(np.tile(a * t, (n, 1)))
    ctx.set_dynamics(rho, dt)
    ctx.dyn_reset(U(0.0), V(0.0), U(-dt), V(-dt))
    u = U(0.0)
    for k in range(1, 4):
        st = ctx.dyn_step(u, tol=1e-12, eta=1e-10, restart=60, max_krylov=400)
        assert st["converged"]
        ex = np.tile(0.5 * a * (k * dt) ** 2, (n, 1))
        assert np.abs(to_host(u) - ex).max() <= 1e-9 * np.abs(ex).max()


def test_bdf2_neo_hookean_beam_matches_oracle():
    """A clamped neo-Hookean beam set moving from rest by a sudden tip traction:
    four time steps on the GPU and in the oracle reach the same states."""
    prob = w.cantilever(shape=(8, 2, 2), p=1, n_plus=20)
    prob.mesh = w.box_mesh((8, 2, 2), lengths=(4.0, 1, 1))
    prob.loads = w.fields.cantilever_loads(4.0, (0.0, -0.02, 0.01))
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
    kw = dict(tol=1e-10, eta=1e-8, max_line_search=-1)
    for k in range(4):
        st = ctx.dyn_step(u, restart=96, max_krylov=400, **kw)
        assert st["converged"]
        uo, hist, _ = ody.step(disc, rho, dt, hist, m=96, maxit_krylov=400, ls_max=-1, tol=1e-10, eta=1e-8)
        assert np.linalg.norm(to_host(u) - uo) <= 1e-7 * np.linalg.norm(uo)
    assert np.abs(to_host(u)[:, 1]).max() > 1e-2  # the beam has moved


def test_dynamics_state_rules():
    prob = w.cantilever(shape=(60, 6, 6), p=1, n_plus=20)
    ctx = _api().context_for(prob, precond_levels=8)
    n = prob.mesh.n_cells
    u = torch.zeros((3, n), device=DEV, dtype=torch.float64)
    R0 = torch.empty_like(u)
    ctx.residual(u, R0)
    ctx.set_dynamics(1.0, 0.1)
    with pytest.raises(_api().HofvError):
        ctx.set_multigrid(True)  # built for the static operator
    with pytest.raises(_api().HofvError):
        ctx.dyn_step(u)  # no history yet
    with pytest.raises(_api().HofvError):
        ctx.set_dynamics(1.0, 0.0)
    ctx.set_dynamics(0.0, 0.0)  # static again
    R1 = torch.empty_like(u)
    ctx.residual(u, R1)
    assert torch.equal(R0, R1)
    ctx.set_multigrid(True)
