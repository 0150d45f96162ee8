"""Pins of the oracle's BDF2 time stepping (App. D)."""
import numpy as np

import workloads as w
from oracle import dynamics as dy
from oracle import precond as pc
from oracle import residual as rs


def free_block(p=1, material=w.LINEAR_ELASTIC, f=(0.3, -0.2, 0.1)):
    """A perturbed block with every face traction-free under a uniform body force."""
    mesh = w.box_mesh((4, 3, 3), lengths=(2.0, 1.0, 1.0), perturb=0.15, seed=3)
    fb = np.asarray(f)
    loads = w.Loads(3, lambda xc, n: np.full(xc.shape[0], w.fields.TRAC, np.int32),
                    lambda x: np.zeros_like(x), lambda x, n: np.zeros_like(x),
                    lambda x: np.tile(fb, (x.shape[0], 1)))
    return w.Problem("free", mesh, p, 20 if p == 1 else 40, 2, material, 1.0, 1.5, loads,
                     stencil_quantum=1e-6), fb


def test_bdf2_is_exact_for_a_uniformly_accelerating_free_body():
    """u(t) = a t^2 / 2 with a = f / rho, uniform in space, is stress free, so the
    momentum balance is rho a = f exactly; BDF2 differentiates quadratics in t
    exactly, so from the exact history every step reproduces u(t)."""
    prob, fb = free_block()
    disc = rs.build(prob)
    n = disc.n_cells
    rho, dt = 2.0, 0.05
    a = fb / rho
    exact_u = lambda t: np.tile(0.5 * a * t * t, (n, 1))
    exact_v = lambda t: np.tile(a * t, (n, 1))
    hist = (exact_u(0.0), exact_u(-dt), exact_v(0.0), exact_v(-dt))
    for k in range(1, 4):
        u, hist, st = dy.step(disc, rho, dt, hist, tol=1e-12, eta=1e-10, m=60, maxit_krylov=400)
        assert np.abs(u - exact_u(k * dt)).max() <= 1e-9 * np.abs(exact_u(k * dt)).max()
        assert np.abs(hist[2] - exact_v(k * dt)).max() <= 1e-8 * np.abs(exact_v(k * dt)).max()


def test_bdf2_residual_vanishes_on_the_exact_trajectory():
    """The step residual R(u) + s - m u at the exact u(t_1) is zero to round-off
    for the free body, neo-Hookean too (a rigid translation is stress free)."""
    for material in (w.LINEAR_ELASTIC, w.NEO_HOOKEAN):
        prob, fb = free_block(material=material)
        disc = rs.build(prob)
        n = disc.n_cells
        rho, dt, t0 = 1.3, 0.1, 0.7  # a moving start: every history term is non-zero
        a = fb / rho
        u_at = lambda t: np.tile(0.5 * a * t * t, (n, 1))
        v_at = lambda t: np.tile(a * t, (n, 1))
        u_t, u_tm1, v_t, v_tm1 = u_at(t0 + dt), u_at(t0), v_at(t0 + dt), v_at(t0)
        inertia = (dy.mass(disc, rho, dt), dy.source(disc, rho, dt, u_t, u_tm1, v_t, v_tm1))
        u1 = u_at(t0 + 2 * dt)
        R = rs.residual(disc, u1, 1.0, inertia)
        assert np.abs(R).max() <= 1e-12 * np.abs(inertia[1]).max()
        # a wrong position (u_t instead) leaves m (u1 - u_t) behind
        assert np.abs(rs.residual(disc, u_t, 1.0, inertia)).max() > 1e-3 * np.abs(inertia[1]).max()


def test_inertia_adds_the_mass_to_the_approximate_jacobian_diagonal():
    prob, _ = free_block()
    disc = rs.build(prob)
    m = dy.mass(disc, 2.0, 0.1)
    A0, A1 = pc.assemble(disc), pc.assemble(disc, m)
    assert np.allclose((A0 - A1).toarray(), np.diag(m))
    assert np.allclose(m, 9 * 2.0 * disc.vol / (4 * 0.01))
