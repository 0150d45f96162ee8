"""BDF2 time stepping of the momentum equation (paper App. D, eq. inertiaTerm).

Test infrastructure (see package docstring).

The inertia integral of cell P, with one integration point at the centroid
(the paper's setting for its vibrating beam), is rho Omega_P a_P, where the
velocity and the acceleration are both second-order backward differences:

    v^{t+1} = (3 u^{t+1} - 4 u^t + u^{t-1}) / (2 dt)
    a^{t+1} = (3 v^{t+1} - 4 v^t + v^{t-1}) / (2 dt).

Written out in the unknown u^{t+1}_P this is m_P u_P - s_P with

    m_P = 9 rho Omega_P / (4 dt^2),
    s_P = -rho Omega_P [3 (-4 u^t + u^{t-1}) / (2 dt) - 4 v^t + v^{t-1}] / (2 dt),

and the residual of a step is R_P(u) + s_P - m_P u_P: static equilibrium
R = 0 becomes R = rho a Omega (the face and body terms drive the acceleration).
"""
from __future__ import annotations

from .newton import newton


def mass(disc, rho, dt):
    """m_P = 9 rho Omega_P / (4 dt^2), (n_c,)."""
    return 9.0 * rho * disc.vol / (4.0 * dt * dt)


def source(disc, rho, dt, u_t, u_tm1, v_t, v_tm1):
    """s_P of the step from the two previous levels, (n_c, D)."""
    rv = (rho * disc.vol)[:, None]
    return -rv * ((3.0 * (-4.0 * u_t + u_tm1) / (2.0 * dt) - 4.0 * v_t + v_tm1) / (2.0 * dt))


def velocity(u_new, u_t, u_tm1, dt):
    return (3.0 * u_new - 4.0 * u_t + u_tm1) / (2.0 * dt)


def step(disc, rho, dt, hist, load=1.0, **newton_kw):
    """One time step from hist = (u_t, u_tm1, v_t, v_tm1); returns the new
    displacement, the advanced history and Newton's statistics.  The guess is
    u_t."""
    u_t, u_tm1, v_t, v_tm1 = hist
    inertia = (mass(disc, rho, dt), source(disc, rho, dt, u_t, u_tm1, v_t, v_tm1))
    # one increment at the given load factor: scale the loads through n_increments = 1
    u, st = newton(disc, u_t, n_increments=1, inertia=inertia, load_scale=load, **newton_kw)
    v = velocity(u, u_t, u_tm1, dt)
    return u, (u, u_t, v, v_t), st
