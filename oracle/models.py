"""Dynamics of the benchmark problems (oracle side; test infrastructure only).

``step(prob, t, x, u)`` returns phi_t(x_t, u_t), the next state of the explicit
dynamics.  All functions accept complex arrays so that complex-step
differentiation gives exact Jacobians.

* ltv      -- x_{t+1} = A_t x_t + B_t u_t + c_t (the LQ problems of App. B.1
              and the uneven LTV batch).  Pinned: Riccati closed form, brute
              force (tests).
* cartpole -- the cart-pole of App. B.2 *as printed* (its equations for the
              cart acceleration and the pole acceleration), explicit Euler.
              Pinned against special cases of the printed equations
              (upright rest, horizontal pole, linearisation at the upright).
* bicycle  -- a dynamic single-track model with Pacejka-type lateral tyre
              forces, built for the drift-shaped differentiation workload;
              the paper does not print its vehicle model, so this one is
              defined here.  Parity unpinned against the paper (only pinned
              by invariants: straight driving at zero slip, symmetry).
"""
from __future__ import annotations

import numpy as np


def step(prob, t, x, u):
    kind = prob["dyn"]
    if kind == "ltv":
        return prob["A"][t] @ x + prob["B"][t] @ u + prob["c"][t]
    if kind == "cartpole":
        return cartpole_step(prob["params"], x, u)
    if kind == "bicycle":
        return bicycle_step(prob["params"], x, u)
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# Cart-pole (App. B.2), explicit Euler
# ---------------------------------------------------------------------------
def cartpole_xdot(params, x, u):
    m_c, m_p, L, g = params[0], params[1], params[2], params[3]
    M = m_p + m_c
    x1, x2, x3, x4 = x[0], x[1], x[2], x[3]
    s, c = np.sin(x3), np.cos(x3)
    den = M + m_p * (1.0 - c * c)
    d1 = x2
    d2 = (-m_p * L * s * x4 * x4 + m_p * g * s * c) / (den * L)
    d3 = x4
    d4 = (-m_p * L * s * x4 + m_p * g * s * c + u[0]) / den
    return np.array([d1, d2, d3, d4])


def cartpole_step(params, x, u):
    dt = params[4]
    return x + dt * cartpole_xdot(params, x, u)


# ---------------------------------------------------------------------------
# Dynamic single-track ("bicycle") model, explicit Euler
# state (r, v, beta, omega_r, dpsi, e, delta, tau), input (ddelta, dtau)
# ---------------------------------------------------------------------------
def bicycle_xdot(params, x, u):
    (a, b, m, Iz, rw, Iw, Bf, Cf, Df, Br, Cr, Dr, Cx, kappa, _dt, vmin) = params
    r, v, beta, om, dpsi, e, delta, tau = x
    vx = v * np.cos(beta)
    vy = v * np.sin(beta)
    vxs = np.sqrt(vx * vx + vmin * vmin)     # smooth floor of the forward speed
    vs = np.sqrt(v * v + vmin * vmin)
    alpha_f = np.arctan((vy + a * r) / vxs) - delta
    alpha_r = np.arctan((vy - b * r) / vxs)
    Fyf = -Df * np.sin(Cf * np.arctan(Bf * alpha_f))
    Fyr = -Dr * np.sin(Cr * np.arctan(Br * alpha_r))
    slip = (om * rw - vx) / vxs
    Fxr = Dr * np.tanh(Cx * slip / Dr)
    Fx = Fxr - Fyf * np.sin(delta)
    Fy = Fyf * np.cos(delta) + Fyr
    d_r = (a * Fyf * np.cos(delta) - b * Fyr) / Iz
    d_v = (Fx * np.cos(beta) + Fy * np.sin(beta)) / m
    d_beta = (Fy * np.cos(beta) - Fx * np.sin(beta)) / (m * vs) - r
    d_om = (tau - rw * Fxr) / Iw
    d_dpsi = r - kappa * v * np.cos(dpsi + beta) / (1.0 - kappa * e)
    d_e = v * np.sin(dpsi + beta)
    return np.array([d_r, d_v, d_beta, d_om, d_dpsi, d_e, u[0], u[1]])


def bicycle_step(params, x, u):
    dt = params[14]
    return x + dt * bicycle_xdot(params, x, u)
