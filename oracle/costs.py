"""Stage costs c_t^x, c_t^u of the benchmark problems (oracle side; test
infrastructure only).

* diag     -- c_t^x(x) = 1/2 x' diag(Qd_t) x + q_t' x,
              c_t^u(u) = 1/2 u' diag(Rd_t) u + r_t' u   (the QP form of Sec. 3.1)
* softplus -- tracking cost whose diagonal weights are softplus functions of a
              parameter vector theta, one block of weights per horizon phase:
              c_t^x(x) = 1/2 sum_i w_{t,i} (x_i - xref_i)^2, c_t^u(u) = 1/2 sum_j w_{t,j} u_j^2.

``stage_x``/``stage_u`` return (value, gradient, Hessian) in closed form.  The
optional ``cp`` argument overrides the differentiable cost parameters (a dict
with the keys of ``cost_param_names``) so that the backward pass can
differentiate the QP data with respect to them by complex step.  All functions
propagate complex arrays.
"""
from __future__ import annotations

import numpy as np


def softplus(v):
    return np.log(1.0 + np.exp(v))


def cost_param_names(prob):
    """Names of the differentiable cost parameters of the problem."""
    return ("Qd", "q", "Rd", "r") if prob["cost"] == "diag" else ("theta", "xref")


def cost_params(prob):
    return {k: prob[k] for k in cost_param_names(prob)}


def _phase(prob, t):
    P, T = prob["phases"], prob["T"]
    return min((P * t) // T, P - 1)


def softplus_weights(prob, t, cp):
    """(wx [nx], wu [nu]) of stage t for the softplus cost."""
    th = cp["theta"]
    nu, nw = prob["nu"], prob["nw"]
    k = _phase(prob, t)
    w = prob["wscale"] * softplus(th[k * (nw + nu):(k + 1) * (nw + nu)])
    wx = np.concatenate([w[:nw], prob["wfix"].astype(w.dtype)])
    return wx, w[nw:]


def stage_x(prob, t, x, cp=None):
    cp = cost_params(prob) if cp is None else cp
    if prob["cost"] == "diag":
        Qd, q = cp["Qd"][t], cp["q"][t]
        return 0.5 * np.sum(Qd * x * x) + np.sum(q * x), Qd * x + q, np.diag(Qd)
    wx, _ = softplus_weights(prob, t, cp)
    d = x - cp["xref"]
    return 0.5 * np.sum(wx * d * d), wx * d, np.diag(wx)


def stage_u(prob, t, u, cp=None):
    cp = cost_params(prob) if cp is None else cp
    if prob["cost"] == "diag":
        Rd, r = cp["Rd"][t], cp["r"][t]
        return 0.5 * np.sum(Rd * u * u) + np.sum(r * u), Rd * u + r, np.diag(Rd)
    _, wu = softplus_weights(prob, t, cp)
    return 0.5 * np.sum(wu * u * u), wu * u, np.diag(wu)
