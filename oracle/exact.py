"""Exact-Hessian variant of the KKT system (oracle side; test infrastructure
only).  Reported beside the Gauss-Newton method, never gated.

The method of the paper forms the QP with the Hessians of the costs only
(Eq. QPmatrices: Gauss-Newton; Sec. 3.4, "Exact SQP vs iLQR", notes that the
curvature of the dynamics is left out and that gradients lose accuracy for
it).  This module adds that curvature so that the gradient of the true
solution map can be computed and compared:

* ``dyn_hessian``     -- the Hessian over (x_t, u_t) of lam_{t+1}' phi_t, by
                         complex step along one coordinate (exact first
                         derivative) and a central difference of that
                         derivative along the other (complex steps cannot be
                         nested); symmetric to about 1e-10 relative.
* ``stage_blocks``    -- the stage blocks of the Hessian of the Lagrangian,
                         L = c(z) + lam_0'(x_0 - x_s) + sum_t lam_{t+1}' f_t
                         with f_t = x_{t+1} - phi_t(x_t, u_t):
                         W_t = Hess c_t - Hess(lam_{t+1}' phi_t), dense over
                         (x_t, u_t); the last stage carries the cost only.
* ``newton_step``     -- one SQP iteration (Alg. sqp, line search of App. A.3
                         unchanged) whose QP uses W_t projected onto
                         {W >= 1e-6 I} stage by stage (Sec. 3.1, dense
                         eigenvalue clamp) and linear term grad c - W_p zbar.
                         Its fixed points are the KKT points of the OCP, the
                         same as those of the Gauss-Newton iteration.
* ``converge``        -- Newton SQP until ||dz||_inf <= tol.
* ``kkt_exact``       -- K = [[W, J'], [J, 0]] at a KKT point, W unprojected.
* ``vjp_exact``       -- gradient of l(z*(theta)) through the implicit
                         function theorem on the true KKT conditions
                         F = [grad c + J' lam; x_0 - x_s; f_t] = 0:
                         dl/dtheta = -xi' dF/dtheta with K xi = [dl/dz; 0];
                         cost parameters by complex step on grad c, x_s
                         directly (dF/dx_s = -I on the x_0 rows).

Pinned (tests): on linear dynamics W is the cost Hessian and the exact and
Gauss-Newton gradients agree to rounding; at the cart-pole's upright rest the
mixed second derivative of the pole-rate update is the hand-derived -dt m_p L
/ M; the exact gradient matches central differences of the fully converged
solution map (SQP to ||dz||_inf <= 1e-12) on small cart-pole and bicycle
problems; the Gauss-Newton bias (exact minus Gauss-Newton) is reported.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import costs, models, qp, sqp

CS_H = 1e-30      # complex step
CD_DELTA = 1e-5   # central-difference step of the second derivative


def _grad_lam_phi(prob, t, v, n, lam_next):
    """grad over (x, u) of lam_next' phi_t at the real point v = (x, u), by
    complex step (exact to rounding)."""
    k = v.shape[0]
    out = np.empty(k)
    for j in range(k):
        vc = v.astype(np.complex128)
        vc[j] += 1j * CS_H
        out[j] = np.imag(np.dot(lam_next, models.step(prob, t, vc[:n], vc[n:]))) / CS_H
    return out


def dyn_hessian(prob, t, x, u, lam_next, symmetric=True):
    """Hessian over (x_t, u_t) of lam_next' phi_t(x_t, u_t), (nx+nu)^2."""
    x = np.asarray(x, np.float64)
    u = np.asarray(u, np.float64)
    n = x.shape[0]
    v0 = np.concatenate([x, u])
    k = v0.shape[0]
    H = np.empty((k, k))
    for i in range(k):
        e = np.zeros(k)
        e[i] = CD_DELTA
        H[:, i] = (_grad_lam_phi(prob, t, v0 + e, n, lam_next)
                   - _grad_lam_phi(prob, t, v0 - e, n, lam_next)) / (2 * CD_DELTA)
    return 0.5 * (H + H.T) if symmetric else H


def stage_blocks(prob, x, u, lam):
    """W_t (t < T: over (x_t, u_t); t = T: over x_T) of the Hessian of the
    Lagrangian, unprojected."""
    T = prob["T"]
    W = []
    for t in range(T):
        Hx = costs.stage_x(prob, t, x[t])[2]
        Hu = costs.stage_u(prob, t, u[t])[2]
        Wt = np.asarray(sla.block_diag(np.real(Hx), np.real(Hu)), np.float64)
        if prob["dyn"] != "ltv":
            Wt = Wt - dyn_hessian(prob, t, x[t], u[t], lam[t + 1])
        W.append(Wt)
    W.append(np.asarray(np.real(costs.stage_x(prob, T, x[T])[2]), np.float64))
    return W


def _cost_gradient(prob, x, u):
    T = prob["T"]
    gx = [np.real(costs.stage_x(prob, t, x[t])[1]) for t in range(T + 1)]
    gu = [np.real(costs.stage_u(prob, t, u[t])[1]) for t in range(T)]
    return gx, gu


def _with_hessian(prob, x, u, W, project):
    """Dense KKT pieces of the QP at (x, u) (constraints as in Eq. QPmatrices)
    with the stage Hessians replaced by W (optionally projected) and the
    linear term grad c - W zbar."""
    T, nx, nu = prob["T"], prob["nx"], prob["nu"]
    qpd = qp.qp_data(prob, x, u)
    K, rhs, parts = qp.kkt(qpd, prob["x0"])
    K = np.real(K).astype(np.float64)
    rhs = np.real(rhs).astype(np.float64)
    nz = parts["nz"]
    xi = parts["xi"]
    gx, gu = _cost_gradient(prob, x, u)
    for t in range(T + 1):
        Wt = qp.project_pd(W[t]) if project else W[t]
        w = nx + (nu if t < T else 0)
        zt = np.concatenate([x[t], u[t]]) if t < T else np.asarray(x[T], np.float64)
        g = np.concatenate([gx[t], gu[t]]) if t < T else gx[T]
        K[xi[t]:xi[t] + w, xi[t]:xi[t] + w] = Wt
        rhs[xi[t]:xi[t] + w] = -(g - Wt @ zt)
    return K, rhs, parts, qpd


def newton_step(prob, x, u, lam, alphas=sqp.ALPHAS, eta=sqp.ETA):
    """One SQP iteration with the projected exact Hessian at (x, u, lam)."""
    W = stage_blocks(prob, x, u, lam)
    K, rhs, parts, _ = _with_hessian(prob, x, u, W, project=True)
    w = sla.lu_solve(sla.lu_factor(K), rhs)
    xp, up, lp = qp.split_w(w, prob["T"], prob["nx"], prob["nu"])
    a, idx, det = sqp.line_search(prob, x, u, xp, up, alphas, eta)
    return x + a * (xp - x), u + a * (up - u), lp, dict(alpha=a, step=max(
        float(np.max(np.abs(xp - x))), float(np.max(np.abs(up - u))) if up.size else 0.0))


def converge(prob, x=None, u=None, lam=None, tol=1e-12, max_iter=100):
    """Newton SQP from (x, u, lam) (default: the problem's initial guess)
    until the QP step has ||dz||_inf <= tol.  Returns (x, u, lam, iterations)."""
    if x is None:
        x, u, lam = sqp.initial_guess(prob)
    x, u, lam = (np.array(a, np.float64) for a in (x, u, lam))
    x[0] = np.asarray(prob["x0"], np.float64)   # as the initial guess of Alg. sqp
    for k in range(1, max_iter + 1):
        x, u, lam, info = newton_step(prob, x, u, lam)
        # (a QP step at rounding level is converged whatever step size the
        # line search then picks among its rounding-level merit differences)
        if info["step"] <= tol:
            return x, u, lam, k
    raise RuntimeError(f"Newton SQP did not reach ||dz|| <= {tol} in {max_iter} iterations")


def kkt_exact(prob, x, u, lam):
    """K of the true KKT conditions at (x, u, lam): [[W, J'], [J, 0]]."""
    W = stage_blocks(prob, x, u, lam)
    K, _, parts, _ = _with_hessian(prob, x, u, W, project=False)
    return K, parts


def vjp_exact(prob, x, u, lam, gx, gu):
    """Gradient of l = <gx, x*> + <gu, u*> with respect to the cost
    parameters and x_s through the true KKT conditions at the KKT point
    (x, u, lam).  Returns (grads dict, (x~, u~, lam~))."""
    T, nx, nu = prob["T"], prob["nx"], prob["nu"]
    K, parts = kkt_exact(prob, x, u, lam)
    v = qp.join_w(np.asarray(gx, np.float64), np.asarray(gu, np.float64), np.zeros((T + 1, nx)))
    xi_ = sla.lu_solve(sla.lu_factor(K), v)
    xt, ut, lt = qp.split_w(xi_, T, nx, nu)
    g = {"x0": np.array(lt[0])}
    cp = costs.cost_params(prob)
    for key, val in cp.items():
        val = np.asarray(val, np.float64)
        gk = np.zeros(val.shape)
        for idx in np.ndindex(val.shape):
            cpc = {k: np.asarray(a, np.complex128).copy() for k, a in cp.items()}
            cpc[key][idx] += 1j * CS_H
            s = 0.0
            for t in range(T + 1):
                s += np.dot(xt[t], np.imag(costs.stage_x(prob, t, x[t].astype(np.complex128), cpc)[1]))
            for t in range(T):
                s += np.dot(ut[t], np.imag(costs.stage_u(prob, t, u[t].astype(np.complex128), cpc)[1]))
            gk[idx] = -s / CS_H
        g[key] = gk
    return g, (xt, ut, lt)
