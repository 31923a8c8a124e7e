"""QP data, dense KKT system and its LU solution (oracle side; test
infrastructure only).

Follows Sec. 3.1 of the paper:

* ``qp_data``   -- Eq. QPmatrices: Q_t, R_t are the (PD-projected) cost
                   Hessians at the linearisation point, q_t, r_t the linear
                   coefficients of the second-order cost model in absolute
                   coordinates (grad c - Q xbar; equal to the cost's own linear
                   term for quadratic costs), (A+_t, A_t, B_t) the Jacobians of
                   the implicit constraint f_t(x_{t+1}, x_t, u_t) =
                   x_{t+1} - phi_t(x_t, u_t) by complex step, and
                   C_t = A+_t x_{t+1} + A_t x_t + B_t u_t - f_t(...).
* ``kkt``       -- Eq. KKTmatrix and Eq. ocp:KKT: K = [[G, H'], [H, 0]],
                   rhs = [-b; d], b = (q_0, r_0, ..., q_T), d = (x_s, C_0, ...,
                   C_{T-1}), with z = (x_0, u_0, ..., x_{T-1}, u_{T-1}, x_T).
* ``solve_qp``  -- LU with partial pivoting of the dense K (LAPACK getrf/getrs).
* ``kkt_residual`` / ``kkt_residual_blocks`` -- ||K w - rhs||_2 / ||rhs||_2,
                   from the dense K or stage by stage from its blocks (long
                   horizons); pinned equal to each other.

Pinned (tests): Riccati closed form on LQ problems, a hand-solved scalar
problem, KKT residual at machine precision, complex-step Jacobians against
central differences and against hand-derived special cases of the models.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import costs, models

PD_EPS = 1e-6   # eigenvalue floor of the PD projection (the paper leaves it unstated)


def project_pd(Hm):
    """Project a symmetric Hessian onto {H >= PD_EPS I} (Sec. 3.1).  For a
    diagonal matrix this is an entrywise clamp (also for complex-step
    arguments, where the clamp acts on the real part)."""
    Hm = np.asarray(Hm)
    if np.count_nonzero(Hm - np.diag(np.diag(Hm))) == 0:
        d = np.diag(Hm).copy()
        low = d.real < PD_EPS
        d[low] = PD_EPS
        return np.diag(d)
    w, V = np.linalg.eigh(Hm)
    return (V * np.maximum(w, PD_EPS)) @ V.T


def complex_step_jacobian(fun, v, h=1e-30):
    """J[:, k] = Im f(v + i h e_k) / h (exact to rounding for analytic f)."""
    v = np.asarray(v, dtype=np.complex128)
    cols = []
    for k in range(v.shape[0]):
        vp = v.copy()
        vp[k] += 1j * h
        cols.append(np.imag(fun(vp)) / h)
    return np.stack(cols, axis=1)


def f_constraint(prob, t, x_next, x, u):
    """Implicit dynamics constraint f_t(x_{t+1}, x_t, u_t) = x_{t+1} - phi_t(x_t, u_t)."""
    return x_next - models.step(prob, t, x, u)


def qp_data(prob, xbar, ubar, cp=None):
    """QP matrices of Eq. QPmatrices at (xbar, ubar)."""
    T = prob["T"]
    Q, q, R, r = [], [], [], []
    for t in range(T + 1):
        _, g, Hm = costs.stage_x(prob, t, xbar[t], cp)
        Qt = project_pd(Hm)
        Q.append(Qt)
        q.append(g - Qt @ xbar[t])
    for t in range(T):
        _, g, Hm = costs.stage_u(prob, t, ubar[t], cp)
        Rt = project_pd(Hm)
        R.append(Rt)
        r.append(g - Rt @ ubar[t])
    Ap, Am, Bm, C = [], [], [], []
    for t in range(T):
        xn, xt, ut = xbar[t + 1], xbar[t], ubar[t]
        Jp = complex_step_jacobian(lambda v: f_constraint(prob, t, v, xt, ut), xn)
        Ja = complex_step_jacobian(lambda v: f_constraint(prob, t, xn, v, ut), xt)
        Jb = complex_step_jacobian(lambda v: f_constraint(prob, t, xn, xt, v), ut)
        ft = np.real(f_constraint(prob, t, xn, xt, ut))
        Ap.append(Jp)
        Am.append(Ja)
        Bm.append(Jb)
        C.append(Jp @ xn + Ja @ xt + Jb @ ut - ft)
    return dict(T=T, nx=prob["nx"], nu=prob["nu"], Q=Q, q=q, R=R, r=r,
                Aplus=Ap, A=Am, B=Bm, C=C)


def z_index(T, nx, nu):
    """Offsets of x_t and u_t inside z = (x_0, u_0, ..., x_{T-1}, u_{T-1}, x_T)."""
    xi = [t * (nx + nu) for t in range(T + 1)]
    ui = [t * (nx + nu) + nx for t in range(T)]
    return xi, ui, T * (nx + nu) + nx


def kkt(qpd, xs):
    """Dense K and rhs of Eq. ocp:KKT (G, H of Eq. KKTmatrix)."""
    T, nx, nu = qpd["T"], qpd["nx"], qpd["nu"]
    xi, ui, nz = z_index(T, nx, nu)
    nl = (T + 1) * nx
    dt = np.result_type(*[np.asarray(a) for a in qpd["Q"]], *[np.asarray(a) for a in qpd["A"]])
    G = np.zeros((nz, nz), dtype=dt)
    Hm = np.zeros((nl, nz), dtype=dt)
    b = np.zeros(nz, dtype=dt)
    d = np.zeros(nl, dtype=dt)
    for t in range(T + 1):
        G[xi[t]:xi[t] + nx, xi[t]:xi[t] + nx] = qpd["Q"][t]
        b[xi[t]:xi[t] + nx] = qpd["q"][t]
    for t in range(T):
        G[ui[t]:ui[t] + nu, ui[t]:ui[t] + nu] = qpd["R"][t]
        b[ui[t]:ui[t] + nu] = qpd["r"][t]
    Hm[0:nx, xi[0]:xi[0] + nx] = np.eye(nx)
    d[0:nx] = xs
    for t in range(T):
        row = (t + 1) * nx
        Hm[row:row + nx, xi[t]:xi[t] + nx] = qpd["A"][t]
        Hm[row:row + nx, ui[t]:ui[t] + nu] = qpd["B"][t]
        Hm[row:row + nx, xi[t + 1]:xi[t + 1] + nx] = qpd["Aplus"][t]
        d[row:row + nx] = qpd["C"][t]
    K = np.block([[G, Hm.T], [Hm, np.zeros((nl, nl), dtype=dt)]])
    rhs = np.concatenate([-b, d])
    return K, rhs, dict(G=G, H=Hm, b=b, d=d, xi=xi, ui=ui, nz=nz, nl=nl)


def split_w(w, T, nx, nu):
    """(x [N,nx], u [T,nu], lam [N,nx]) from w = (z, lam)."""
    xi, ui, nz = z_index(T, nx, nu)
    x = np.stack([w[i:i + nx] for i in xi])
    u = np.stack([w[i:i + nu] for i in ui]) if T > 0 else np.zeros((0, nu))
    lam = w[nz:].reshape(T + 1, nx)
    return x, u, lam


def join_w(x, u, lam):
    T, nx = u.shape[0], x.shape[1]
    parts = []
    for t in range(T):
        parts += [x[t], u[t]]
    parts.append(x[T])
    return np.concatenate(parts + [lam.reshape(-1)])


def solve_qp(qpd, xs):
    """QP solution (x, u, lam) of Eq. ocp:KKT by dense LU; also returns the
    LU factors and the KKT pieces for reuse by the backward pass."""
    K, rhs, parts = kkt(qpd, xs)
    lu = sla.lu_factor(K)
    w = sla.lu_solve(lu, rhs)
    x, u, lam = split_w(w, qpd["T"], qpd["nx"], qpd["nu"])
    return dict(x=x, u=u, lam=lam, w=w, K=K, rhs=rhs, lu=lu, parts=parts)


def kkt_residual(qpd, xs, x, u, lam):
    """Relative KKT residual ||K w - rhs||_2 / ||rhs||_2 of the QP."""
    K, rhs, _ = kkt(qpd, xs)
    w = join_w(np.asarray(x, np.float64), np.asarray(u, np.float64), np.asarray(lam, np.float64))
    return float(np.linalg.norm(K @ w - rhs) / max(np.linalg.norm(rhs), 1e-300))


def kkt_residual_blocks(qpd, xs, x, u, lam):
    """The same relative KKT residual as ``kkt_residual``, accumulated stage by
    stage from the blocks of G, H, b, d (Eq. KKTmatrix) instead of the dense
    K, so that long horizons do not need the dense matrix."""
    T = qpd["T"]
    x = np.asarray(x, np.float64)
    u = np.asarray(u, np.float64)
    lam = np.asarray(lam, np.float64)
    r2 = 0.0
    rhs2 = float(np.dot(xs, xs))
    for t in range(T + 1):
        # stationarity in x_t: Q_t x_t + (H' lam)_{x_t} + q_t
        g = qpd["Q"][t] @ x[t] + qpd["q"][t]
        g = g + (lam[0] if t == 0 else qpd["Aplus"][t - 1].T @ lam[t])
        if t < T:
            g = g + qpd["A"][t].T @ lam[t + 1]
        r2 += float(np.dot(g, g))
        rhs2 += float(np.dot(qpd["q"][t], qpd["q"][t]))
    for t in range(T):
        g = qpd["R"][t] @ u[t] + qpd["r"][t] + qpd["B"][t].T @ lam[t + 1]
        r2 += float(np.dot(g, g))
        rhs2 += float(np.dot(qpd["r"][t], qpd["r"][t]))
        # dynamics row t+1: A+_t x_{t+1} + A_t x_t + B_t u_t - C_t
        h = qpd["Aplus"][t] @ x[t + 1] + qpd["A"][t] @ x[t] + qpd["B"][t] @ u[t] - qpd["C"][t]
        r2 += float(np.dot(h, h))
        rhs2 += float(np.dot(qpd["C"][t], qpd["C"][t]))
    h = x[0] - xs
    r2 += float(np.dot(h, h))
    return float(np.sqrt(r2) / max(np.sqrt(rhs2), 1e-300))
