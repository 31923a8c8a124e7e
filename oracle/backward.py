"""Backward pass: implicit-function-theorem VJP through the dense KKT matrix
(oracle side; test infrastructure only).

* ``adjoint``        -- Eq. ocp:backward / Eq. loss_gradient: solve
                        K [z~; lam~] = [dl/dz; dl/dlam] with the LU factors of
                        the final QP's K (the paper's Alg. backward uses
                        dl/dlam = 0; a non-zero one is the general VJP).
* ``qp_cotangents``  -- -dF/dtheta' [z~; lam~] with F = [G z + b + H' lam;
                        H z - d] (Eq. KKT) taken with respect to the dense
                        matrices: dG = -z~ z', db = -z~, dH = -(lam z~' + lam~ z'),
                        dd = lam~; then read off at the positions where the QP
                        data sit in G, b, H, d (Eq. KKTmatrix).
* ``jvp``            -- forward-mode sensitivity of the same solution map:
                        differentiating K(theta) w(theta) = rhs(theta) along a
                        tangent v gives K dw = d rhs - dK w, solved with the
                        same LU factors.  K and rhs are affine in the inputs
                        the tangent may move (linear dynamics A, B, c; diagonal
                        costs Qd, q, Rd, r away from the PD clamp; x_s), so
                        (dK, d rhs) are the symmetric differences of the
                        dense KKT builders at theta +- s v divided by 2 s.
* ``vjp``            -- cotangents of the problem's own inputs: x_s, the cost
                        parameters (through the QP cost data, by complex step
                        for the softplus weights; for diagonal costs an entry
                        clamped by the PD projection reaches the linear term
                        only, q = Qd xbar + q_raw - Q_proj xbar), and for
                        linear dynamics A, B, c
                        (the constraint's Jacobians are A+ = I, -A, -B and
                        C_t = c_t by definition of f_t).  The linearisation
                        point is held fixed: the backward is the VJP of the
                        final QP's solution map.

Pinned (tests): central finite differences of the oracle's QP solution map
(also with cost entries below the PD floor, where the clamp moves the linear
terms: a hand-worked instance gives d lam_0 / d Qd_0 = -xbar_0 exactly), the
envelope identity (dl/dz = G z + b gives z~ = 0, lam~ = -lam), dJ*/dx_s =
-lam_0 on LQ problems, and the duality of the two modes: <g, JVP(v)> =
<VJP(g), v> for random g and v, with and without clamped entries.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import costs, qp


def adjoint(sol, gx, gu, glam=None):
    """(x~ [N,nx], u~ [T,nu], lam~ [N,nx]) solving K xi = (dl/dz, dl/dlam)."""
    T, nx = gu.shape[0], gx.shape[1]
    nu = gu.shape[1]
    if glam is None:
        glam = np.zeros_like(gx)
    v = qp.join_w(np.asarray(gx, np.float64), np.asarray(gu, np.float64),
                  np.asarray(glam, np.float64))
    xi = sla.lu_solve(sol["lu"], v)
    return qp.split_w(xi, T, nx, nu)


def qp_cotangents(qpd, sol, xt, ut, lamt):
    """Cotangents of the QP data (lists per stage, paper's sign convention)."""
    T, nx, nu = qpd["T"], qpd["nx"], qpd["nu"]
    parts = sol["parts"]
    xi, ui = parts["xi"], parts["ui"]
    z = sol["w"][:parts["nz"]]
    lam = sol["w"][parts["nz"]:]
    w_t = qp.join_w(xt, ut, lamt)
    zt, lt = w_t[:parts["nz"]], w_t[parts["nz"]:]
    dG = -np.outer(zt, z)
    db = -zt
    dH = -(np.outer(lam, zt) + np.outer(lt, z))
    dd = lt
    out = dict(Q=[], q=[], R=[], r=[], A=[], B=[], C=[])
    for t in range(T + 1):
        out["Q"].append(dG[xi[t]:xi[t] + nx, xi[t]:xi[t] + nx])
        out["q"].append(db[xi[t]:xi[t] + nx])
    for t in range(T):
        out["R"].append(dG[ui[t]:ui[t] + nu, ui[t]:ui[t] + nu])
        out["r"].append(db[ui[t]:ui[t] + nu])
        row = (t + 1) * nx
        out["A"].append(dH[row:row + nx, xi[t]:xi[t] + nx])
        out["B"].append(dH[row:row + nx, ui[t]:ui[t] + nu])
        out["C"].append(dd[row:row + nx])
    out["xs"] = dd[0:nx]
    return out


def _cost_qp_part(prob, xbar, ubar, cp):
    """(Q_t, q_t, R_t, r_t) of Eq. QPmatrices as a function of the cost
    parameters cp at a fixed linearisation point."""
    T = prob["T"]
    Q, q, R, r = [], [], [], []
    for t in range(T + 1):
        _, g, Hm = costs.stage_x(prob, t, xbar[t].astype(np.complex128), cp)
        Qt = qp.project_pd(Hm)
        Q.append(Qt)
        q.append(g - Qt @ xbar[t])
    for t in range(T):
        _, g, Hm = costs.stage_u(prob, t, ubar[t].astype(np.complex128), cp)
        Rt = qp.project_pd(Hm)
        R.append(Rt)
        r.append(g - Rt @ ubar[t])
    return Q, q, R, r


def _pair(cot, part):
    """<cotangent, perturbation> summed over all stages."""
    s = 0.0
    for key, val in zip(("Q", "q", "R", "r"), part):
        for a, b in zip(cot[key], val):
            s += np.sum(np.asarray(a) * np.asarray(b))
    return s


def vjp(prob, xbar, ubar, qpd, sol, gx, gu, glam=None, h=1e-30):
    """Gradient of l with respect to the problem inputs through the final QP's
    solution map.  Returns (grads dict, (x~, u~, lam~))."""
    xt, ut, lamt = adjoint(sol, gx, gu, glam)
    cot = qp_cotangents(qpd, sol, xt, ut, lamt)
    g = {"x0": np.array(cot["xs"])}
    cp = costs.cost_params(prob)
    if prob["cost"] == "diag":
        # the cost parameters are the QP cost data, through the projection of
        # Sec. 3.1: an entry at or above the floor is the Hessian entry itself;
        # a clamped entry leaves the Hessian at the floor and moves the linear
        # term q = Qd xbar + q_raw - Q_proj xbar by xbar (r likewise by ubar)
        Qd, Rd = np.asarray(cp["Qd"]), np.asarray(cp["Rd"])
        cq, cr = np.array(cot["q"]), np.array(cot["r"])
        g["Qd"] = np.where(Qd >= qp.PD_EPS, np.array([np.diag(a) for a in cot["Q"]]),
                           cq * np.asarray(xbar, np.float64))
        g["Rd"] = np.where(Rd >= qp.PD_EPS, np.array([np.diag(a) for a in cot["R"]]),
                           cr * np.asarray(ubar, np.float64))
        g["q"] = cq
        g["r"] = cr
    else:
        for key, val in cp.items():
            val = np.asarray(val, dtype=np.float64)
            gk = np.zeros(val.shape)
            for idx in np.ndindex(val.shape):
                cpc = {k: np.asarray(v, dtype=np.complex128).copy() for k, v in cp.items()}
                cpc[key][idx] += 1j * h
                part = _cost_qp_part(prob, xbar, ubar, cpc)
                gk[idx] = np.imag(_pair(cot, part)) / h
            g[key] = gk
    if prob["dyn"] == "ltv":
        g["A"] = -np.array(cot["A"])
        g["B"] = -np.array(cot["B"])
        g["c"] = np.array(cot["C"])
    return g, (xt, ut, lamt)


JVP_KEYS_DIAG = ("Qd", "q", "Rd", "r")
JVP_KEYS_LTV = ("A", "B", "c")


def _moved(prob, tangent, s):
    """The problem with its inputs moved by s * tangent (keys as the VJP's
    gradient: A, B, c for linear dynamics, Qd, q, Rd, r for diagonal costs,
    x0)."""
    out = dict(prob)
    keys = ("x0",) + (JVP_KEYS_DIAG if prob["cost"] == "diag" else ()) + \
        (JVP_KEYS_LTV if prob["dyn"] == "ltv" else ())
    for k in keys:
        if k in tangent:
            out[k] = np.asarray(prob[k], np.float64) + s * np.asarray(tangent[k], np.float64)
    return out


def _clamp_safe_step(prob, tangent, s):
    """The largest step <= s along which no diagonal cost entry crosses the
    PD floor (K and rhs are affine in the inputs on each side of it)."""
    for k in ("Qd", "Rd"):
        if k in tangent and prob["cost"] == "diag":
            h = np.asarray(prob[k], np.float64)
            v = np.abs(np.asarray(tangent[k], np.float64))
            gap = np.abs(h - qp.PD_EPS)
            moving = v > 0
            if np.any(moving):
                s = min(s, 0.5 * float(np.min(gap[moving] / v[moving])))
    return s


def jvp(prob, xbar, ubar, qpd, sol, tangent, s=1e-3):
    """(dx [N,nx], du [T,nu], dlam [N,nx]): derivative of the final QP's
    solution (x, u, lam) along `tangent`, linearisation point fixed.  Only
    diagonal costs; a tangent of nonlinear model parameters is not read."""
    if prob["cost"] != "diag":
        raise ValueError("jvp: diagonal costs only")
    T, nx, nu = qpd["T"], qpd["nx"], qpd["nu"]
    s = _clamp_safe_step(prob, tangent, s)
    Kp, rp, _ = qp.kkt(qp.qp_data(_moved(prob, tangent, s), xbar, ubar), _moved(prob, tangent, s)["x0"])
    Km, rm, _ = qp.kkt(qp.qp_data(_moved(prob, tangent, -s), xbar, ubar), _moved(prob, tangent, -s)["x0"])
    dK = (Kp - Km) / (2 * s)
    drhs = (rp - rm) / (2 * s)
    dw = sla.lu_solve(sol["lu"], drhs - dK @ sol["w"])
    return qp.split_w(dw, T, nx, nu)
