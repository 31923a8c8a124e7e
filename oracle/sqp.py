"""Forward pass: SQP with the merit line search (oracle side; test
infrastructure only).

* ``initial_guess`` -- the starting iterate: as given, or a rollout of the
  given controls from x_s; in both cases x_0 = x_s.
* ``merit``/``line_search`` -- App. A.3, Alg. linesearch: merit of Eq.
  linesearch:merit (costs of every stage plus mu times the l1 norm of every
  dynamics defect; the x_0 = x_s row is not part of it), penalty of Eq.
  linesearch:penalty, descent of Eq. linesearch:descent, decrease test of
  Eq. linesearch:decrease with eta = 0.4.  Readings where the paper is silent:
  mu is clamped below at 0 and its denominator at 1e-30; the first candidate
  (candidates in decreasing order) with a strictly negative decrease value is
  taken, else the smallest candidate.
* ``sqp`` -- Alg. sqp with a fixed number of iterations: QP data (Eq.
  QPmatrices) -> QP solution (Eq. ocp:KKT, dense LU) -> line search on (x, u);
  the multipliers are taken from the QP.

Pinned (tests): on LQ problems one step with alpha = 1 equals the Riccati
solution and the next QP step is zero; hand-built merit cases exercise every
branch of the selection.
"""
from __future__ import annotations

import numpy as np

from . import costs, models, qp

ALPHAS = (1.0, 0.7, 0.3, 0.1, 0.01)
ETA = 0.4


def initial_guess(prob):
    T = prob["T"]
    x = np.array(prob["xbar"], dtype=np.float64).copy()
    u = np.array(prob["ubar"], dtype=np.float64).copy()
    lam = np.array(prob["lam"], dtype=np.float64).copy()
    x[0] = prob["x0"]
    if prob.get("init", "given") == "rollout":
        for t in range(T):
            x[t + 1] = np.real(models.step(prob, t, x[t], u[t]))
        lam[:] = 0.0
    return x, u, lam


def total_cost(prob, x, u):
    T = prob["T"]
    s = sum(costs.stage_x(prob, t, x[t])[0] for t in range(T + 1))
    return s + sum(costs.stage_u(prob, t, u[t])[0] for t in range(T))


def defect_l1(prob, x, u):
    T = prob["T"]
    return sum(np.sum(np.abs(qp.f_constraint(prob, t, x[t + 1], x[t], u[t])))
               for t in range(T))


def merit(prob, x, u, mu):
    """Eq. linesearch:merit."""
    return total_cost(prob, x, u) + mu * defect_l1(prob, x, u)


def directional(prob, x, u, xp, up):
    """sum_t grad c_t^x(x_t)'(x+_t - x_t) + grad c_t^u(u_t)'(u+_t - u_t)."""
    T = prob["T"]
    s = sum(costs.stage_x(prob, t, x[t])[1] @ (xp[t] - x[t]) for t in range(T + 1))
    return s + sum(costs.stage_u(prob, t, u[t])[1] @ (up[t] - u[t]) for t in range(T))


def line_search(prob, x, u, xp, up, alphas=ALPHAS, eta=ETA):
    """Alg. linesearch.  Returns (alpha, index of alpha, details)."""
    num = directional(prob, x, u, xp, up)
    fl1 = defect_l1(prob, x, u)
    mu = max(num, 0.0) / max(0.5 * fl1, 1e-30)          # Eq. linesearch:penalty
    D = num - mu * fl1                                  # Eq. linesearch:descent
    phi0 = merit(prob, x, u, mu)
    dphi = []
    for a in alphas:                                    # evaluated "in parallel"
        xa, ua = x + a * (xp - x), u + a * (up - u)
        dphi.append(merit(prob, xa, ua, mu) - phi0 - eta * a * D)   # Eq. decrease
    idx = int(np.argmin(alphas))
    for k, a in enumerate(alphas):                      # sequential selection
        if dphi[k] < 0.0:
            idx = k
            break
    return alphas[idx], idx, dict(mu=mu, D=D, phi0=phi0, dphi=np.array(dphi), num=num, fl1=fl1)


def sqp_step(prob, x, u, alphas=ALPHAS, eta=ETA):
    """One iteration of Alg. sqp from (x, u).  Returns the new iterate, the QP
    data and the QP solution."""
    qpd = qp.qp_data(prob, x, u)
    sol = qp.solve_qp(qpd, prob["x0"])
    a, idx, det = line_search(prob, x, u, sol["x"], sol["u"], alphas, eta)
    xn = x + a * (sol["x"] - x)
    un = u + a * (sol["u"] - u)
    return xn, un, sol["lam"], dict(qp=qpd, sol=sol, alpha=a, alpha_idx=idx, ls=det,
                                      xbar=x, ubar=u)


def sqp(prob, iters, alphas=ALPHAS, eta=ETA, x=None, u=None):
    """Alg. sqp with a fixed iteration count.  Returns (x, u, lam, history);
    history[-1]['qp'] / ['sol'] are the final QP and its solution."""
    if x is None:
        x, u, lam = initial_guess(prob)
    else:
        lam = np.zeros_like(x)
    hist = []
    for _ in range(iters):
        x, u, lam, h = sqp_step(prob, x, u, alphas, eta)
        hist.append(h)
    return x, u, lam, hist
