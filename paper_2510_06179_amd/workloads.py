"""Seeded synthetic workloads shaped like the paper's control tasks.

This module only draws inputs: it holds none of the solver's arithmetic and
imports neither the oracle nor the GPU binding, so both sides can consume the
same problems.  Every array is drawn in float64 and rounded to float32 (then
kept as float64), so the FP64 oracle sees exactly the values the FP32 GPU path
sees.

A problem is a plain dict:

    T, nx, nu          horizon and sizes (N = T + 1 stages of x, T of u)
    dyn                "ltv" | "cartpole" | "bicycle"
      ltv:      A [T,nx,nx], B [T,nx,nu], c [T,nx]   x_{t+1} = A_t x_t + B_t u_t + c_t
      cartpole: params [5] = (m_c, m_p, L, g, dt)
      bicycle:  params [BICYCLE_NPARAM] (see BICYCLE_PARAM_NAMES)
    cost               "diag" | "softplus"
      diag:     Qd [N,nx], q [N,nx], Rd [T,nu], r [T,nu]
                c_t^x(x) = 1/2 x'diag(Qd_t)x + q_t'x,  c_t^u(u) = 1/2 u'diag(Rd_t)u + r_t'u
      softplus: theta [P*(nw+nu)], wscale [nw+nu], wfix [nx-nw], xref [nx]
                phase k(t) = min(floor(P t / T), P-1); weights of the first nw states
                and of all inputs are wscale * softplus(theta[k]); the other
                states get wfix; c_t^x = 1/2 sum_i w_i (x_i - xref_i)^2, c_t^u = 1/2 sum w u^2
    x0 [nx]            initial state x_s
    xbar [N,nx], ubar [T,nu], lam [N,nx]   initial guess / warm start
    init               "given" (use xbar, ubar, lam) | "rollout" (roll ubar out from x0)

Config recipes follow the batch descriptions of the five benchmark workloads
(LQ parity batch, cart-pole SQP batch, bicycle differentiation batch, uneven
LTV batch, serving mix).
"""
from __future__ import annotations

import numpy as np

CARTPOLE_PARAM_NAMES = ("m_c", "m_p", "L", "g", "dt")
BICYCLE_PARAM_NAMES = (
    "a", "b", "m", "Iz", "rw", "Iw",
    "Bf", "Cf", "Df", "Br", "Cr", "Dr",
    "Cx", "kappa", "dt", "vmin",
)
BICYCLE_NPARAM = len(BICYCLE_PARAM_NAMES)


def f32(a):
    """Round to float32 and return float64 (exactly representable in FP32)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def _zeros_guess(T, nx, nu):
    N = T + 1
    return np.zeros((N, nx)), np.zeros((T, nu)), np.zeros((N, nx))


# ---------------------------------------------------------------------------
# LQ parity batch: 8 LTI problems, nx=4, nu=2, T=20
# ---------------------------------------------------------------------------
def lq_batch(seed=0, batch=8, nx=4, nu=2, T=20, rho=0.95):
    rng = np.random.default_rng(seed)
    probs = []
    N = T + 1
    for _ in range(batch):
        G = rng.standard_normal((nx, nx))
        sr = np.max(np.abs(np.linalg.eigvals(G)))
        A = G * (rho / sr)
        B = rng.standard_normal((nx, nu))
        Qd = rng.uniform(0.1, 1.0, size=nx)
        Rd = rng.uniform(0.01, 0.1, size=nu)
        p = dict(
            T=T, nx=nx, nu=nu, dyn="ltv", cost="diag",
            A=f32(np.broadcast_to(A, (T, nx, nx)).copy()),
            B=f32(np.broadcast_to(B, (T, nx, nu)).copy()),
            c=np.zeros((T, nx)),
            Qd=f32(np.broadcast_to(Qd, (N, nx)).copy()),
            q=f32(rng.normal(0.0, 0.1, size=(N, nx))),
            Rd=f32(np.broadcast_to(Rd, (T, nu)).copy()),
            r=f32(rng.normal(0.0, 0.1, size=(T, nu))),
            x0=f32(rng.standard_normal(nx)),
            init="given",
        )
        p["xbar"], p["ubar"], p["lam"] = _zeros_guess(T, nx, nu)
        p["xbar"][0] = p["x0"]
        probs.append(p)
    return probs


# ---------------------------------------------------------------------------
# Cart-pole SQP batch: nx=4, nu=1, T=50, dt=0.05
# ---------------------------------------------------------------------------
def cartpole_batch(seed=0, batch=1024, T=50, dt=0.05):
    rng = np.random.default_rng(seed)
    nx, nu, N = 4, 1, T + 1
    probs = []
    Qd = np.array([1.0, 1.0, 10.0, 1.0])
    for _ in range(batch):
        mp = rng.uniform(0.05, 0.2)
        L = rng.uniform(0.3, 0.7)
        ang = rng.uniform(-0.5, 0.5)
        p = dict(
            T=T, nx=nx, nu=nu, dyn="cartpole", cost="diag",
            params=f32([1.0, mp, L, 9.81, dt]),
            Qd=f32(np.broadcast_to(Qd, (N, nx)).copy()),
            q=np.zeros((N, nx)),
            Rd=f32(np.full((T, nu), 0.1)),
            r=np.zeros((T, nu)),
            x0=f32([0.0, 0.0, ang, 0.0]),
            init="rollout",
        )
        p["xbar"], p["ubar"], p["lam"] = _zeros_guess(T, nx, nu)
        p["xbar"][0] = p["x0"]
        probs.append(p)
    return probs


# ---------------------------------------------------------------------------
# Uneven LTV batch: T in {16,32,64,128}, nx in {4,8,12,16}, nu in {2,4}
# ---------------------------------------------------------------------------
def ltv_uneven_batch(seed=0, batch=4096, Ts=(16, 32, 64, 128), nxs=(4, 8, 12, 16),
                     nus=(2, 4), init="rollout"):
    """The uneven batch.  Its initial guess is the zero-input rollout from x0
    (as for the cart-pole batch): a feasible start, from which the first
    full QP step passes the decrease test and later iterations stay at the
    solution.  (From the infeasible guess x = 0, u = 0 with x_0 = x0 the
    penalty of the merit function is zero whenever the cost's directional
    derivative is negative, and most problems then take the smallest step
    size at every iteration.)"""
    rng = np.random.default_rng(seed)
    probs = []
    for _ in range(batch):
        T = int(rng.choice(Ts))
        nx = int(rng.choice(nxs))
        nu = int(rng.choice(nus))
        p = ltv_problem(rng, T, nx, nu)
        p["init"] = init
        probs.append(p)
    return probs


def ltv_problem(rng, T, nx, nu):
    """One time-varying linear problem of the uneven batch's distribution."""
    N = T + 1
    A = np.eye(nx)[None] + rng.normal(0.0, 0.05, size=(T, nx, nx))
    B = rng.normal(0.0, 0.3, size=(T, nx, nu))
    Qd = np.exp(rng.uniform(np.log(1e-2), np.log(1e1), size=(N, nx)))
    Rd = np.exp(rng.uniform(np.log(1e-2), np.log(1e1), size=(T, nu)))
    p = dict(
        T=T, nx=nx, nu=nu, dyn="ltv", cost="diag",
        A=f32(A), B=f32(B), c=np.zeros((T, nx)),
        Qd=f32(Qd), q=f32(rng.normal(0.0, 0.1, size=(N, nx))),
        Rd=f32(Rd), r=f32(rng.normal(0.0, 0.1, size=(T, nu))),
        x0=f32(rng.standard_normal(nx)),
        init="given",
    )
    p["xbar"], p["ubar"], p["lam"] = _zeros_guess(T, nx, nu)
    p["xbar"][0] = p["x0"]
    return p


# ---------------------------------------------------------------------------
# Bicycle differentiation batch: nx=8, nu=2, T=64, dt=0.02, theta in R^32
# ---------------------------------------------------------------------------
# State (r, v, beta, omega_r, dpsi, e, delta, tau), input (ddelta, dtau).
# Units are scaled to keep FP32 conditioning sane: forces in kN, mass in t,
# inertias in t*m^2, torque in kN*m.
BICYCLE_NOMINAL = dict(
    a=1.239, b=1.209, m=1.476, Iz=2.0, rw=0.323, Iw=0.25,
    Bf=8.0, Cf=1.3, Df=0.99 * 1.476 * 9.81 * 1.209 / 2.448,
    Br=8.0, Cr=1.3, Dr=0.90 * 1.476 * 9.81 * 1.239 / 2.448,
    Cx=40.0, kappa=0.0625, dt=0.02, vmin=1.0,
)
# steady drift of the nominal model on the constant-curvature (radius 16 m)
# reference at sideslip -0.3 rad (heading error = -sideslip, lateral error 0),
# found offline by a root solve of the model's equilibrium conditions
BICYCLE_XREF = np.array([0.7583, 12.13287, -0.3, 39.47268, 0.3, 0.0, -0.07232, 1.15019])


def bicycle_batch(seed=0, batch=512, T=64, phases=4, perturb=0.2, variant="nominal"):
    """variant "nominal": every learned weight has scale 1 and the two
    actuator states (steering angle, torque) weight 1e-2.  variant
    "conditioned": per-state scales that make the weights O(1) in the scaled
    units and unit actuator weights; its preconditioned Schur complement is
    about ten times better conditioned (~3e4 instead of ~4e5)."""
    if variant not in ("nominal", "conditioned"):
        raise ValueError(variant)
    rng = np.random.default_rng(seed)
    nx, nu, N = 8, 2, T + 1
    nw = 6
    probs = []
    base = np.array([BICYCLE_NOMINAL[k] for k in BICYCLE_PARAM_NAMES])
    tire_idx = [BICYCLE_PARAM_NAMES.index(k) for k in ("Bf", "Cf", "Df", "Br", "Cr", "Dr")]
    theta = f32(rng.normal(0.0, 0.1, size=phases * (nw + nu)))
    if variant == "nominal":
        wscale = f32(np.ones(nw + nu))
        wfix = f32([1e-2, 1e-2])
    else:
        wscale = f32([1.0, 0.5, 4.0, 0.01, 2.0, 0.5, 2.0, 2.0])
        wfix = f32([1.0, 1.0])
    ranges = np.array([0.1, 0.5, 0.05, 1.0, 0.05, 0.2, 0.02, 0.05])
    for _ in range(batch):
        par = base.copy()
        par[tire_idx] *= rng.uniform(1.0 - perturb, 1.0 + perturb, size=len(tire_idx))
        x0 = BICYCLE_XREF + rng.uniform(-1.0, 1.0, size=nx) * ranges
        p = dict(
            T=T, nx=nx, nu=nu, dyn="bicycle", cost="softplus",
            params=f32(par), theta=theta.copy(), phases=phases, nw=nw,
            wscale=wscale.copy(), wfix=wfix.copy(), xref=f32(BICYCLE_XREF),
            x0=f32(x0), init="rollout",
        )
        p["xbar"], p["ubar"], p["lam"] = _zeros_guess(T, nx, nu)
        p["xbar"][0] = p["x0"]
        probs.append(p)
    return probs


# ---------------------------------------------------------------------------
# Loss cotangents and serving arrivals
# ---------------------------------------------------------------------------
def loss_cotangents(probs, seed=0, with_lambda=False):
    """Seeded dl/dz for l = <g, z> (g ~ N(0,1)); dl/dlambda = 0 unless asked."""
    rng = np.random.default_rng(seed + 7919)
    out = []
    for p in probs:
        N, T, nx, nu = p["T"] + 1, p["T"], p["nx"], p["nu"]
        gx = f32(rng.standard_normal((N, nx)))
        gu = f32(rng.standard_normal((T, nu)))
        gl = f32(rng.standard_normal((N, nx))) if with_lambda else np.zeros((N, nx))
        out.append(dict(gx=gx, gu=gu, glam=gl))
    return out


def poisson_arrivals(seed, rate_hz, duration_s):
    """Arrival times (s) of a seeded Poisson process."""
    rng = np.random.default_rng(seed)
    n_est = int(rate_hz * duration_s * 1.2) + 16
    gaps = rng.exponential(1.0 / rate_hz, size=n_est)
    t = np.cumsum(gaps)
    return t[t < duration_s]
