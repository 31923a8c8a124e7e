"""Pins of the FP64 oracle against facts that do not come from the oracle
itself: the textbook Riccati recursion, hand-solved fixtures, closed-form
special cases of the models, identities of the KKT system and central finite
differences.  CPU only."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import backward, costs, models, qp, sqp
from paper_2510_06179_amd import workloads as W


# ---------------------------------------------------------------------------
# Textbook finite-horizon LQR with affine dynamics (independent of the oracle)
# ---------------------------------------------------------------------------
def riccati_lq(p):
    """Backward Riccati recursion V_t(x) = 1/2 x'P_t x + p_t'x and forward
    rollout; multipliers from the costate lam_t = -(P_t x_t + p_t)."""
    T, nx, nu = p["T"], p["nx"], p["nu"]
    Pm = np.diag(p["Qd"][T])
    pv = p["q"][T].copy()
    Ks, ks, Ps, ps = [None] * T, [None] * T, [None] * (T + 1), [None] * (T + 1)
    Ps[T], ps[T] = Pm, pv
    for t in range(T - 1, -1, -1):
        A, B, c = p["A"][t], p["B"][t], p["c"][t]
        Q, R = np.diag(p["Qd"][t]), np.diag(p["Rd"][t])
        M = R + B.T @ Pm @ B
        K = -np.linalg.solve(M, B.T @ Pm @ A)
        k = -np.linalg.solve(M, p["r"][t] + B.T @ (Pm @ c + pv))
        pv = p["q"][t] + A.T @ (Pm @ c + pv) + A.T @ Pm @ B @ k
        Pm = Q + A.T @ Pm @ A + A.T @ Pm @ B @ K
        Ks[t], ks[t], Ps[t], ps[t] = K, k, Pm, pv
    x = np.zeros((T + 1, nx))
    u = np.zeros((T, nu))
    x[0] = p["x0"]
    for t in range(T):
        u[t] = Ks[t] @ x[t] + ks[t]
        x[t + 1] = p["A"][t] @ x[t] + p["B"][t] @ u[t] + p["c"][t]
    lam = np.array([-(Ps[t] @ x[t] + ps[t]) for t in range(T + 1)])
    return x, u, lam


def _ltv_random(seed, T=7, nx=3, nu=2):
    rng = np.random.default_rng(seed)
    p = W.ltv_problem(rng, T, nx, nu)
    p["c"] = W.f32(rng.normal(0, 0.3, size=(T, nx)))
    return p


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_qp_matches_riccati_lq_batch(seed):
    for p in W.lq_batch(seed, batch=3):
        x, u, lam, hist = sqp.sqp(p, 1, alphas=(1.0,))
        xr, ur, lr = riccati_lq(p)
        assert np.allclose(x, xr, atol=1e-10, rtol=1e-9)
        assert np.allclose(u, ur, atol=1e-10, rtol=1e-9)
        assert np.allclose(lam, lr, atol=1e-10, rtol=1e-9)


@pytest.mark.parametrize("seed", [3, 4])
def test_qp_matches_riccati_ltv_affine(seed):
    p = _ltv_random(seed)
    qpd = qp.qp_data(p, np.zeros((p["T"] + 1, p["nx"])), np.zeros((p["T"], p["nu"])))
    sol = qp.solve_qp(qpd, p["x0"])
    xr, ur, lr = riccati_lq(p)
    assert np.allclose(sol["x"], xr, atol=1e-10)
    assert np.allclose(sol["u"], ur, atol=1e-10)
    assert np.allclose(sol["lam"], lr, atol=1e-10)


def test_scalar_hand_solution(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "scalar_lq.json")))
    d = g["data"]
    p = dict(T=1, nx=1, nu=1, dyn="ltv", cost="diag",
             A=np.array([[[d["a"]]]], float), B=np.array([[[d["b"]]]], float),
             c=np.array([[d["c"]]], float),
             Qd=np.array([[d["Q0"]], [d["Q1"]]], float), q=np.array([[d["q0"]], [d["q1"]]], float),
             Rd=np.array([[d["R"]]], float), r=np.array([[d["r"]]], float),
             x0=np.array([d["xs"]], float))
    qpd = qp.qp_data(p, np.zeros((2, 1)), np.zeros((1, 1)))
    sol = qp.solve_qp(qpd, p["x0"])
    e = {k: float(Fraction(v)) for k, v in g["expected"].items()}
    assert sol["x"][0, 0] == pytest.approx(e["x0"], abs=1e-14)
    assert sol["u"][0, 0] == pytest.approx(e["u0"], abs=1e-14)
    assert sol["x"][1, 0] == pytest.approx(e["x1"], abs=1e-14)
    assert sol["lam"][0, 0] == pytest.approx(e["lam0"], abs=1e-14)
    assert sol["lam"][1, 0] == pytest.approx(e["lam1"], abs=1e-14)


def test_kkt_residual_machine_precision():
    for p in W.lq_batch(5, batch=2) + [_ltv_random(6)]:
        x, u, lam, hist = sqp.sqp(p, 1, alphas=(1.0,))
        res = qp.kkt_residual(hist[-1]["qp"], p["x0"], x, u, lam)
        assert res < 1e-13


def test_dynamics_feasibility_and_initial_state():
    p = _ltv_random(7)
    qpd = qp.qp_data(p, np.zeros((p["T"] + 1, p["nx"])), np.zeros((p["T"], p["nu"])))
    sol = qp.solve_qp(qpd, p["x0"])
    assert np.allclose(sol["x"][0], p["x0"], atol=1e-13)
    for t in range(p["T"]):
        nxt = p["A"][t] @ sol["x"][t] + p["B"][t] @ sol["u"][t] + p["c"][t]
        assert np.allclose(sol["x"][t + 1], nxt, atol=1e-12)


# ---------------------------------------------------------------------------
# Models: complex step vs central differences, printed special cases
# ---------------------------------------------------------------------------
def _central_fd(fun, v, h=1e-6):
    cols = []
    for k in range(v.shape[0]):
        e = np.zeros_like(v)
        e[k] = h
        cols.append((fun(v + e) - fun(v - e)) / (2 * h))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("kind", ["cartpole", "bicycle"])
def test_complex_step_matches_central_fd(kind):
    rng = np.random.default_rng(11)
    if kind == "cartpole":
        p = W.cartpole_batch(1, batch=1)[0]
        x = rng.normal(0, 0.7, 4)
        u = rng.normal(0, 1.0, 1)
    else:
        p = W.bicycle_batch(1, batch=1)[0]
        x = p["x0"] + rng.normal(0, 0.05, 8)
        u = rng.normal(0, 0.5, 2)
    fx = lambda v: np.real(models.step(p, 0, v, u))
    fu = lambda v: np.real(models.step(p, 0, x, v))
    Jx = qp.complex_step_jacobian(lambda v: models.step(p, 0, v, u), x)
    Ju = qp.complex_step_jacobian(lambda v: models.step(p, 0, x, v), u)
    assert np.allclose(Jx, _central_fd(fx, x), atol=2e-7, rtol=1e-6)
    assert np.allclose(Ju, _central_fd(fu, u), atol=2e-7, rtol=1e-6)


def test_cartpole_printed_special_cases():
    # parameters of the imitation-learning task: m_c=1, m_p=0.1, L=0.5, g=9.81
    mc, mp, L, g = 1.0, 0.1, 0.5, 9.81
    M = mc + mp
    par = np.array([mc, mp, L, g, 0.05])
    # upright rest is an equilibrium
    assert np.allclose(models.cartpole_xdot(par, np.zeros(4), np.zeros(1)), 0.0)
    # linearisation at the upright: d(x4dot)/du = 1/M, d(x4dot)/dx3 = m_p g / M,
    # d(x2dot)/dx3 = m_p g / (M L), d(x2dot)/du = 0, d(x1dot)/dx2 = d(x3dot)/dx4 = 1
    J = qp.complex_step_jacobian(lambda v: models.cartpole_xdot(par, v, np.zeros(1)), np.zeros(4))
    Ju = qp.complex_step_jacobian(lambda v: models.cartpole_xdot(par, np.zeros(4), v), np.zeros(1))
    assert J[3, 2] == pytest.approx(mp * g / M, rel=1e-14)
    assert J[1, 2] == pytest.approx(mp * g / (M * L), rel=1e-14)
    assert J[0, 1] == 1.0 and J[2, 3] == 1.0
    assert Ju[3, 0] == pytest.approx(1.0 / M, rel=1e-14)
    assert Ju[1, 0] == 0.0
    # horizontal pole (x3 = pi/2): cos = 0, sin = 1, denominator M + m_p
    x4, u = 0.7, 0.3
    xd = models.cartpole_xdot(par, np.array([0.0, 0.0, np.pi / 2, x4]), np.array([u]))
    assert xd[3] == pytest.approx((-mp * L * x4 + u) / (M + mp), rel=1e-12)
    assert xd[1] == pytest.approx(-mp * L * x4 * x4 / ((M + mp) * L), rel=1e-12)
    # Euler step
    x = np.array([0.1, -0.2, 0.3, 0.4])
    assert np.allclose(models.cartpole_step(par, x, np.array([0.5])),
                       x + 0.05 * models.cartpole_xdot(par, x, np.array([0.5])))


def test_bicycle_invariants():
    p = W.bicycle_batch(2, batch=1)[0]
    par = p["params"].copy()
    par[13] = 0.0                     # straight reference
    rw = par[4]
    v = 8.0
    x = np.array([0.0, v, 0.0, v / rw, 0.0, 0.0, 0.0, 0.0])
    xd = models.bicycle_xdot(par, x, np.zeros(2))
    assert np.allclose(xd[:6], 0.0, atol=1e-12)        # straight rolling is an equilibrium
    # mirror symmetry: flip (r, beta, dpsi, e, delta) and the steering rate
    rng = np.random.default_rng(3)
    x = np.array([0.3, 9.0, -0.2, 30.0, 0.05, 0.4, -0.1, 0.3]) + rng.normal(0, 0.01, 8)
    u = np.array([0.2, -0.1])
    S = np.diag([-1, 1, -1, 1, -1, -1, -1, 1.0])
    Su = np.diag([-1, 1.0])
    a = models.bicycle_xdot(par, S @ x, Su @ u)
    b = S @ models.bicycle_xdot(par, x, u)
    assert np.allclose(a, b, atol=1e-12)


# ---------------------------------------------------------------------------
# Line search and SQP
# ---------------------------------------------------------------------------
def test_line_search_hand_cases(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "linesearch_cases.json")))
    p = dict(T=1, nx=1, nu=1, dyn="ltv", cost="diag",
             A=np.zeros((1, 1, 1)), B=np.ones((1, 1, 1)), c=np.zeros((1, 1)),
             Qd=np.ones((2, 1)), q=np.zeros((2, 1)), Rd=np.ones((1, 1)), r=np.zeros((1, 1)),
             x0=np.zeros(1))
    x = np.array([[0.0], [1.0]])
    u = np.array([[1.0]])
    for case in g["cases"]:
        s = case["s"]
        xp = x - s * np.array([[0.0], [1.0]])
        up = u - s
        a, idx, det = sqp.line_search(p, x, u, xp, up)
        assert det["fl1"] == 0.0 and det["D"] == pytest.approx(-2.0 * s)
        if s > 0:
            assert det["mu"] == 0.0
        assert a == case["alpha"] and idx == case["index"]


def test_sqp_lq_converges_in_one_step():
    # From a dynamically feasible start (a rollout) the defect sum is 0, so
    # mu = 0 and D = grad'dz = -dz'G dz; then Delta_1 = -0.1 dz'G dz < 0 and the
    # full QP step is taken, which is the Riccati solution.
    p = _ltv_random(8)
    p["init"] = "rollout"
    p["ubar"] = np.random.default_rng(0).normal(0, 0.5, size=p["ubar"].shape)
    x, u, lam, hist = sqp.sqp(p, 2)
    assert hist[0]["alpha"] == 1.0
    xr, ur, _ = riccati_lq(p)
    assert np.allclose(x, xr, atol=1e-10)
    # second QP step is (numerically) zero
    s = hist[1]["sol"]
    assert np.max(np.abs(s["x"] - hist[0]["sol"]["x"])) < 1e-10


def test_lq_merit_quadratic_identity():
    # For linear dynamics the QP point is feasible, so the defects scale as
    # (1 - alpha) and the merit along the step is exactly quadratic:
    # Delta_alpha = alpha (1 - eta) D + 1/2 alpha^2 dz'G dz, with D the
    # descent value; this holds for any mu, here from an infeasible start.
    p = _ltv_random(13)
    T, nx, nu = p["T"], p["nx"], p["nu"]
    x, u, _ = sqp.initial_guess(p)            # z = 0 apart from x_0: infeasible
    qpd = qp.qp_data(p, x, u)
    sol = qp.solve_qp(qpd, p["x0"])
    a, idx, det = sqp.line_search(p, x, u, sol["x"], sol["u"])
    assert det["fl1"] > 0
    dz = qp.join_w(sol["x"] - x, sol["u"] - u, np.zeros((T + 1, nx)))[:sol["parts"]["nz"]]
    curv = dz @ sol["parts"]["G"] @ dz
    for k, al in enumerate(sqp.ALPHAS):
        expect = al * (1 - sqp.ETA) * det["D"] + 0.5 * al * al * curv
        assert det["dphi"][k] == pytest.approx(expect, rel=1e-9, abs=1e-10)
    # the first candidate with a negative value is selected, else the smallest
    neg = [k for k in range(len(sqp.ALPHAS)) if det["dphi"][k] < 0]
    assert idx == (neg[0] if neg else len(sqp.ALPHAS) - 1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sqp_cartpole_reaches_fixed_point(seed):
    # converged SQP: the QP formed at the iterate reproduces the iterate
    p = W.cartpole_batch(seed, batch=1)[0]
    x, u, lam, hist = sqp.sqp(p, 8)
    assert [h["alpha"] for h in hist[:3]] == [1.0, 1.0, 1.0]
    qpd = qp.qp_data(p, x, u)
    sol = qp.solve_qp(qpd, p["x0"])
    assert np.max(np.abs(sol["x"] - x)) < 1e-7
    assert np.max(np.abs(sol["u"] - u)) < 1e-7
    assert np.max(np.abs(sol["lam"] - lam)) < 1e-5


# ---------------------------------------------------------------------------
# Backward pass
# ---------------------------------------------------------------------------
def _qp_map(p, xbar, ubar):
    qpd = qp.qp_data(p, xbar, ubar)
    return qp.solve_qp(qpd, p["x0"])


def _loss(p, xbar, ubar, gx, gu, gl):
    s = _qp_map(p, xbar, ubar)
    return np.sum(gx * s["x"]) + np.sum(gu * s["u"]) + np.sum(gl * s["lam"])


@pytest.mark.parametrize("with_lambda", [False, True])
def test_vjp_matches_central_fd_ltv(with_lambda):
    p = _ltv_random(9, T=5, nx=3, nu=2)
    T, nx, nu = p["T"], p["nx"], p["nu"]
    xbar, ubar = np.zeros((T + 1, nx)), np.zeros((T, nu))
    g = W.loss_cotangents([p], seed=1, with_lambda=with_lambda)[0]
    qpd = qp.qp_data(p, xbar, ubar)
    sol = qp.solve_qp(qpd, p["x0"])
    grads, _ = backward.vjp(p, xbar, ubar, qpd, sol, g["gx"], g["gu"], g["glam"])
    rng = np.random.default_rng(0)
    for key in ("A", "B", "c", "Qd", "q", "Rd", "r", "x0"):
        dirn = rng.standard_normal(p[key].shape)
        h = 1e-6
        pp = dict(p); pp[key] = p[key] + h * dirn
        pm = dict(p); pm[key] = p[key] - h * dirn
        fd = (_loss(pp, xbar, ubar, g["gx"], g["gu"], g["glam"])
              - _loss(pm, xbar, ubar, g["gx"], g["gu"], g["glam"])) / (2 * h)
        an = np.sum(grads[key] * dirn)
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-8), key


def test_envelope_identity():
    p = _ltv_random(10)
    T, nx, nu = p["T"], p["nx"], p["nu"]
    xbar, ubar = np.zeros((T + 1, nx)), np.zeros((T, nu))
    qpd = qp.qp_data(p, xbar, ubar)
    sol = qp.solve_qp(qpd, p["x0"])
    gx = np.array([np.diag(qpd["Q"][t]) * sol["x"][t] + qpd["q"][t] for t in range(T + 1)])
    gu = np.array([np.diag(qpd["R"][t]) * sol["u"][t] + qpd["r"][t] for t in range(T)])
    xt, ut, lt = backward.adjoint(sol, gx, gu)
    assert np.max(np.abs(xt)) < 1e-12 and np.max(np.abs(ut)) < 1e-12
    assert np.allclose(lt, -sol["lam"], atol=1e-12)


def test_optimal_cost_sensitivity_to_initial_state():
    p = _ltv_random(12)
    T, nx, nu = p["T"], p["nx"], p["nu"]
    xbar, ubar = np.zeros((T + 1, nx)), np.zeros((T, nu))

    def jstar(x0):
        pp = dict(p); pp["x0"] = x0
        s = _qp_map(pp, xbar, ubar)
        return sqp.total_cost(pp, s["x"], s["u"]), s["lam"]

    _, lam = jstar(p["x0"])
    h = 1e-6
    for i in range(nx):
        e = np.zeros(nx); e[i] = h
        fd = (jstar(p["x0"] + e)[0] - jstar(p["x0"] - e)[0]) / (2 * h)
        assert fd == pytest.approx(-lam[0, i], rel=1e-6, abs=1e-9)


def test_softplus_theta_vjp_matches_fd():
    p = W.bicycle_batch(5, batch=1, T=12)[0]
    T, nx, nu = p["T"], p["nx"], p["nu"]
    xbar, ubar, _ = sqp.initial_guess(p)
    g = W.loss_cotangents([p], seed=2)[0]
    qpd = qp.qp_data(p, xbar, ubar)
    sol = qp.solve_qp(qpd, p["x0"])
    grads, _ = backward.vjp(p, xbar, ubar, qpd, sol, g["gx"], g["gu"])
    rng = np.random.default_rng(1)
    for key in ("theta", "xref", "x0"):
        dirn = rng.standard_normal(p[key].shape)
        h = 1e-4   # the map is smooth; a larger step keeps round-off out
        pp = dict(p); pp[key] = p[key] + h * dirn
        pm = dict(p); pm[key] = p[key] - h * dirn
        fd = (_loss(pp, xbar, ubar, g["gx"], g["gu"], 0.0)
              - _loss(pm, xbar, ubar, g["gx"], g["gu"], 0.0)) / (2 * h)
        an = np.sum(grads[key] * dirn)
        assert an == pytest.approx(fd, rel=2e-6, abs=1e-8), key


def test_blockwise_kkt_residual_equals_dense():
    # the stage-by-stage residual is the dense ||K w - rhs|| / ||rhs|| written
    # out by blocks: equal on random points and problems of every model
    rng = np.random.default_rng(11)
    cases = [W.ltv_problem(rng, 6, 3, 2), W.cartpole_batch(2, batch=1, T=7)[0],
             W.bicycle_batch(3, batch=1, T=5)[0]]
    for p in cases:
        T, nx, nu = p["T"], p["nx"], p["nu"]
        xb, ub, _ = oracle.sqp.initial_guess(p)
        qpd = oracle.qp.qp_data(p, xb, ub)
        for _ in range(3):
            x = rng.standard_normal((T + 1, nx))
            u = rng.standard_normal((T, nu))
            lam = rng.standard_normal((T + 1, nx))
            a = oracle.qp.kkt_residual(qpd, p["x0"], x, u, lam)
            b = oracle.qp.kkt_residual_blocks(qpd, p["x0"], x, u, lam)
            assert abs(a - b) <= 1e-12 * max(a, 1.0), (a, b)
        s = oracle.qp.solve_qp(qpd, p["x0"])
        assert oracle.qp.kkt_residual_blocks(qpd, p["x0"], s["x"], s["u"], s["lam"]) < 1e-12


# ---------------------------------------------------------------------------
# Forward-mode sensitivity (JVP) of the final QP's solution map
# ---------------------------------------------------------------------------
def _jvp_case(p, seed):
    from oracle import backward, qp, sqp
    xb, ub, _ = sqp.initial_guess(p)
    qpd = qp.qp_data(p, xb, ub)
    sol = qp.solve_qp(qpd, p["x0"])
    rng = np.random.default_rng(seed)
    keys = ["x0", "Qd", "q", "Rd", "r"] + (["A", "B", "c"] if p["dyn"] == "ltv" else [])
    tan = {k: rng.standard_normal(np.shape(p[k])) for k in keys}
    return backward, qp, xb, ub, qpd, sol, tan, rng


@pytest.mark.parametrize("which", ["lq", "cartpole"])
def test_jvp_is_dual_to_the_vjp(which):
    # <g, J v> = <J' g, v>: the forward and reverse modes are computed by
    # different code (dK w versus the QP-data cotangents)
    p = W.lq_batch(3)[1] if which == "lq" else W.cartpole_batch(2, batch=2)[0]
    backward, qp, xb, ub, qpd, sol, tan, rng = _jvp_case(p, 5)
    dx, du, dl = backward.jvp(p, xb, ub, qpd, sol, tan)
    gx, gu, gl = (rng.standard_normal(a.shape) for a in (dx, du, dl))
    g, _ = backward.vjp(p, xb, ub, qpd, sol, gx, gu, gl)
    lhs = np.sum(gx * dx) + np.sum(gu * du) + np.sum(gl * dl)
    rhs = sum(np.sum(g[k] * tan[k]) for k in tan)
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1.0), (lhs, rhs)


def test_jvp_matches_finite_differences_of_the_solution_map():
    p = W.lq_batch(3)[2]
    backward, qp, xb, ub, qpd, sol, tan, rng = _jvp_case(p, 6)
    dw = backward.jvp(p, xb, ub, qpd, sol, tan)
    h = 1e-6

    def solve_at(s):
        pm = backward._moved(p, tan, s)
        so = qp.solve_qp(qp.qp_data(pm, xb, ub), pm["x0"])
        return so["x"], so["u"], so["lam"]

    fd = [(a - b) / (2 * h) for a, b in zip(solve_at(h), solve_at(-h))]
    for f, j in zip(fd, dw):
        assert np.max(np.abs(f - j)) <= 1e-7 * np.max(np.abs(j)), np.max(np.abs(f - j))
