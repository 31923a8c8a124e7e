"""Pins of the oracle's PD projection (Sec. 3.1) and of its exact-Hessian
variant (Sec. 3.4, "Exact SQP vs iLQR") against hand-worked values, special
cases and central differences of the fully converged solution map.  CPU only.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import backward, costs, exact, models, qp, sqp
from paper_2510_06179_amd import workloads as W


def _fr(v):
    return float(Fraction(v))


# ---------------------------------------------------------------------------
# PD projection
# ---------------------------------------------------------------------------
def test_dense_projection_hand_cases(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "pd_projection_2x2.json")))
    for case in g["cases"]:
        H = np.array([[_fr(v) for v in row] for row in case["H"]])
        E = np.array([[_fr(v) for v in row] for row in case["expected"]])
        assert np.allclose(qp.project_pd(H), E, rtol=0, atol=1e-15)


def _clamp_problem(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "pd_clamp_scalar.json")))
    d = {k: _fr(v) for k, v in g["data"].items()}
    p = dict(T=1, nx=1, nu=1, dyn="ltv", cost="diag",
             A=np.array([[[d["a"]]]]), B=np.array([[[d["b"]]]]), c=np.array([[d["c"]]]),
             Qd=np.array([[d["Q0"]], [d["Q1"]]]), q=np.array([[d["q0"]], [d["q1"]]]),
             Rd=np.array([[d["R"]]]), r=np.array([[d["r"]]]), x0=np.array([d["xs"]]))
    xbar = np.array([[d["xbar0"]], [d["xbar1"]]])
    ubar = np.array([[d["ubar"]]])
    assert d["eps"] == qp.PD_EPS
    return g, p, xbar, ubar


def test_clamp_hand_worked_qp_and_solution(golden_dir):
    g, p, xbar, ubar = _clamp_problem(golden_dir)
    qpd = qp.qp_data(p, xbar, ubar)
    e = {k: _fr(v) for k, v in g["expected_qp"].items()}
    assert qpd["Q"][0][0, 0] == e["Q0p"] and qpd["R"][0][0, 0] == e["Rp"]
    assert qpd["Q"][1][0, 0] == e["Q1p"]
    assert qpd["q"][0][0] == pytest.approx(e["q0p"], rel=1e-15)
    assert qpd["r"][0][0] == pytest.approx(e["rp"], rel=1e-12)
    assert qpd["q"][1][0] == pytest.approx(e["q1p"], rel=1e-15)
    sol = qp.solve_qp(qpd, p["x0"])
    e = {k: _fr(v) for k, v in g["expected"].items()}
    assert sol["u"][0, 0] == pytest.approx(e["u0"], rel=1e-12)
    assert sol["x"][1, 0] == pytest.approx(e["x1"], rel=1e-12)
    assert sol["lam"][1, 0] == pytest.approx(e["lam1"], rel=1e-9)
    assert sol["lam"][0, 0] == pytest.approx(e["lam0"], rel=1e-12)


def test_clamp_hand_worked_derivatives(golden_dir):
    # the VJP of the oracle reproduces the hand derivatives through the
    # clamped entries (which reach the linear terms only)
    g, p, xbar, ubar = _clamp_problem(golden_dir)
    e = {k: _fr(v) for k, v in g["expected"].items()}
    qpd = qp.qp_data(p, xbar, ubar)
    sol = qp.solve_qp(qpd, p["x0"])
    z = np.zeros((2, 1))
    gl = np.zeros((2, 1)); gl[0, 0] = 1.0           # l = lam_0
    grads, _ = backward.vjp(p, xbar, ubar, qpd, sol, z, np.zeros((1, 1)), gl)
    assert grads["Qd"][0, 0] == pytest.approx(e["dlam0_dQ0"], rel=1e-9)
    gu = np.ones((1, 1))                             # l = u_0
    grads, _ = backward.vjp(p, xbar, ubar, qpd, sol, z, gu, np.zeros((2, 1)))
    assert grads["Rd"][0, 0] == pytest.approx(e["du0_dR"], rel=1e-9)


def _clamped_ltv(seed=21, T=6, nx=3, nu=2):
    """A linear problem with several cost entries below the PD floor (negative,
    zero and tiny positive), linearised away from zero so that the clamp
    moves the linear terms."""
    rng = np.random.default_rng(seed)
    p = W.ltv_problem(rng, T, nx, nu)
    p["c"] = W.f32(rng.normal(0, 0.3, size=(T, nx)))
    Qd, Rd = p["Qd"].astype(np.float64).copy(), p["Rd"].astype(np.float64).copy()
    Qd[1, 0], Qd[3, 2], Qd[T, 1] = -0.3, 0.0, 1e-8
    Rd[0, 1], Rd[4, 0] = -0.05, 2e-7
    p["Qd"], p["Rd"] = Qd, Rd
    xbar = rng.normal(0, 0.5, size=(T + 1, nx))
    xbar[0] = p["x0"]
    ubar = rng.normal(0, 0.5, size=(T, nu))
    return p, xbar, ubar


def test_clamped_vjp_matches_central_fd():
    p, xbar, ubar = _clamped_ltv()
    qpd = qp.qp_data(p, xbar, ubar)
    assert any(qpd["Q"][t][i, i] == qp.PD_EPS for t in range(p["T"] + 1) for i in range(p["nx"]))
    sol = qp.solve_qp(qpd, p["x0"])
    g = W.loss_cotangents([p], seed=4, with_lambda=True)[0]
    grads, _ = backward.vjp(p, xbar, ubar, qpd, sol, g["gx"], g["gu"], g["glam"])

    def loss(pp):
        s = qp.solve_qp(qp.qp_data(pp, xbar, ubar), pp["x0"])
        return np.sum(g["gx"] * s["x"]) + np.sum(g["gu"] * s["u"]) + np.sum(g["glam"] * s["lam"])

    for key, entries in (("Qd", [(1, 0), (3, 2), (p["T"], 1), (2, 2)]),
                         ("Rd", [(0, 1), (4, 0), (2, 0)])):
        for idx in entries:
            # a step that does not cross the floor: on the clamped side the
            # loss is affine in the entry (it moves the right-hand side only)
            h = min(1e-5, 0.5 * abs(p[key][idx] - qp.PD_EPS))
            pp = dict(p); pp[key] = p[key].copy(); pp[key][idx] += h
            pm = dict(p); pm[key] = p[key].copy(); pm[key][idx] -= h
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert grads[key][idx] == pytest.approx(fd, rel=1e-5, abs=1e-7), (key, idx)


def test_clamped_jvp_is_dual_to_the_vjp():
    p, xbar, ubar = _clamped_ltv(seed=22)
    qpd = qp.qp_data(p, xbar, ubar)
    sol = qp.solve_qp(qpd, p["x0"])
    rng = np.random.default_rng(7)
    tan = {k: rng.standard_normal(np.shape(p[k])) for k in ("x0", "Qd", "q", "Rd", "r", "A", "B", "c")}
    dx, du, dl = backward.jvp(p, xbar, ubar, qpd, sol, tan)
    gx, gu, gl = (rng.standard_normal(a.shape) for a in (dx, du, dl))
    g, _ = backward.vjp(p, xbar, ubar, qpd, sol, gx, gu, gl)
    lhs = np.sum(gx * dx) + np.sum(gu * du) + np.sum(gl * dl)
    rhs = sum(np.sum(g[k] * tan[k]) for k in tan)
    assert abs(lhs - rhs) <= 1e-9 * max(abs(lhs), 1.0), (lhs, rhs)


# ---------------------------------------------------------------------------
# Exact-Hessian variant
# ---------------------------------------------------------------------------
def test_dyn_hessian_linear_dynamics_is_zero():
    rng = np.random.default_rng(3)
    p = W.ltv_problem(rng, 3, 3, 2)
    H = exact.dyn_hessian(p, 1, rng.standard_normal(3), rng.standard_normal(2), rng.standard_normal(3))
    assert np.max(np.abs(H)) < 1e-9


def test_dyn_hessian_cartpole_upright_hand_value():
    # at the upright rest the pole-rate update x4+ = x4 + dt (m_p g s c -
    # m_p L s x4 + u) / den has d2/dx3 dx4 = -dt m_p L / M (den = M there);
    # the other entries of that row vanish (d4 is odd in x3 at x4 = u = 0,
    # and d(1/den)/dx3 = 0 at x3 = 0)
    mc, mp, L, g, dt = 1.0, 0.15, 0.4, 9.81, 0.05
    p = dict(dyn="cartpole", params=np.array([mc, mp, L, g, dt]))
    lam = np.array([0.0, 0.0, 0.0, 1.0])
    H = exact.dyn_hessian(p, 0, np.zeros(4), np.zeros(1), lam, symmetric=False)
    assert H[2, 3] == pytest.approx(-dt * mp * L / (mc + mp), rel=1e-8)
    assert H[3, 2] == pytest.approx(-dt * mp * L / (mc + mp), rel=1e-8)
    assert abs(H[2, 2]) < 1e-9 and abs(H[2, 4]) < 1e-9 and abs(H[3, 3]) < 1e-9


@pytest.mark.parametrize("kind", ["cartpole", "bicycle"])
def test_dyn_hessian_is_symmetric_at_random_points(kind):
    rng = np.random.default_rng(5)
    if kind == "cartpole":
        p = W.cartpole_batch(1, batch=1, T=4)[0]
        x, u = rng.normal(0, 0.5, 4), rng.normal(0, 1, 1)
    else:
        p = W.bicycle_batch(1, batch=1, T=4)[0]
        x, u = p["x0"] + rng.normal(0, 0.05, 8), rng.normal(0, 0.3, 2)
    H = exact.dyn_hessian(p, 0, x, u, rng.standard_normal(p["nx"]), symmetric=False)
    assert np.max(np.abs(H - H.T)) <= 1e-7 * max(np.max(np.abs(H)), 1.0)


def test_exact_equals_gauss_newton_on_linear_dynamics():
    p = W.lq_batch(2, batch=1)[0]
    x, u, lam, it = exact.converge(p, tol=1e-13)
    g = W.loss_cotangents([p], seed=3)[0]
    ge, _ = exact.vjp_exact(p, x, u, lam, g["gx"], g["gu"])
    qpd = qp.qp_data(p, x, u)
    sol = qp.solve_qp(qpd, p["x0"])
    gg, _ = backward.vjp(p, x, u, qpd, sol, g["gx"], g["gu"])
    for k in ("Qd", "q", "Rd", "r", "x0"):
        assert np.allclose(ge[k], gg[k], rtol=1e-9, atol=1e-11), k


def _converged_loss(p, x, u, lam, g):
    xs, us, _, _ = exact.converge(p, x, u, lam, tol=1e-12)
    return float(np.sum(g["gx"] * xs) + np.sum(g["gu"] * us))


def _moved(p, key, dirn, s):
    q = dict(p)
    q[key] = np.asarray(p[key], np.float64) + s * dirn
    return q


def _gn_bias_case(p, keys, seed, h):
    """Exact-Hessian gradient vs central differences of the converged map;
    returns (worst relative FD mismatch, GN bias ||gn - exact|| / ||exact||)."""
    x, u, lam, _ = exact.converge(p, tol=1e-13)
    g = W.loss_cotangents([p], seed=seed)[0]
    ge, _ = exact.vjp_exact(p, x, u, lam, g["gx"], g["gu"])
    qpd = qp.qp_data(p, x, u)
    sol = qp.solve_qp(qpd, p["x0"])
    gg, _ = backward.vjp(p, x, u, qpd, sol, g["gx"], g["gu"])
    rng = np.random.default_rng(seed)
    worst = 0.0
    for key in keys:
        dirn = rng.standard_normal(np.shape(p[key]))
        fd = (_converged_loss(_moved(p, key, dirn, h), x, u, lam, g)
              - _converged_loss(_moved(p, key, dirn, -h), x, u, lam, g)) / (2 * h)
        an = float(np.sum(ge[key] * dirn))
        worst = max(worst, abs(an - fd) / max(abs(fd), 1e-12))
    num = np.sqrt(sum(np.sum((ge[k] - gg[k]) ** 2) for k in keys))
    den = np.sqrt(sum(np.sum(ge[k] ** 2) for k in keys))
    return worst, float(num / den)


def test_exact_gradient_matches_fd_of_converged_map_cartpole():
    p = W.cartpole_batch(4, batch=1, T=10)[0]
    worst, bias = _gn_bias_case(p, ("Qd", "q", "x0"), seed=6, h=1e-4)
    print(f"cart-pole T=10: exact-vs-FD {worst:.2e}, Gauss-Newton bias {bias:.3e}")
    assert worst <= 1e-6
    assert bias > 1e-6     # the dynamics curvature is not negligible here


def test_exact_gradient_matches_fd_of_converged_map_bicycle():
    p = W.bicycle_batch(4, batch=1, T=8)[0]
    worst, bias = _gn_bias_case(p, ("theta", "x0"), seed=7, h=1e-4)
    print(f"bicycle T=8: exact-vs-FD {worst:.2e}, Gauss-Newton bias {bias:.3e}")
    assert worst <= 1e-6
    assert bias > 1e-6
