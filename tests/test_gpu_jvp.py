"""GPU parity of the forward-mode sensitivity (dmpc_solve_jvp): the
derivative of the last QP's (x, u, lambda) along a tangent of the inputs,
against the oracle's JVP (differentiated dense KKT system) at the GPU's last
linearisation point; and the duality <g, J v> = <J' g, v> between the GPU's
JVP and the GPU's VJP."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06179_amd import _lib, batch
from paper_2510_06179_amd import workloads as W
from _parity import REL_TOL, gpu_only, gpu_solve, rel_err, saved_qp

pytestmark = [pytest.mark.gpu, gpu_only]

BAD = _lib.PROB_NONPD | _lib.PROB_NONFINITE | _lib.PROB_BWD_PCG_MAXITER


def _tangents(probs, seed):
    """Seeded tangents of the inputs the JVP reads, and their arena (the data
    arena's layout: a packed batch of tangent 'problems')."""
    rng = np.random.default_rng(seed)
    tans, tps = [], []
    for p in probs:
        keys = ["x0", "Qd", "q", "Rd", "r"] + (["A", "B", "c"] if p["dyn"] == "ltv" else [])
        t = {k: W.f32(rng.standard_normal(np.shape(p[k]))) for k in keys}
        q = dict(p)
        q.update(t)
        if p["dyn"] != "ltv":
            q["params"] = np.zeros_like(np.asarray(p["params"]))
        tans.append(t)
        tps.append(q)
    return tans, torch.from_numpy(batch.pack(tps).data)


def _check(probs, seed, **opts):
    s, res, status, info = gpu_solve(probs, **opts)
    tans, arena = _tangents(probs, seed)
    out = s.solve_jvp(arena.to(s.device))
    torch.cuda.synchronize()
    assert not np.any(s.status.cpu().numpy() & BAD)
    out = out.cpu().numpy()
    for k, p in enumerate(probs):
        sq = saved_qp(s, k)
        qpd = oracle.qp.qp_data(p, sq["xlin"], sq["ulin"])
        sol = oracle.qp.solve_qp(qpd, p["x0"])
        ref = oracle.backward.jvp(p, sq["xlin"], sq["ulin"], qpd, sol, tans[k])
        got = batch.split_sol(s.packed, out, k)
        for name, a, b in zip(("dx", "du", "dlam"), got, ref):
            assert rel_err(a, b) <= REL_TOL, (k, name, rel_err(a, b))
    return s, tans, arena, out


def test_jvp_lq():
    _check(W.lq_batch(3), 21, sqp_iters=1, alphas=(1.0,), pcg_tol=1e-6, bwd_pcg_tol=1e-6)


def test_jvp_ragged_ltv():
    rng = np.random.default_rng(8)
    probs = [W.ltv_problem(rng, T, nx, nu) for T, nx, nu in
             [(5, 2, 1), (20, 4, 2), (33, 4, 2), (9, 8, 4), (40, 8, 2), (7, 12, 3), (30, 16, 4)]]
    _check(probs, 22, sqp_iters=1, alphas=(1.0,), pcg_tol=1e-6, bwd_pcg_tol=1e-6)


def test_jvp_cartpole_after_ten_iterations():
    _check(W.cartpole_batch(4, batch=16), 23, sqp_iters=10, pcg_tol=1e-6, bwd_pcg_tol=1e-6)


def test_jvp_is_dual_to_the_gpu_vjp():
    probs = W.lq_batch(5)
    s, tans, arena, out = _check(probs, 24, sqp_iters=1, alphas=(1.0,), pcg_tol=1e-6,
                                 bwd_pcg_tol=1e-6)
    cots = W.loss_cotangents(probs, seed=24, with_lambda=True)
    dl = torch.from_numpy(batch.sol_like(s.packed, [(c["gx"], c["gu"], c["glam"]) for c in cots]))
    _, grad = s.solve_backward(dl.to(s.device))
    torch.cuda.synchronize()
    grad = grad.cpu().numpy()
    for k in range(len(probs)):
        dx, du, dlam = batch.split_sol(s.packed, out, k)
        c = cots[k]
        lhs = np.sum(c["gx"] * dx) + np.sum(c["gu"] * du) + np.sum(c["glam"] * dlam)
        g = batch.split_grad(s.packed, grad, k)
        rhs = sum(np.sum(np.asarray(g[key], np.float64) * tans[k][key]) for key in tans[k])
        assert abs(lhs - rhs) <= 1e-4 * max(abs(lhs), 1.0), (k, lhs, rhs)


def test_jvp_refuses_softplus_costs():
    probs = W.bicycle_batch(0, batch=2)
    s, res, status, info = gpu_solve(probs, sqp_iters=1, pcg_tol=1e-6)
    with pytest.raises(_lib.DmpcError):
        s.solve_jvp(torch.zeros_like(s.data))
