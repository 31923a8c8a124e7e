"""GPU parity of the backward pass (Alg. backward): adjoint solve and VJP
through the C ABI against the oracle's dense-KKT IFT gradient."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06179_amd import _lib, batch
from paper_2510_06179_amd import workloads as W
from paper_2510_06179_amd.solver import dmpc
from _parity import REL_TOL, gpu_only, gpu_solve, rel_err, saved_qp

pytestmark = [pytest.mark.gpu, gpu_only]

BAD = _lib.PROB_NONPD | _lib.PROB_NONFINITE


def _cotangent_arena(s, cots):
    return torch.from_numpy(batch.sol_like(
        s.packed, [(c["gx"], c["gu"], c["glam"]) for c in cots])).to(s.device)


def _run(probs, cots, **opts):
    s, res, status, info = gpu_solve(probs, **opts)
    adj, grad = s.solve_backward(_cotangent_arena(s, cots))
    torch.cuda.synchronize()
    return s, res, adj.cpu().numpy(), grad.cpu().numpy(), s.status.cpu().numpy(), s.info.cpu().numpy()


def _oracle_grads(p, s, k, c):
    sq = saved_qp(s, k)
    qpd = oracle.qp.qp_data(p, sq["xlin"], sq["ulin"])
    sol = oracle.qp.solve_qp(qpd, p["x0"])
    return oracle.backward.vjp(p, sq["xlin"], sq["ulin"], qpd, sol, c["gx"], c["gu"], c["glam"])


@pytest.mark.parametrize("with_lambda", [False, True])
def test_lq_gradients(with_lambda):
    probs = W.lq_batch(3)
    cots = W.loss_cotangents(probs, seed=3, with_lambda=with_lambda)
    s, res, adj, grad, status, info = _run(probs, cots, sqp_iters=1, alphas=(1.0,), pcg_tol=1e-6,
                                           bwd_pcg_tol=1e-6)
    assert not np.any(status & BAD), status
    for k, p in enumerate(probs):
        g_o, (xt, ut, lt) = _oracle_grads(p, s, k, cots[k])
        g = batch.split_grad(s.packed, grad, k)
        for key in ("A", "B", "c", "Qd", "q", "Rd", "r", "x0"):
            assert rel_err(g[key], g_o[key]) <= REL_TOL, (k, key, rel_err(g[key], g_o[key]))
        ax, au, al = batch.split_sol(s.packed, adj, k)
        assert rel_err(ax, xt) <= REL_TOL and rel_err(au, ut) <= REL_TOL
        assert rel_err(al, lt) <= REL_TOL


def test_cartpole_gradients_after_ten_iterations():
    probs = W.cartpole_batch(5, batch=16)
    cots = W.loss_cotangents(probs, seed=5)
    s, res, adj, grad, status, info = _run(probs, cots, sqp_iters=10, pcg_tol=1e-6,
                                           bwd_pcg_tol=1e-6)
    assert not np.any(status & BAD), status
    for k, p in enumerate(probs):
        g_o, _ = _oracle_grads(p, s, k, cots[k])
        g = batch.split_grad(s.packed, grad, k)
        for key in ("Qd", "q", "Rd", "r", "x0"):
            assert rel_err(g[key], g_o[key]) <= REL_TOL, (k, key, rel_err(g[key], g_o[key]))
        assert np.all(g["params"] == 0.0)


def test_envelope_identity_on_gpu():
    # dl/dz = G z + b (gradient of the QP objective at its solution) gives
    # z~ = 0 and lambda~ = -lambda
    probs = W.lq_batch(6, batch=4)
    s, res, status, info = gpu_solve(probs, sqp_iters=1, alphas=(1.0,), pcg_tol=1e-6)
    cots = []
    for k, p in enumerate(probs):
        sq = saved_qp(s, k)
        gx = sq["Qd"] * sq["xp"] + p["q"]
        gu = sq["Rd"] * sq["up"] + p["r"]
        cots.append(dict(gx=gx, gu=gu, glam=np.zeros_like(gx)))
    adj, grad = s.solve_backward(_cotangent_arena(s, cots))
    adj = adj.cpu().numpy()
    for k in range(len(probs)):
        ax, au, al = batch.split_sol(s.packed, adj, k)
        lam = saved_qp(s, k)["lam"]
        assert np.max(np.abs(ax)) <= 1e-4 * max(1.0, np.max(np.abs(lam)))
        assert rel_err(al, -lam) <= REL_TOL


def test_autograd_function_matches_abi():
    probs = W.lq_batch(7, batch=3)
    s, res, status, info = gpu_solve(probs, sqp_iters=1, alphas=(1.0,))
    cots = W.loss_cotangents(probs, seed=7)
    g_sol = _cotangent_arena(s, cots)
    data = s.data.clone().requires_grad_(True)
    sol = dmpc(data, s)
    (gd,) = torch.autograd.grad(sol, data, grad_outputs=g_sol)
    _, grad = s.solve_backward(g_sol)
    torch.cuda.synchronize()
    assert torch.allclose(gd, grad, rtol=0, atol=0)


def test_backward_warm_start_reduces_iterations():
    probs = W.lq_batch(8, batch=4)
    cots = W.loss_cotangents(probs, seed=8)
    s, res, adj, grad, status, info = _run(probs, cots, sqp_iters=1, alphas=(1.0,),
                                           bwd_warm_start=True)
    cold = info[:, 1].copy()
    adj_t = torch.from_numpy(adj).to(s.device)
    _, grad2 = s.solve_backward(_cotangent_arena(s, cots), adj=adj_t)
    torch.cuda.synchronize()
    warm = s.info.cpu().numpy()[:, 1]
    assert np.all(warm < cold)
    assert rel_err(grad2.cpu().numpy(), grad) <= REL_TOL
