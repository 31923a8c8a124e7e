"""GPU parity for the large state size of the serving mix (nx=32, nu=8):
the Schur rows are read from the workspace, and at the long horizon (T=256)
the iterate, QP solution and line-search region live in the workspace too.
Short horizons are checked against the dense FP64 oracle; the long horizon
(KKT dimension 18,496) through the stage-by-stage KKT residual of the forward
QP and of the adjoint system."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06179_amd import _lib, batch
from paper_2510_06179_amd import workloads as W
from _parity import KKT_TOL, REL_TOL, fp32_floor, gpu_only, gpu_solve, kkt_gate, rel_err, saved_qp

pytestmark = [pytest.mark.gpu, gpu_only]

BAD = _lib.PROB_NONPD | _lib.PROB_NONFINITE | _lib.PROB_PCG_MAXITER | _lib.PROB_BWD_PCG_MAXITER
OPTS = dict(sqp_iters=1, alphas=(1.0,), pcg_tol=1e-6, bwd_pcg_tol=1e-6)


def _large(seed, n, T):
    rng = np.random.default_rng(seed)
    return [W.ltv_problem(rng, T, 32, 8) for _ in range(n)]


def _adjoint_residual(qpd, cot, xt, ut, lt):
    """K [z~; lam~] = (dl/dz, dl/dlam), stage by stage."""
    q2 = dict(qpd)
    q2["q"] = [-g for g in cot["gx"]]
    q2["r"] = [-g for g in cot["gu"]]
    q2["C"] = [cot["glam"][t + 1] for t in range(qpd["T"])]
    return oracle.qp.kkt_residual_blocks(q2, cot["glam"][0], xt, ut, lt)


def test_nx32_short_horizon_against_dense_oracle():
    probs = _large(41, 3, 40)
    s, res, status, info = gpu_solve(probs, **OPTS)
    assert not np.any(status & BAD), status
    assert all(d["nx"] == 32 for d in s.describe())
    cots = W.loss_cotangents(probs, seed=41)
    dl = torch.from_numpy(batch.sol_like(s.packed, [(c["gx"], c["gu"], c["glam"]) for c in cots]))
    adj, grad = s.solve_backward(dl.to(s.device))
    torch.cuda.synchronize()
    adj, grad = adj.cpu().numpy(), grad.cpu().numpy()
    assert not np.any(s.status.cpu().numpy() & BAD)
    for k, p in enumerate(probs):
        sq = saved_qp(s, k)
        qpd = oracle.qp.qp_data(p, sq["xlin"], sq["ulin"])
        kkt = oracle.qp.kkt_residual(qpd, p["x0"], sq["xp"], sq["up"], sq["lam"])
        assert kkt <= kkt_gate(fp32_floor(p, qpd)), (k, kkt)
        sol = oracle.qp.solve_qp(qpd, p["x0"])
        x, u, lam = res[k]
        assert rel_err(x, sol["x"]) <= REL_TOL and rel_err(lam, sol["lam"]) <= REL_TOL
        g_o, _ = oracle.backward.vjp(p, sq["xlin"], sq["ulin"], qpd, sol, cots[k]["gx"],
                                     cots[k]["gu"])
        g = batch.split_grad(s.packed, grad, k)
        for key in ("A", "B", "c", "Qd", "q", "Rd", "r", "x0"):
            assert rel_err(g[key], g_o[key]) <= REL_TOL, (k, key, rel_err(g[key], g_o[key]))


def test_nx32_long_horizon_kkt_residuals():
    # T=256: the serving mix's large requests (workspace-resident bulk regions)
    probs = _large(42, 2, 256)
    s, res, status, info = gpu_solve(probs, **OPTS)
    assert not np.any(status & BAD), status
    cots = W.loss_cotangents(probs, seed=42)
    dl = torch.from_numpy(batch.sol_like(s.packed, [(c["gx"], c["gu"], c["glam"]) for c in cots]))
    adj, grad = s.solve_backward(dl.to(s.device))
    torch.cuda.synchronize()
    adj = adj.cpu().numpy()
    assert not np.any(s.status.cpu().numpy() & BAD)
    for k, p in enumerate(probs):
        sq = saved_qp(s, k)
        N, T = p["T"] + 1, p["T"]
        qpd = oracle.qp.qp_data(p, np.zeros((N, 32)), np.zeros((T, 8)))
        kkt = oracle.qp.kkt_residual_blocks(qpd, p["x0"], sq["xp"], sq["up"], sq["lam"])
        assert kkt <= KKT_TOL, (k, kkt)
        xt, ut, lt = (np.asarray(a, np.float64) for a in batch.split_sol(s.packed, adj, k))
        ra = _adjoint_residual(qpd, cots[k], xt, ut, lt)
        assert ra <= KKT_TOL, (k, ra)
        assert info[k, 0] > 0 and s.info.cpu().numpy()[k, 1] > 0
