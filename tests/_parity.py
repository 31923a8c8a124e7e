"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare with the FP64 oracle.

Tolerances (float32 GPU vs float64 oracle): relative KKT residual of the QP
<= 1e-5, relative 2-norm error of solutions, multipliers and gradients <= 1e-4.

Float32 floor.  The outputs are float32, so no answer can have a smaller KKT
residual than the oracle's exact solution rounded to float32.  For problems
whose multipliers are large next to the right-hand side (the cart-pole, whose
costs have no linear term) that floor alone exceeds 1e-5.  Such an instance is
"beyond float32": it is held to FLOOR_FACTOR times its floor instead of 1e-5,
and the tests report how many there were.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06179_amd import batch
from paper_2510_06179_amd.solver import BatchSolver

KKT_TOL = 1e-5
REL_TOL = 1e-4
FLOOR_FACTOR = 4.0

gpu_only = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def gpu_solve(problems, **opts):
    """Run dmpc_solve; returns (solver, per-problem (x, u, lam), status, info)."""
    s = BatchSolver(problems, **opts)
    sol = s.solve()
    torch.cuda.synchronize()
    out = sol.cpu().numpy()
    res = [tuple(np.array(a, np.float64) for a in batch.split_sol(s.packed, out, k))
           for k in range(s.packed.count)]
    return s, res, s.status.cpu().numpy(), s.info.cpu().numpy()


def saved_qp(solver, k):
    return {key: v.cpu().numpy().astype(np.float64) for key, v in solver.saved_qp(k).items()}


def fp32_floor(prob, qpd):
    """KKT residual of the oracle's exact QP solution rounded to float32."""
    s = oracle.qp.solve_qp(qpd, prob["x0"])
    f = lambda a: np.asarray(a, np.float32).astype(np.float64)
    return oracle.qp.kkt_residual(qpd, prob["x0"], f(s["x"]), f(s["u"]), f(s["lam"]))


def kkt_gate(floor):
    """Per-instance KKT bound: 1e-5, or FLOOR_FACTOR x the float32 floor for
    an instance beyond float32."""
    return max(KKT_TOL, FLOOR_FACTOR * floor)


def oracle_kkt_of_gpu_qp(prob, solver, k):
    """Relative KKT residual (FP64) of the GPU's last QP solution, for the QP
    the oracle forms at the GPU's last linearisation point; also the bound it
    is held to.  Returns (residual, bound, saved workspace views, QP data)."""
    sq = saved_qp(solver, k)
    qpd = oracle.qp.qp_data(prob, sq["xlin"], sq["ulin"])
    res = oracle.qp.kkt_residual(qpd, prob["x0"], sq["xp"], sq["up"], sq["lam"])
    return res, kkt_gate(fp32_floor(prob, qpd)), sq, qpd
