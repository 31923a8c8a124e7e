"""GPU parity of the kernels that keep the Schur rows in registers and apply
the preconditioner of Eq. S_Phiinv in factored form (Phi^-1 = D^-1 - D^-1 E
D^-1 with the inverted diagonal blocks in LDS), forced through the tuning
table: forward (several SQP iterations) and backward against the FP64 oracle
on ragged shapes (rows not a multiple of the workgroup, one or two rows per
thread), and JVP.  The same for the variant whose last value slot keeps its
Schur rows in LDS (T = 128, nx = 16: 16 rows past four register slots of 512
threads; T = 127: none; shorter horizons: register slots partly empty), and
for the PCG on the Schur system scaled by the Cholesky factors of its
diagonal blocks."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06179_amd import _lib, batch
from paper_2510_06179_amd import workloads as W
from _parity import REL_TOL, gpu_only, gpu_solve, oracle_kkt_of_gpu_qp, rel_err

pytestmark = [pytest.mark.gpu, gpu_only]

BAD = _lib.PROB_NONPD | _lib.PROB_NONFINITE | _lib.PROB_PCG_MAXITER | _lib.PROB_BWD_PCG_MAXITER


def _saved_table():
    lib = _lib.load()
    n = lib.dmpc_get_tuning(None, 0)
    rows = np.zeros((max(n, 1), 7), np.int32)
    lib.dmpc_get_tuning(rows.ctypes.data, n)
    return [tuple(int(v) for v in r) for r in rows[:n]]


@pytest.fixture
def factored_table():
    saved = _saved_table()
    # two rows per thread: 640 threads hold N <= 80 stages of nx = 16,
    # 1024 threads N <= 170 of nx = 12; smaller horizons with fewer threads
    _lib.install_tuning([(16, 1, 19, 2, 640, 3, 192), (16, 20, 79, 2, 640, 3, 640),
                         (16, 80, 127, 2, 1024, 3, 1024),
                         (12, 1, 39, 2, 1024, 3, 256), (12, 40, 169, 2, 1024, 3, 1024)])
    yield
    _lib.install_tuning(saved)


def _shapes(seed):
    rng = np.random.default_rng(seed)
    shapes = [(3, 16, 4), (11, 16, 2), (40, 16, 4), (64, 16, 4), (90, 16, 3),
              (5, 12, 2), (33, 12, 4), (128, 12, 4), (150, 12, 2)]
    probs = []
    for T, nx, nu in shapes:
        p = W.ltv_problem(rng, T, nx, nu)
        p["c"] = W.f32(rng.normal(0, 0.1, size=(T, nx)))
        p["init"] = "rollout"
        probs.append(p)
    return probs


@pytest.fixture
def lds_row_table():
    saved = _saved_table()
    _lib.install_tuning([(16, 1, 128, 5, 512, 4, 512)])
    yield
    _lib.install_tuning(saved)


@pytest.fixture
def lds_row_mixed_table():
    # nx = 12 with three register slots; nx = 16 with one and two
    saved = _saved_table()
    _lib.install_tuning([(12, 1, 132, 4, 512, 4, 512), (16, 1, 35, 2, 512, 4, 512),
                         (16, 36, 67, 3, 512, 4, 512)])
    yield
    _lib.install_tuning(saved)


def test_factored_forward_backward_jvp(factored_table):
    _check(_shapes(11), 3)


def test_lds_row_slot_forward_backward_jvp(lds_row_table):
    rng = np.random.default_rng(21)
    probs = []
    for T, nu in [(128, 4), (128, 2), (127, 3), (100, 2), (9, 4)]:
        p = W.ltv_problem(rng, T, 16, nu)
        p["c"] = W.f32(rng.normal(0, 0.1, size=(T, 16)))
        p["init"] = "rollout"
        probs.append(p)
    _check(probs, 4)


@pytest.fixture
def scaled_table():
    saved = _saved_table()
    _lib.install_tuning([(16, 1, 159, 5, 512, 5, 512)])
    yield
    _lib.install_tuning(saved)


def test_scaled_system_forward_backward_jvp(scaled_table):
    # the Cholesky-scaled Schur system (register_rows 5): full and partly
    # empty register slots
    rng = np.random.default_rng(29)
    probs = []
    for T, nx, nu in [(128, 16, 4), (64, 16, 2), (31, 16, 3), (9, 16, 4), (159, 16, 2)]:
        p = W.ltv_problem(rng, T, nx, nu)
        p["c"] = W.f32(rng.normal(0, 0.1, size=(T, nx)))
        p["init"] = "rollout"
        probs.append(p)
    _check(probs, 5)


@pytest.fixture
def scaled_small_table():
    saved = _saved_table()
    _lib.install_tuning([(16, 1, 23, 2, 192, 5, 192), (16, 24, 35, 3, 192, 5, 192),
                         (8, 1, 71, 3, 192, 5, 192), (8, 72, 143, 3, 384, 5, 384)])
    yield
    _lib.install_tuning(saved)


def test_scaled_system_small_workgroups(scaled_small_table):
    # register_rows 5 on 192 and 384 threads, nx = 16 and 8, full and partly
    # empty slots
    rng = np.random.default_rng(31)
    probs = []
    for T, nx, nu in [(20, 16, 2), (32, 16, 4), (35, 16, 3), (64, 8, 2), (71, 8, 4), (10, 8, 3),
                      (128, 8, 4), (100, 8, 2)]:
        p = W.ltv_problem(rng, T, nx, nu)
        p["c"] = W.f32(rng.normal(0, 0.1, size=(T, nx)))
        p["init"] = "rollout"
        probs.append(p)
    _check(probs, 5)


@pytest.fixture
def scaled_nx12_table():
    saved = _saved_table()
    _lib.install_tuning([(12, 1, 47, 3, 192, 5, 192), (12, 48, 143, 3, 576, 5, 576)])
    yield
    _lib.install_tuning(saved)


def test_scaled_system_nx12(scaled_nx12_table):
    # nx = 12: a stage's rows can straddle two waves (workgroup barriers in
    # the factorisation); 192 and 576 threads
    rng = np.random.default_rng(37)
    probs = []
    for T, nu in [(128, 4), (143, 2), (100, 3), (32, 2), (16, 4), (5, 3)]:
        p = W.ltv_problem(rng, T, 12, nu)
        p["c"] = W.f32(rng.normal(0, 0.1, size=(T, 12)))
        p["init"] = "rollout"
        probs.append(p)
    _check(probs, 5)


def test_lds_row_slot_other_widths(lds_row_mixed_table):
    # nx = 12: T = 128 (12 LDS rows), 100 (register slots partly empty), 5;
    # nx = 16: T = 32 and 64 (16 LDS rows each), 20, 50
    rng = np.random.default_rng(23)
    probs = []
    for T, nx, nu in [(128, 12, 4), (100, 12, 2), (5, 12, 3), (32, 16, 2), (20, 16, 4),
                      (64, 16, 3), (50, 16, 2)]:
        p = W.ltv_problem(rng, T, nx, nu)
        p["c"] = W.f32(rng.normal(0, 0.1, size=(T, nx)))
        p["init"] = "rollout"
        probs.append(p)
    _check(probs, 4)


def _check(probs, mode):
    s, res, status, info = gpu_solve(probs, sqp_iters=3, pcg_tol=1e-6, bwd_pcg_tol=1e-6)
    assert all(d["register_rows"] == mode for d in s.describe()), s.describe()
    assert not np.any(status & BAD), (status, info)
    cots = W.loss_cotangents(probs, seed=11, with_lambda=True)
    dl = torch.from_numpy(batch.sol_like(s.packed, [(c["gx"], c["gu"], c["glam"]) for c in cots]))
    adj, grad = s.solve_backward(dl.to(s.device))
    torch.cuda.synchronize()
    assert not np.any(s.status.cpu().numpy() & BAD)
    grad = grad.cpu().numpy()
    rng = np.random.default_rng(12)
    tans, tps = [], []
    for p in probs:
        t = {k: W.f32(rng.standard_normal(np.shape(p[k])))
             for k in ("x0", "Qd", "q", "Rd", "r", "A", "B", "c")}
        q = dict(p)
        q.update(t)
        tans.append(t)
        tps.append(q)
    jv = s.solve_jvp(torch.from_numpy(batch.pack(tps).data).to(s.device))
    torch.cuda.synchronize()
    jv = jv.cpu().numpy()
    for k, p in enumerate(probs):
        kkt, bound, sq, qpd = oracle_kkt_of_gpu_qp(p, s, k)
        assert kkt <= bound, (k, kkt, bound)
        sol = oracle.qp.solve_qp(qpd, p["x0"])
        x, u, lam = res[k]
        assert rel_err(x, sol["x"]) <= REL_TOL and rel_err(u, sol["u"]) <= REL_TOL, k
        assert rel_err(lam, sol["lam"]) <= REL_TOL, k
        g_o, _ = oracle.backward.vjp(p, sq["xlin"], sq["ulin"], qpd, sol, cots[k]["gx"],
                                     cots[k]["gu"], cots[k]["glam"])
        g = batch.split_grad(s.packed, grad, k)
        for key in ("A", "B", "c", "Qd", "q", "Rd", "r", "x0"):
            assert rel_err(g[key], g_o[key]) <= REL_TOL, (k, key, rel_err(g[key], g_o[key]))
        ref = oracle.backward.jvp(p, sq["xlin"], sq["ulin"], qpd, sol, tans[k])
        got = batch.split_sol(s.packed, jv, k)
        for name, a, b in zip(("dx", "du", "dlam"), got, ref):
            assert rel_err(a, b) <= REL_TOL, (k, name, rel_err(a, b))
