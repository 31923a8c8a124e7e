"""GPU tests of the continuous-batching server: every result is the same when
its request is served alone and inside a concurrent mix, served results match
the oracle (KKT residual and gradients), and the device-resident warm start
cuts PCG iterations."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06179_amd import _lib, batch
from paper_2510_06179_amd import workloads as W
from paper_2510_06179_amd.serving import Server
from _parity import REL_TOL, fp32_floor, gpu_only, kkt_gate, rel_err

pytestmark = [pytest.mark.gpu, gpu_only]

# linear problems: one SQP iteration with the full step solves them exactly
OPTS = dict(sqp_iters=1, alphas=(1.0,), pcg_tol=1e-6, bwd_pcg_tol=1e-6, bwd_warm_start=True)


def sessions(n, seed, Ts=(16, 32, 64, 128)):
    rng = np.random.default_rng(seed)
    return [W.ltv_problem(rng, int(rng.choice(Ts)), int(rng.choice([4, 8, 12, 16])),
                          int(rng.choice([2, 4]))) for _ in range(n)]


def request_stream(probs, n_req, seed, p_bwd=0.3):
    """Seeded requests: (session, backward, x0, dl or None)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_req):
        s = int(rng.integers(len(probs)))
        p = probs[s]
        bwd = bool(rng.random() < p_bwd)
        x0 = W.f32(p["x0"] + rng.normal(0.0, 0.01, size=p["nx"])).astype(np.float32)
        dl = None
        if bwd and rng.random() < 0.7:
            N, T = p["T"] + 1, p["T"]
            dl = np.concatenate([rng.standard_normal(N * p["nx"]), rng.standard_normal(T * p["nu"]),
                                 np.zeros(N * p["nx"])]).astype(np.float32)
        out.append((s, bwd, x0, dl))
    return out


def make_server(probs, **kw):
    args = dict(max_sessions=len(probs), max_T=max(p["T"] for p in probs),
                max_nx=max(p["nx"] for p in probs), max_nu=max(p["nu"] for p in probs),
                hbm_budget=1 << 30)
    args.update(OPTS)
    args.update(kw)
    srv = Server(**args)
    for k, p in enumerate(probs):
        srv.add_session(k, p)
    return srv


def serve_alone(probs, reqs):
    srv = make_server(probs, max_batch=1, max_inflight=1)
    try:
        out = []
        for s, bwd, x0, dl in reqs:
            out.append(srv.wait(srv.submit(s, bwd, x0, dl), timeout=60))
        return out
    finally:
        srv.close()


def serve_mix(probs, reqs, max_inflight=3, max_batch=64):
    srv = make_server(probs, max_batch=max_batch, max_inflight=max_inflight)
    try:
        tickets = [srv.submit(s, bwd, x0, dl) for s, bwd, x0, dl in reqs]
        out = [srv.wait(t, timeout=120) for t in tickets]
        return out, srv.stats()
    finally:
        srv.close()


def test_alone_and_in_the_mix_are_identical():
    probs = sessions(40, seed=11)
    reqs = request_stream(probs, 200, seed=12)
    alone = serve_alone(probs, reqs)
    mix, st = serve_mix(probs, reqs)
    assert st["max_group_size"] > 1, "the mix never batched"
    for k, (a, b) in enumerate(zip(alone, mix)):
        assert a["state"] == b["state"] == _lib.REQ_DONE, k
        assert a["status"] == b["status"], k
        assert np.array_equal(a["info"], b["info"]), k
        assert np.array_equal(a["sol"], b["sol"]), (k, rel_err(b["sol"], a["sol"]))
        if reqs[k][1]:
            assert np.array_equal(a["grad"], b["grad"]), (k, rel_err(b["grad"], a["grad"]))


def test_served_results_match_the_oracle():
    probs = sessions(12, seed=21, Ts=(16, 32, 64))
    reqs = request_stream(probs, 60, seed=22, p_bwd=0.5)
    mix, st = serve_mix(probs, reqs, max_inflight=2, max_batch=16)
    cur_dl = [np.zeros(batch.pack([p]).sol_len, np.float32) for p in probs]
    bad = _lib.PROB_NONPD | _lib.PROB_NONFINITE | _lib.PROB_PCG_MAXITER
    n_grad = 0
    for k, ((s, bwd, x0, dl), r) in enumerate(zip(reqs, mix)):
        assert r["state"] == _lib.REQ_DONE and not (r["status"] & bad), (k, r["status"])
        p = dict(probs[s])
        p["x0"] = x0.astype(np.float64)
        if dl is not None:
            cur_dl[s] = dl
        pk = batch.pack([p])
        x, u, lam = (np.asarray(a, np.float64) for a in batch.split_sol(pk, r["sol"], 0))
        N, T = p["T"] + 1, p["T"]
        qpd = oracle.qp.qp_data(p, np.zeros((N, p["nx"])), np.zeros((T, p["nu"])))
        res = oracle.qp.kkt_residual(qpd, p["x0"], x, u, lam)
        assert res <= kkt_gate(fp32_floor(p, qpd)), (k, res)
        if bwd:
            gx, gu, gl = batch.split_sol(pk, cur_dl[s].astype(np.float64), 0)
            sol = oracle.qp.solve_qp(qpd, p["x0"])
            g_o, _ = oracle.backward.vjp(p, np.zeros((N, p["nx"])), np.zeros((T, p["nu"])), qpd,
                                         sol, gx, gu, gl)
            g = batch.split_grad(pk, r["grad"], 0)
            for key in ("A", "B", "c", "Qd", "q", "Rd", "r", "x0"):
                assert rel_err(g[key], g_o[key]) <= REL_TOL, (k, key, rel_err(g[key], g_o[key]))
            n_grad += 1
    assert n_grad >= 10


def test_device_warm_start_cuts_pcg_iterations():
    probs = sessions(16, seed=31)
    rng = np.random.default_rng(32)
    srv = make_server(probs, max_batch=16, max_inflight=1)
    try:
        cold, warm = [], []
        for rnd in range(2):
            ts = []
            for k, p in enumerate(probs):
                x0 = (p["x0"] + rng.normal(0.0, 0.01, size=p["nx"])).astype(np.float32)
                ts.append(srv.submit(k, False, x0))
            res = [srv.wait(t, timeout=60) for t in ts]
            (cold if rnd == 0 else warm).extend(int(r["info"][0]) for r in res)
        assert sum(warm) < 0.8 * sum(cold), (sum(warm), sum(cold))
    finally:
        srv.close()
