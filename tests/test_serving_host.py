"""Host logic of the continuous-batching server, on the CPU: the server runs in
dry-run mode (no device work; groups complete after a fixed delay), so
admission, grouping, session exclusivity, ordering, rejection and statistics
are checked without a GPU."""
import ctypes
import time

import numpy as np
import pytest

from paper_2510_06179_amd import _lib, batch
from paper_2510_06179_amd import workloads as W
from paper_2510_06179_amd.serving import Server


def ws_bytes(p):
    pk = batch.pack([p])
    n = ctypes.c_size_t()
    o = _lib.make_opts()
    _lib.check(_lib.load().dmpc_workspace_size(pk.descs.ctypes.data, 1, ctypes.byref(o),
                                               ctypes.byref(n)))
    return n.value


def dry(**kw):
    args = dict(max_sessions=64, max_T=128, max_nx=16, max_nu=4, max_batch=16, max_inflight=2,
                hbm_budget=64 << 20, dry_run=True, dry_run_us=2000)
    args.update(kw)
    return Server(**args)


def uneven(n, seed=0):
    rng = np.random.default_rng(seed)
    return [W.ltv_problem(rng, int(rng.choice([16, 32, 64, 128])), int(rng.choice([4, 8, 12, 16])),
                          int(rng.choice([2, 4]))) for _ in range(n)]


def test_config_validation():
    with pytest.raises(_lib.DmpcError):
        dry(max_inflight=0)
    with pytest.raises(_lib.DmpcError):
        dry(max_inflight=9)
    with pytest.raises(_lib.DmpcError):
        dry(max_batch=0)
    with pytest.raises(_lib.DmpcError):
        dry(max_nx=33)
    # one request of the largest shape must fit a share of the budget
    with pytest.raises(_lib.DmpcError):
        dry(hbm_budget=1 << 16)
    with pytest.raises(_lib.DmpcError):
        dry(staging_bytes=1 << 10)
    c = _lib.ServerConfig()
    c.max_sessions = c.max_batch = c.max_inflight = 1
    c.max_T, c.max_nx, c.max_nu = 8, 4, 2
    c.hbm_budget = 1 << 24
    c.dry_run = 1
    c.opts = _lib.make_opts(init="rollout")   # the server always warm starts
    h = ctypes.c_void_p()
    assert _lib.load().dmpc_server_create(ctypes.byref(c), ctypes.byref(h)) == _lib.DMPC_ERR_INVALID_ARG
    c.opts = _lib.make_opts()
    c.reserved = 1
    assert _lib.load().dmpc_server_create(ctypes.byref(c), ctypes.byref(h)) == _lib.DMPC_ERR_INVALID_ARG


def test_session_validation():
    srv = dry(max_T=32, max_nx=8, max_nu=2)
    try:
        rng = np.random.default_rng(1)
        with pytest.raises(_lib.DmpcError):
            srv.add_session(0, W.ltv_problem(rng, 64, 4, 2))     # T above max_T
        with pytest.raises(_lib.DmpcError):
            srv.add_session(0, W.ltv_problem(rng, 16, 8, 4))     # nu above max_nu
        with pytest.raises(_lib.DmpcError):
            srv.add_session(64, W.ltv_problem(rng, 16, 4, 2))    # session out of range
        with pytest.raises(_lib.DmpcError):
            srv.add_session(0, W.ltv_problem(rng, 16, 5, 2))     # no kernel for nx = 5
        srv.add_session(0, W.ltv_problem(rng, 16, 4, 2))
        with pytest.raises(_lib.DmpcError):
            srv.submit(1)                                         # unregistered session
        t = ctypes.c_int64()
        assert srv.lib.dmpc_server_submit(srv._h, 0, 2, None, None, ctypes.byref(t)) == \
            _lib.DMPC_ERR_INVALID_ARG
    finally:
        srv.close()


def test_admission_grouping_and_order():
    probs = uneven(24, seed=2)
    sizes = [ws_bytes(p) for p in probs]
    share = (3 * max(sizes)) // 256 * 256       # a share holds a few problems at most
    srv = dry(max_sessions=24, max_inflight=2, hbm_budget=2 * share, max_batch=8, dry_run_us=3000)
    try:
        for k, p in enumerate(probs):
            srv.add_session(k, p)
        rng = np.random.default_rng(3)
        seq = [int(s) for s in rng.integers(0, 24, size=300)]
        tickets = []
        for s in seq:
            tickets.append(srv.submit(s, backward=bool(s % 3 == 0)))
        srv.drain(timeout=120)
        for t in tickets:
            r = srv.wait(t, timeout=0)
            assert r["state"] == _lib.REQ_DONE
        st = srv.stats()
        assert st["completed"] == st["submitted"] == len(seq)
        assert st["backward_completed"] == sum(1 for s in seq if s % 3 == 0)
        assert st["failed"] == st["rejected"] == 0
        trace = srv.trace()
        assert sum(len(g["tickets"]) for g in trace) == len(seq)
        ticket_session = dict(zip(tickets, seq))
        size_of = {t: sizes[s] for t, s in ticket_session.items()}
        group_of = {}
        for g in trace:
            ts = g["tickets"]
            assert 1 <= len(ts) <= 8
            assert g["ws_bytes"] == sum(size_of[t] for t in ts) <= share
            sess = [ticket_session[t] for t in ts]
            assert len(set(sess)) == len(sess), "a session twice in one group"
            for t in ts:
                group_of[t] = g
        # one request of a session at a time, in submission order
        for s in set(seq):
            ts = [t for t in tickets if ticket_session[t] == s]
            gs = [group_of[t] for t in ts]
            for a, b in zip(gs, gs[1:]):
                assert b["id"] > a["id"]
                assert b["t_launch"] >= a["t_done"]
        # requests queued while the GPU was busy were batched together
        assert st["max_group_size"] > 1
        assert st["max_pending_seen"] > 8
    finally:
        srv.close()


def test_staging_limits_group_size():
    probs = uneven(16, seed=4)
    srv = dry(max_sessions=16, max_batch=16, max_inflight=1, staging_bytes=1 << 20,
              dry_run_us=1000)
    try:
        for k, p in enumerate(probs):
            srv.add_session(k, p)
        big = []
        for k in range(16):
            pk = srv.sessions[k]
            big.append(srv.submit(k, backward=True, dl=np.ones(pk.sol_len, np.float32)))
        srv.drain(timeout=60)
        st = srv.stats()
        assert st["completed"] == 16
        # staging bound: each group's result bytes fit 1 MiB
        for g in srv.trace():
            out = 0
            for t in g["tickets"]:
                k = big.index(t)
                pk = srv.sessions[k]
                out += 4 * (pk.sol_len + pk.data_len) + 20
            assert out <= (1 << 20)
    finally:
        srv.close()


def test_queue_limit_rejects():
    srv = dry(max_sessions=2, max_inflight=1, max_batch=1, max_pending=3, dry_run_us=200000)
    try:
        rng = np.random.default_rng(5)
        srv.add_session(0, W.ltv_problem(rng, 16, 4, 2))
        raised = 0
        for _ in range(6):
            try:
                srv.submit(0)
            except _lib.DmpcError:
                raised += 1
        assert raised >= 2
        assert srv.stats()["rejected"] == raised
        srv.drain(timeout=30)
        assert srv.stats()["completed"] == 6 - raised
    finally:
        srv.close()


def test_wait_timeout_and_unknown_ticket():
    srv = dry(max_sessions=2, max_inflight=1, dry_run_us=300000)
    try:
        rng = np.random.default_rng(6)
        p = W.ltv_problem(rng, 16, 4, 2)
        srv.add_session(0, p)
        t = srv.submit(0, x0=np.zeros(4, np.float32))
        r = srv.wait(t, timeout=0.0)
        assert r["state"] in (_lib.REQ_PENDING, _lib.REQ_RUNNING)
        # a session with work queued cannot be replaced
        with pytest.raises(_lib.DmpcError):
            srv.add_session(0, p)
        r = srv.wait(t, timeout=30.0)
        assert r["state"] == _lib.REQ_DONE
        # results are released once returned: the ticket is unknown afterwards
        assert srv.lib.dmpc_server_wait(srv._h, t, 0.0, None, None, None,
                                        ctypes.byref(ctypes.c_int32()),
                                        ctypes.byref(ctypes.c_int32())) == _lib.DMPC_ERR_INVALID_ARG
        srv.add_session(0, p)
    finally:
        srv.close()


def test_latency_statistics_and_reset():
    srv = dry(max_sessions=8, max_inflight=1, dry_run_us=5000)
    try:
        rng = np.random.default_rng(7)
        for k in range(8):
            srv.add_session(k, W.ltv_problem(rng, 16, 4, 2))
        for k in range(8):
            srv.submit(k)
        srv.drain(timeout=30)
        st = srv.stats()
        assert st["completed"] == 8
        assert 0.004 <= st["p50_latency_s"] <= st["p99_latency_s"] <= st["max_latency_s"] < 10
        assert st["throughput"] > 0
        srv.reset_stats()
        st = srv.stats()
        assert st["completed"] == 0 and st["p50_latency_s"] == 0 and srv.trace() == []
    finally:
        srv.close()


def test_destroy_with_pending_requests():
    srv = dry(max_sessions=1, max_inflight=1, dry_run_us=50000)
    rng = np.random.default_rng(8)
    srv.add_session(0, W.ltv_problem(rng, 16, 4, 2))
    for _ in range(4):
        srv.submit(0)
    t0 = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t0 < 5


def test_heavy_sessions_run_in_groups_of_their_own():
    # nx=32, T=256 problems do not fit a workgroup's LDS: their requests never
    # share a group with the others, and at most two heavy groups (4 shares /
    # 2) run at a time
    rng = np.random.default_rng(9)
    probs = [W.ltv_problem(rng, 256, 32, 8) if k % 4 == 0 else W.ltv_problem(rng, 32, 4, 2)
             for k in range(12)]
    srv = dry(max_sessions=12, max_T=256, max_nx=32, max_nu=8, max_inflight=4, max_batch=8,
              hbm_budget=1 << 30, dry_run_us=3000)
    try:
        for k, p in enumerate(probs):
            srv.add_session(k, p)
        seq = [int(s) for s in rng.integers(0, 12, size=120)]
        tickets = [srv.submit(s) for s in seq]
        srv.drain(timeout=60)
        heavy = {t: s % 4 == 0 for t, s in zip(tickets, seq)}
        trace = srv.trace()
        hg = []
        for g in trace:
            kinds = {heavy[t] for t in g["tickets"]}
            assert len(kinds) == 1, g
            if kinds == {True}:
                hg.append(g)
        assert hg and len(hg) < len(trace)
        # heavy groups in flight at every launch of one: at most 2
        for g in hg:
            live = [h for h in hg if h["t_launch"] <= g["t_launch"] < h["t_done"]]
            assert len(live) <= 2, (g, live)
        st = srv.stats()
        assert st["heavy_completed"] == sum(heavy.values())
        assert st["completed"] == len(seq)
        assert st["heavy_p50_latency_s"] > 0 and st["light_p50_latency_s"] > 0
    finally:
        srv.close()
