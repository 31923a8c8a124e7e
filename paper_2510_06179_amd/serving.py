"""Python binding of the continuous-batching server (dmpc_server_* in
include/dmpc.h): argument marshalling only.  The queue, admission, batching,
device stores and every solve run inside libdmpc.so.

    srv = Server(max_sessions=4096, max_T=128, max_nx=16, max_nu=4)
    srv.add_session(0, problem_dict)              # keeps data + warm start on the device
    t = srv.submit(0, backward=True, x0=x_s)      # returns at once
    r = srv.wait(t)                               # {"sol": (x, u, lam), "grad": {...}, ...}
"""
from __future__ import annotations

import ctypes
import json

import numpy as np

from . import _lib, batch


class Server:
    def __init__(self, max_sessions, max_T, max_nx, max_nu, device=0, max_batch=1024,
                 max_inflight=2, hbm_budget=32 << 30, staging_bytes=0, max_pending=0,
                 batch_window_us=0, dry_run=False, dry_run_us=0, **opts):
        self.lib = _lib.load()
        opts = dict(opts)
        opts["init"] = "given"
        c = _lib.ServerConfig()
        c.device = int(device)
        c.max_sessions = int(max_sessions)
        c.max_batch = int(max_batch)
        c.max_inflight = int(max_inflight)
        c.max_T, c.max_nx, c.max_nu = int(max_T), int(max_nx), int(max_nu)
        c.max_pending = int(max_pending)
        c.batch_window_us = int(batch_window_us)
        c.dry_run = int(bool(dry_run))
        c.dry_run_us = int(dry_run_us)
        c.hbm_budget = int(hbm_budget)
        c.staging_bytes = int(staging_bytes)
        c.opts = _lib.make_opts(**opts)
        self.config = c
        self._h = ctypes.c_void_p()
        _lib.check(self.lib.dmpc_server_create(ctypes.byref(c), ctypes.byref(self._h)),
                   "dmpc_server_create")
        self.sessions = {}
        self._ticket_session = {}
        self._ticket = ctypes.c_int64()

    # -- sessions ---------------------------------------------------------
    def add_session(self, session, problem, sol0=None, dl=None):
        """Register `problem` (a problem dict of the workload generators) as
        session `session`.  sol0 / dl: optional (x, u, lam) triples."""
        pk = batch.pack([problem])
        d = pk.descs[0]
        desc = _lib.Problem(*[d[name].item() for name in _lib.PROBLEM_DTYPE.names])
        data = np.ascontiguousarray(pk.data, np.float32)
        s0 = pk.sol0 if sol0 is None else batch.sol_like(pk, [sol0])
        s0 = np.ascontiguousarray(s0, np.float32)
        dlv = None if dl is None else np.ascontiguousarray(batch.sol_like(pk, [dl]), np.float32)
        rc = self.lib.dmpc_server_add_session(
            self._h, int(session), ctypes.byref(desc), data.ctypes.data, int(data.shape[0]),
            s0.ctypes.data, None if dlv is None else dlv.ctypes.data)
        _lib.check(rc, "dmpc_server_add_session")
        self.sessions[int(session)] = pk
        return pk

    # -- requests ---------------------------------------------------------
    def submit(self, session, backward=False, x0=None, dl=None):
        """Queue a request; returns its ticket.  x0: float32 [nx] or None;
        dl: float32 cotangent laid out like the session's solution block."""
        x0p = None if x0 is None else np.ascontiguousarray(x0, np.float32).ctypes.data
        dlp = None if dl is None else np.ascontiguousarray(dl, np.float32).ctypes.data
        rc = self.lib.dmpc_server_submit(self._h, int(session), int(bool(backward)), x0p, dlp,
                                         ctypes.byref(self._ticket))
        _lib.check(rc, "dmpc_server_submit")
        t = self._ticket.value
        self._ticket_session[t] = int(session)
        return t

    def wait(self, ticket, timeout=-1.0, outputs=True):
        """Wait for a request.  Returns {"state", "status", "info", "sol",
        "grad"} (sol/grad are flat float32 blocks, None if not requested or
        not available)."""
        pk = self.sessions[self._ticket_session[ticket]]
        sol = grad = None
        info = np.zeros(4, np.int32)
        if outputs:
            sol = np.zeros(pk.sol_len, np.float32)
            grad = np.zeros(pk.data_len, np.float32)
        state, status = ctypes.c_int32(), ctypes.c_int32()
        rc = self.lib.dmpc_server_wait(
            self._h, int(ticket), float(timeout), None if sol is None else sol.ctypes.data,
            None if grad is None else grad.ctypes.data, info.ctypes.data, ctypes.byref(state),
            ctypes.byref(status))
        _lib.check(rc, "dmpc_server_wait")
        if state.value in (_lib.REQ_DONE, _lib.REQ_FAILED):
            self._ticket_session.pop(ticket, None)
        return {"state": state.value, "status": status.value, "info": info, "sol": sol,
                "grad": grad}

    def drain(self, timeout=-1.0):
        _lib.check(self.lib.dmpc_server_drain(self._h, float(timeout)), "dmpc_server_drain")

    # -- statistics -------------------------------------------------------
    def stats(self):
        st = _lib.ServerStats()
        _lib.check(self.lib.dmpc_server_get_stats(self._h, ctypes.byref(st)), "dmpc_server_get_stats")
        return {name: getattr(st, name) for name, _ in st._fields_}

    def reset_stats(self):
        _lib.check(self.lib.dmpc_server_reset_stats(self._h), "dmpc_server_reset_stats")

    def trace(self, size=1 << 22):
        buf = ctypes.create_string_buffer(size)
        _lib.check(self.lib.dmpc_server_trace(self._h, buf, size), "dmpc_server_trace")
        return json.loads(buf.value.decode())

    def close(self):
        if self._h:
            self.lib.dmpc_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
