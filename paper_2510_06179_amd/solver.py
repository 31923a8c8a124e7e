"""Python binding of the C ABI (argument marshalling only).

PyTorch supplies device memory and the stream; every step of the solver runs
in the HIP kernels of libdmpc.so.  Names follow the C ABI:

    s = BatchSolver(problems_or_packed, sqp_iters=10, pcg_tol=1e-6, ...)
    sol = s.solve(data)                  # dmpc_solve
    adj, grad = s.solve_backward(dl)     # dmpc_solve_backward
    s.solve_one(i, ...), s.solve_backward_one(i, ...)   # one problem per launch
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .batch import Packed, pack


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class BatchSolver:
    """A plan over a fixed batch of problems plus its device buffers."""

    def __init__(self, problems, device=0, **opts):
        if not torch.cuda.is_available():
            raise _lib.DmpcError("BatchSolver needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = _lib.load()
        self.packed = problems if isinstance(problems, Packed) else pack(problems)
        if "init" not in opts and self.packed.problems:
            opts["init"] = self.packed.problems[0].get("init", "given")
        self.opts = _lib.make_opts(**opts)
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        _lib.check(self.lib.dmpc_create(ctypes.byref(h), device), "dmpc_create")
        self.handle = h
        plan = ctypes.c_void_p()
        descs = np.ascontiguousarray(self.packed.descs)
        _lib.check(self.lib.dmpc_plan_create(
            h, descs.ctypes.data_as(ctypes.c_void_p), len(descs), self.packed.data_len,
            self.packed.sol_len, ctypes.byref(self.opts), ctypes.byref(plan)), "dmpc_plan_create")
        self.plan = plan
        nb = ctypes.c_size_t()
        _lib.check(self.lib.dmpc_plan_workspace_size(plan, ctypes.byref(nb)), "workspace size")
        dev = self.device
        n = self.packed.count
        self.workspace = torch.empty(max(1, nb.value // 4), dtype=torch.float32, device=dev)
        self.status = torch.zeros(max(1, n), dtype=torch.int32, device=dev)
        self.info = torch.zeros((max(1, n), 4), dtype=torch.int32, device=dev)
        self.data = torch.from_numpy(self.packed.data).to(dev)
        self.sol0 = torch.from_numpy(self.packed.sol0).to(dev)
        self.sol = self.sol0.clone()

    # ---- forward
    def solve(self, data=None, sol=None, stream=None):
        """dmpc_solve.  ``sol`` (default: a copy of the packed initial guess) is
        overwritten with the solution and returned."""
        data = self.data if data is None else data
        if sol is None:
            self.sol.copy_(self.sol0)
            sol = self.sol
        _lib.check(self.lib.dmpc_solve(self.plan, _ptr(data), _ptr(sol), _ptr(self.workspace),
                                       _ptr(self.status), _ptr(self.info), _stream(stream)),
                   "dmpc_solve")
        return sol

    def solve_static(self, data=None, sol=None, status=None, info=None, stream=None):
        """dmpc_solve_static: the forward pass with the workspace in the
        library's static device buffer (no allocation in the call)."""
        data = self.data if data is None else data
        sol = self.sol if sol is None else sol
        status = self.status if status is None else status
        info = self.info if info is None else info
        _lib.check(self.lib.dmpc_solve_static(self.plan, _ptr(data), _ptr(sol), _ptr(status),
                                              _ptr(info), _stream(stream)), "dmpc_solve_static")
        return sol

    def solve_one(self, index, data=None, sol=None, stream=None):
        data = self.data if data is None else data
        sol = self.sol if sol is None else sol
        _lib.check(self.lib.dmpc_solve_one(self.plan, int(index), _ptr(data), _ptr(sol),
                                           _ptr(self.workspace), _ptr(self.status),
                                           _ptr(self.info), _stream(stream)), "dmpc_solve_one")
        return sol

    # ---- backward
    def solve_backward(self, dl_dsol, data=None, adj=None, grad=None, stream=None):
        """dmpc_solve_backward.  Returns (adj, grad): adjoint arena (x~, u~,
        lambda~) and the gradient laid out like the data arena."""
        data = self.data if data is None else data
        if adj is None:
            adj = torch.zeros_like(self.sol)
        if grad is None:
            grad = torch.zeros_like(data)
        dl = dl_dsol.contiguous()
        _lib.check(self.lib.dmpc_solve_backward(self.plan, _ptr(data), _ptr(dl), _ptr(adj),
                                                _ptr(grad), _ptr(self.workspace),
                                                _ptr(self.status), _ptr(self.info),
                                                _stream(stream)), "dmpc_solve_backward")
        return adj, grad

    def solve_jvp(self, tangent, data=None, out=None, rhs=None, grad=None, stream=None):
        """dmpc_solve_jvp: derivative of the last QP's (x, u, lambda) along
        ``tangent`` (laid out like the data arena).  Returns the arena of
        (dx, du, dlambda), laid out like the solution arena."""
        data = self.data if data is None else data
        out = torch.zeros_like(self.sol) if out is None else out
        rhs = torch.empty_like(self.sol) if rhs is None else rhs
        grad = torch.empty_like(data) if grad is None else grad
        tan = tangent.contiguous()
        _lib.check(self.lib.dmpc_solve_jvp(self.plan, _ptr(data), _ptr(tan), _ptr(rhs),
                                           _ptr(out), _ptr(grad), _ptr(self.workspace),
                                           _ptr(self.status), _ptr(self.info),
                                           _stream(stream)), "dmpc_solve_jvp")
        return out

    def solve_backward_one(self, index, dl_dsol, data=None, adj=None, grad=None, stream=None):
        data = self.data if data is None else data
        _lib.check(self.lib.dmpc_solve_backward_one(
            self.plan, int(index), _ptr(data), _ptr(dl_dsol), _ptr(adj), _ptr(grad),
            _ptr(self.workspace), _ptr(self.status), _ptr(self.info), _stream(stream)),
            "dmpc_solve_backward_one")
        return adj, grad

    def saved_qp(self, index):
        """Views into the workspace of what the forward pass kept for problem
        ``index``: dict(xlin, ulin, xp, up, lam, Qd, Rd) (device tensors)."""
        out = (ctypes.c_int64 * 7)()
        _lib.check(self.lib.dmpc_workspace_offsets(self.plan, int(index), out), "offsets")
        d = self.packed.descs[index]
        T, nx, nu = int(d["T"]), int(d["nx"]), int(d["nu"])
        N = T + 1
        ws = self.workspace
        shp = [(N, nx), (T, nu), (N, nx), (T, nu), (N, nx), (N, nx), (T, nu)]
        keys = ["xlin", "ulin", "xp", "up", "lam", "Qd", "Rd"]
        return {k: ws[o:o + s[0] * s[1]].view(*s) for k, o, s in zip(keys, out, shp)}

    def describe(self):
        """Launch groups of the plan (list of dicts)."""
        import json
        buf = ctypes.create_string_buffer(8192)
        _lib.check(self.lib.dmpc_plan_describe(self.plan, buf, len(buf)), "describe")
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "plan", None):
            self.lib.dmpc_plan_destroy(self.plan)
            self.plan = None
        if getattr(self, "handle", None):
            self.lib.dmpc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DMPCFunction(torch.autograd.Function):
    """Differentiable solve: data arena -> solution arena (x, u, lambda).

    The backward pass is dmpc_solve_backward (Alg. backward); the workspace of
    ``solver`` must not be reused by another solve between the two passes."""

    @staticmethod
    def forward(ctx, data, solver):
        sol = solver.solve(data, sol=solver.sol0.clone())
        ctx.solver = solver
        ctx.save_for_backward(data)
        return sol

    @staticmethod
    def backward(ctx, gsol):
        (data,) = ctx.saved_tensors
        _, grad = ctx.solver.solve_backward(gsol, data=data)
        return grad, None


def dmpc(data, solver):
    """Functional form of DMPCFunction."""
    return DMPCFunction.apply(data, solver)
