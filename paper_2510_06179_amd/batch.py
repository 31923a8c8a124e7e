"""Packing of problem dicts into the flat arenas of the C ABI, and unpacking of
results (argument marshalling only; no solver arithmetic).

Per problem the data arena holds [dynamics block | cost block | x_s] and the
solution arena [x (T+1)*nx | u T*nu | lambda (T+1)*nx]; the gradient arena of
the backward pass mirrors the data arena and the adjoint/cotangent arenas
mirror the solution arena (see include/dmpc.h).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from ._lib import COST_KIND, DYN_KIND, PROBLEM_DTYPE


@dataclass
class Packed:
    descs: np.ndarray       # PROBLEM_DTYPE [count]
    data: np.ndarray        # float32 [data_len]
    sol0: np.ndarray        # float32 [sol_len] initial guess
    problems: list          # the source dicts (shapes, kinds)

    @property
    def count(self):
        return len(self.descs)

    @property
    def data_len(self):
        return int(self.data.shape[0])

    @property
    def sol_len(self):
        return int(self.sol0.shape[0])


def _dyn_block(p):
    if p["dyn"] == "ltv":
        return np.concatenate([np.ravel(p["A"]), np.ravel(p["B"]), np.ravel(p["c"])])
    return np.ravel(p["params"])


def _cost_block(p):
    if p["cost"] == "diag":
        return np.concatenate([np.ravel(p["Qd"]), np.ravel(p["q"]), np.ravel(p["Rd"]), np.ravel(p["r"])])
    return np.concatenate([np.ravel(p["theta"]), np.ravel(p["wscale"]), np.ravel(p["wfix"]),
                           np.ravel(p["xref"])])


def pack(problems, align=4):
    n = len(problems)
    descs = np.zeros(n, dtype=PROBLEM_DTYPE)
    data_parts, sol_parts = [], []
    off = soff = 0

    def put(arr):
        nonlocal off
        arr = np.asarray(arr, dtype=np.float32).ravel()
        pad = (-arr.shape[0]) % align
        o = off
        data_parts.append(arr)
        if pad:
            data_parts.append(np.zeros(pad, np.float32))
        off += arr.shape[0] + pad
        return o

    for k, p in enumerate(problems):
        T, nx, nu = int(p["T"]), int(p["nx"]), int(p["nu"])
        d = descs[k]
        d["T"], d["nx"], d["nu"] = T, nx, nu
        d["dyn"] = DYN_KIND[p["dyn"]]
        d["cost"] = COST_KIND[p["cost"]]
        if p["cost"] == "softplus":
            d["cost_phases"], d["cost_nw"] = int(p["phases"]), int(p["nw"])
        d["dyn_off"] = put(_dyn_block(p))
        d["cost_off"] = put(_cost_block(p))
        d["x0_off"] = put(p["x0"])
        s = np.concatenate([np.ravel(p["xbar"]), np.ravel(p["ubar"]), np.ravel(p["lam"])])
        d["sol_off"] = soff
        sol_parts.append(s.astype(np.float32))
        soff += s.shape[0]
    data = np.concatenate(data_parts) if data_parts else np.zeros(0, np.float32)
    sol0 = np.concatenate(sol_parts) if sol_parts else np.zeros(0, np.float32)
    return Packed(descs, data, sol0, list(problems))


def split_sol(packed, sol, k):
    """(x [N,nx], u [T,nu], lam [N,nx]) of problem k from a solution-shaped arena."""
    d = packed.descs[k]
    T, nx, nu, o = int(d["T"]), int(d["nx"]), int(d["nu"]), int(d["sol_off"])
    N = T + 1
    x = sol[o:o + N * nx].reshape(N, nx)
    u = sol[o + N * nx:o + N * nx + T * nu].reshape(T, nu)
    lam = sol[o + N * nx + T * nu:o + 2 * N * nx + T * nu].reshape(N, nx)
    return x, u, lam


def sol_like(packed, parts):
    """Assemble a solution-shaped arena from per-problem (x, u, lam) triples."""
    out = np.zeros(packed.sol_len, np.float32)
    for k, (x, u, lam) in enumerate(parts):
        d = packed.descs[k]
        o = int(d["sol_off"])
        s = np.concatenate([np.ravel(x), np.ravel(u), np.ravel(lam)]).astype(np.float32)
        out[o:o + s.shape[0]] = s
    return out


def split_grad(packed, grad, k):
    """Gradient arena of problem k as a dict keyed like the problem's inputs."""
    d = packed.descs[k]
    p = packed.problems[k]
    T, nx, nu = int(d["T"]), int(d["nx"]), int(d["nu"])
    N = T + 1
    out = {}
    o = int(d["dyn_off"])
    if p["dyn"] == "ltv":
        out["A"] = grad[o:o + T * nx * nx].reshape(T, nx, nx)
        o += T * nx * nx
        out["B"] = grad[o:o + T * nx * nu].reshape(T, nx, nu)
        o += T * nx * nu
        out["c"] = grad[o:o + T * nx].reshape(T, nx)
    else:
        out["params"] = grad[o:o + np.size(p["params"])]
    o = int(d["cost_off"])
    if p["cost"] == "diag":
        for key, n_, shp in (("Qd", N * nx, (N, nx)), ("q", N * nx, (N, nx)),
                             ("Rd", T * nu, (T, nu)), ("r", T * nu, (T, nu))):
            out[key] = grad[o:o + n_].reshape(shp)
            o += n_
    else:
        for key in ("theta", "wscale", "wfix", "xref"):
            n_ = np.size(p[key])
            out[key] = grad[o:o + n_].reshape(np.shape(p[key]))
            o += n_
    o = int(d["x0_off"])
    out["x0"] = grad[o:o + nx]
    return out
