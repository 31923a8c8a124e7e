"""ctypes view of the C ABI in include/dmpc.h (argument marshalling only).

The shared library is the in-tree ``libdmpc.so`` built by
``paper_2510_06179_amd.build``.  Loading fails loudly when it is missing: there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdmpc.so")

# enums of dmpc.h
DMPC_OK, DMPC_ERR_INVALID_ARG, DMPC_ERR_UNSUPPORTED, DMPC_ERR_HIP, DMPC_ERR_NOMEM = range(5)
DYN_LTV, DYN_CARTPOLE, DYN_BICYCLE = 0, 1, 2
COST_DIAG, COST_SOFTPLUS = 0, 1
INIT_GIVEN, INIT_ROLLOUT = 0, 1
PROB_PCG_MAXITER, PROB_NONPD, PROB_NONFINITE, PROB_LS_FALLBACK, PROB_BWD_PCG_MAXITER = 1, 2, 4, 8, 16
PROB_KKT_UNMET, PROB_BWD_KKT_UNMET = 32, 64

DYN_KIND = {"ltv": DYN_LTV, "cartpole": DYN_CARTPOLE, "bicycle": DYN_BICYCLE}
COST_KIND = {"diag": COST_DIAG, "softplus": COST_SOFTPLUS}
INIT_KIND = {"given": INIT_GIVEN, "rollout": INIT_ROLLOUT}

EXPORTED = (
    "dmpc_default_opts", "dmpc_create", "dmpc_destroy", "dmpc_validate", "dmpc_workspace_size",
    "dmpc_plan_create", "dmpc_plan_workspace_size", "dmpc_plan_destroy", "dmpc_solve",
    "dmpc_solve_static",
    "dmpc_solve_backward", "dmpc_solve_one", "dmpc_solve_backward_one", "dmpc_status_string",
    "dmpc_version", "dmpc_workspace_offsets", "dmpc_plan_describe",
    "dmpc_server_create", "dmpc_server_destroy", "dmpc_server_add_session", "dmpc_server_submit",
    "dmpc_server_wait", "dmpc_server_drain", "dmpc_server_get_stats", "dmpc_server_reset_stats",
    "dmpc_server_trace", "dmpc_list_variants", "dmpc_set_tuning", "dmpc_get_tuning",
    "dmpc_choose_mapping", "dmpc_solve_jvp",
)
TUNING_PATH = os.path.join(PKG, "tuning_gfx950.json")
REQ_PENDING, REQ_RUNNING, REQ_DONE, REQ_FAILED = range(4)


class Problem(ctypes.Structure):
    _fields_ = [
        ("T", ctypes.c_int32), ("nx", ctypes.c_int32), ("nu", ctypes.c_int32),
        ("dyn", ctypes.c_int32), ("cost", ctypes.c_int32), ("cost_phases", ctypes.c_int32),
        ("cost_nw", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("dyn_off", ctypes.c_int64), ("cost_off", ctypes.c_int64),
        ("x0_off", ctypes.c_int64), ("sol_off", ctypes.c_int64),
    ]


PROBLEM_DTYPE = np.dtype([
    ("T", "<i4"), ("nx", "<i4"), ("nu", "<i4"), ("dyn", "<i4"), ("cost", "<i4"),
    ("cost_phases", "<i4"), ("cost_nw", "<i4"), ("reserved", "<i4"),
    ("dyn_off", "<i8"), ("cost_off", "<i8"), ("x0_off", "<i8"), ("sol_off", "<i8"),
])
assert PROBLEM_DTYPE.itemsize == ctypes.sizeof(Problem) == 64


class Opts(ctypes.Structure):
    _fields_ = [
        ("sqp_iters", ctypes.c_int32), ("pcg_max_iter", ctypes.c_int32),
        ("pcg_tol", ctypes.c_float), ("pcg_abs_tol", ctypes.c_float),
        ("n_alphas", ctypes.c_int32), ("alphas", ctypes.c_float * 8),
        ("ls_eta", ctypes.c_float), ("init", ctypes.c_int32),
        ("bwd_warm_start", ctypes.c_int32), ("bwd_pcg_max_iter", ctypes.c_int32),
        ("bwd_pcg_tol", ctypes.c_float), ("block_threads", ctypes.c_int32),
        ("refine_steps", ctypes.c_int32), ("refine_tol", ctypes.c_float),
        ("kkt_tol", ctypes.c_float), ("graph", ctypes.c_int32),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32), ("max_sessions", ctypes.c_int32),
        ("max_batch", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
        ("max_T", ctypes.c_int32), ("max_nx", ctypes.c_int32), ("max_nu", ctypes.c_int32),
        ("max_pending", ctypes.c_int32), ("batch_window_us", ctypes.c_int32),
        ("dry_run", ctypes.c_int32), ("dry_run_us", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("hbm_budget", ctypes.c_int64), ("staging_bytes", ctypes.c_int64),
        ("opts", Opts),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("rejected", ctypes.c_int64),
        ("completed", ctypes.c_int64), ("backward_completed", ctypes.c_int64),
        ("failed", ctypes.c_int64), ("groups", ctypes.c_int64),
        ("mean_group_size", ctypes.c_double), ("max_group_size", ctypes.c_int64),
        ("max_pending_seen", ctypes.c_int64), ("p50_latency_s", ctypes.c_double),
        ("p99_latency_s", ctypes.c_double), ("max_latency_s", ctypes.c_double),
        ("throughput", ctypes.c_double), ("heavy_completed", ctypes.c_int64),
        ("light_p50_latency_s", ctypes.c_double), ("light_p99_latency_s", ctypes.c_double),
        ("heavy_p50_latency_s", ctypes.c_double), ("heavy_p99_latency_s", ctypes.c_double),
    ]


class DmpcError(RuntimeError):
    pass


_lib = None


def load():
    """Load libdmpc.so (once).  Raises DmpcError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise DmpcError(f"{LIB_PATH} is missing: run `python -m paper_2510_06179_amd.build`")
    # PyTorch ships its own HIP runtime; loading it first makes the library
    # bind to that one instead of bringing a second runtime into the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    sig = {
        "dmpc_default_opts": (None, [P(Opts)]),
        "dmpc_create": (i32, [P(vp), ctypes.c_int]),
        "dmpc_destroy": (i32, [vp]),
        "dmpc_validate": (i32, [vp, i32, i64, i64, P(Opts), P(i32)]),
        "dmpc_workspace_size": (i32, [vp, i32, P(Opts), P(ctypes.c_size_t)]),
        "dmpc_plan_create": (i32, [vp, vp, i32, i64, i64, P(Opts), P(vp)]),
        "dmpc_plan_workspace_size": (i32, [vp, P(ctypes.c_size_t)]),
        "dmpc_plan_destroy": (i32, [vp]),
        "dmpc_solve": (i32, [vp, vp, vp, vp, vp, vp, vp]),
        "dmpc_solve_static": (i32, [vp, vp, vp, vp, vp, vp]),
        "dmpc_solve_backward": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "dmpc_solve_jvp": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "dmpc_solve_one": (i32, [vp, i32, vp, vp, vp, vp, vp, vp]),
        "dmpc_solve_backward_one": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]),
        "dmpc_status_string": (ctypes.c_char_p, [i32]),
        "dmpc_version": (i32, []),
        "dmpc_workspace_offsets": (i32, [vp, i32, P(i64)]),
        "dmpc_plan_describe": (i32, [vp, ctypes.c_char_p, ctypes.c_size_t]),
        "dmpc_server_create": (i32, [P(ServerConfig), P(vp)]),
        "dmpc_server_destroy": (i32, [vp]),
        "dmpc_server_add_session": (i32, [vp, i32, P(Problem), vp, i64, vp, vp]),
        "dmpc_server_submit": (i32, [vp, i32, i32, vp, vp, P(i64)]),
        "dmpc_server_wait": (i32, [vp, i64, ctypes.c_double, vp, vp, vp, P(i32), P(i32)]),
        "dmpc_server_drain": (i32, [vp, ctypes.c_double]),
        "dmpc_server_get_stats": (i32, [vp, P(ServerStats)]),
        "dmpc_server_reset_stats": (i32, [vp]),
        "dmpc_server_trace": (i32, [vp, ctypes.c_char_p, ctypes.c_size_t]),
        "dmpc_list_variants": (i32, [vp, i32]),
        "dmpc_set_tuning": (i32, [vp, i32]),
        "dmpc_get_tuning": (i32, [vp, i32]),
        "dmpc_choose_mapping": (i32, [P(Problem), P(Opts), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    if os.path.exists(TUNING_PATH) and not os.environ.get("DMPC_NO_TUNING"):
        install_tuning(load_tuning(TUNING_PATH))
    return lib


def load_tuning(path):
    """Rows (nx, T_min, T_max, slots, launch_bound, register_rows,
    block_threads) of a tuning file written by paper_2510_06179_amd.tune."""
    import json
    with open(path) as f:
        return [tuple(int(v) for v in r) for r in json.load(f)["rows"]]


def install_tuning(rows):
    arr = np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1, 7))
    check(load().dmpc_set_tuning(arr.ctypes.data if len(arr) else None, len(arr)),
          "dmpc_set_tuning")


def variants():
    """(nx, slots, launch_bound, register_rows) of every instantiated kernel."""
    lib = load()
    n = lib.dmpc_list_variants(None, 0)
    out = np.zeros((n, 4), np.int32)
    lib.dmpc_list_variants(out.ctypes.data, n)
    return [tuple(int(v) for v in r) for r in out]


def check(rc, what=""):
    if rc != DMPC_OK:
        msg = load().dmpc_status_string(rc).decode()
        raise DmpcError(f"{what}: {msg} (code {rc})")


def make_opts(sqp_iters=1, pcg_tol=1e-6, pcg_abs_tol=0.0, pcg_max_iter=0,
              alphas=(1.0, 0.7, 0.3, 0.1, 0.01), ls_eta=0.4, init="given",
              bwd_warm_start=False, bwd_pcg_tol=None, bwd_pcg_max_iter=0, block_threads=0,
              refine_steps=3, refine_tol=1e-1, kkt_tol=1e-6, graph=True):
    o = Opts()
    load().dmpc_default_opts(ctypes.byref(o))
    o.sqp_iters = int(sqp_iters)
    o.pcg_tol = float(pcg_tol)
    o.pcg_abs_tol = float(pcg_abs_tol)
    o.pcg_max_iter = int(pcg_max_iter)
    o.n_alphas = len(alphas)
    for i in range(8):
        o.alphas[i] = float(alphas[i]) if i < len(alphas) else 0.0
    o.ls_eta = float(ls_eta)
    o.init = INIT_KIND[init] if isinstance(init, str) else int(init)
    o.bwd_warm_start = int(bool(bwd_warm_start))
    o.bwd_pcg_tol = float(pcg_tol if bwd_pcg_tol is None else bwd_pcg_tol)
    o.bwd_pcg_max_iter = int(bwd_pcg_max_iter)
    o.block_threads = int(block_threads)
    o.refine_steps = int(refine_steps)
    o.refine_tol = float(refine_tol)
    o.kkt_tol = float(kkt_tol)
    o.graph = int(bool(graph))
    return o
