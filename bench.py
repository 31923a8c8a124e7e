"""Throughput benchmark of the batched differentiable-MPC hot path on one GPU.

One step = one forward solve (Alg. sqp, 8 SQP iterations with the line
search, PCG inside) plus one backward solve (Alg. backward: adjoint PCG +
VJP) of the uneven batch: 4096 time-varying linear OCPs with T uniform in
{16, 32, 64, 128}, nx in {4, 8, 12, 16}, nu in {2, 4}, all in one call, inputs
resident in HBM.  Beside it: the accuracy of a stratified sample against the
FP64 oracle, the plain one-problem-per-launch GPU form, the FP64 oracle on the
host cores, the other batch workloads (cart-pole SQP, bicycle
differentiation, JVP) and the continuous-batching server under Poisson
arrivals (p50/p99 latency).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu] [--plain-sample 2]
                    [--serve-seconds 60] [--no-extra] [--traffic-reference]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2510_06179_amd import workloads as W  # noqa: E402

METRIC = "OCP solves/s fwd+bwd @1e-5 KKT resid vs plain GPU; p50/p99 serve latency"
B, SQP, PCG_TOL = 4096, 8, 1e-6
KKT_TOL, REL_TOL = 1e-5, 1e-4
FP32_VECTOR_PEAK = 157.3e12   # MI355X published FP32 vector peak (FLOP/s)
HBM_PEAK = 8.0e12             # MI355X HBM3E (B/s)
CPU_SHARE = 16                # host cores per GPU on the measurement box


def headline_batch():
    return W.ltv_uneven_batch(0, batch=B)


def shape_classes(probs):
    """(T, nx, nu) -> problem indices, in batch order."""
    cls = {}
    for k, p in enumerate(probs):
        cls.setdefault((p["T"], p["nx"], p["nu"]), []).append(k)
    return cls


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, CPU_SHARE))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


# ---------------------------------------------------------------------------
# CPU-baseline leg: the FP64 oracle on the host cores (timed before the GPU is
# touched), and the accuracy of the GPU's answers on the same sample
# ---------------------------------------------------------------------------
def _oracle_fwd_bwd(k):
    from threadpoolctl import threadpool_limits

    import oracle
    probs = _ORACLE_PROBS
    p, c = probs[k], _ORACLE_COTS[k]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        x, u, lam, hist = oracle.sqp.sqp(p, SQP)
        h = hist[-1]   # VJP of the last QP's solution map at its linearisation point
        g, _ = oracle.backward.vjp(p, h["xbar"], h["ubar"], h["qp"], h["sol"], c["gx"], c["gu"])
        dt = time.perf_counter() - t0
    return k, dt, x, u, lam, h["xbar"], h["ubar"], g


_ORACLE_PROBS = None
_ORACLE_COTS = None


class CpuBaseline:
    """The oracle on a stratified sample of the headline batch: one problem of
    every (T, nx, nu) class, each in its own worker process with one thread.
    The batch rate is extrapolated per class (the class's mean single-core
    time times its count, spread over the cores).  check() then holds the
    GPU's answers for the same problems against the oracle's."""

    def __init__(self, probs, cots, per_class=1):
        global _ORACLE_PROBS, _ORACLE_COTS
        _ORACLE_PROBS, _ORACLE_COTS = probs, cots
        self.probs = probs
        self.cls = shape_classes(probs)
        self.sample = [k for key in sorted(self.cls) for k in self.cls[key][:per_class]]
        self.cores = host_cores()

    def run(self):
        ctx = mp.get_context("fork")
        t0 = time.perf_counter()
        with ctx.Pool(self.cores) as pool:
            # biggest first, so that the pool's wall time is not set by a late big problem
            order = sorted(self.sample, key=lambda k: -self.probs[k]["T"] * self.probs[k]["nx"] ** 3)
            res = list(pool.imap_unordered(_oracle_fwd_bwd, order, chunksize=1))
        wall = time.perf_counter() - t0
        self.results = {r[0]: r for r in res}
        per_cls = {}
        for key, ks in self.cls.items():
            ts = [self.results[k][1] for k in ks if k in self.results]
            per_cls[key] = float(np.mean(ts))
        core_s = sum(len(ks) * per_cls[key] for key, ks in self.cls.items())
        est = core_s / self.cores
        return {"value": len(self.probs) / est, "unit": "solves/s", "cores": self.cores,
                "kind": "oracle",
                "sample": f"{len(self.sample)} problems, one of each (T, nx, nu) class of the "
                          f"{len(self.probs)}-problem uneven batch, fwd ({SQP} SQP iters, dense "
                          f"LU) + IFT VJP, FP64, {self.cores} worker processes x 1 thread on "
                          f"{cpu_model()}; {wall:.1f} s wall; batch time extrapolated per class "
                          f"from single-core times ({core_s:.0f} core-s / {self.cores} cores)"}

    def check(self, solver, sol, grad):
        """Accuracy of the GPU's answers on the sample: relative KKT residual of
        the last QP's solution (the QP the oracle forms at the GPU's last
        linearisation point) and relative errors of x, u, lambda and of the
        gradients against the oracle's."""
        import oracle
        from paper_2510_06179_amd import batch
        kkts, ex, el, eg = [], [], [], []
        for k in self.sample:
            p = self.probs[k]
            _, _, xo, uo, lo, _, _, go = self.results[k]
            sq = {n: v.cpu().numpy().astype(np.float64) for n, v in solver.saved_qp(k).items()}
            qpd = oracle.qp.qp_data(p, sq["xlin"], sq["ulin"])
            kkts.append(oracle.qp.kkt_residual_blocks(qpd, p["x0"], sq["xp"], sq["up"], sq["lam"]))
            x, u, lam = batch.split_sol(solver.packed, sol, k)
            z = np.concatenate([np.ravel(x), np.ravel(u)])
            zo = np.concatenate([np.ravel(xo), np.ravel(uo)])
            ex.append(_rel(z, zo))
            el.append(_rel(lam, lo))
            g = batch.split_grad(solver.packed, grad, k)
            eg.append(max(_rel(g[key], go[key]) for key in go))
        kkts = np.array(kkts)
        return {"sample": len(self.sample), "kkt_max": float(kkts.max()),
                "kkt_frac_le_1e-5": float(np.mean(kkts <= KKT_TOL)),
                "rel_err_z_max": float(max(ex)), "rel_err_lambda_max": float(max(el)),
                "rel_err_grad_max": float(max(eg)),
                "rel_err_frac_le_1e-4": float(np.mean((np.array(ex) <= REL_TOL)
                                                      & (np.array(el) <= REL_TOL)
                                                      & (np.array(eg) <= REL_TOL)))}


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


# ---------------------------------------------------------------------------
# Algorithmic work (the method's own counts, not the dense O(K^3) it avoids)
# ---------------------------------------------------------------------------
def pcg_flops(N, n):
    """One PCG iteration on one problem: two block-tridiagonal row products
    (3n FMAs per row each) over N*n rows plus five vector updates/dot products."""
    return 12 * N * n * n + 10 * N * n


def qp_flops(T, n, m):
    """Forming one QP's Schur system: assembly T(2n^3 + 2n^2 m), the
    preconditioner (Cholesky-equivalent inversion N n^3/3 plus the explicit
    off-diagonal blocks 4 T n^3), and the recovery of z, T(2n^2 + 2nm)."""
    N = T + 1
    return T * (2 * n ** 3 + 2 * n * n * m) + N * n ** 3 / 3 + 4 * T * n ** 3 + T * (2 * n * n + 2 * n * m)


def ltv_bytes(T, n, m):
    """Bytes a problem's QP data occupies in HBM (float32): A_t, B_t, c_t,
    the diagonal cost data and x_s in, x, u, lambda out."""
    N = T + 1
    return 4 * (T * (n * n + n * m + n) + 2 * N * n + 2 * T * m + n) + 4 * (2 * N * n + T * m)


KERNEL_SOURCES = ("csrc/dmpc_device.h", "csrc/dmpc_internal.h", "csrc/dmpc_launch.hip",
                  "csrc/dmpc_k4.hip", "csrc/dmpc_k8.hip", "csrc/dmpc_k12.hip", "csrc/dmpc_k16.hip",
                  "csrc/dmpc_host.cpp", "tuning_gfx950.json")   # (the mapping decides the kernels)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "forward_pass_uneven_ltv_traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_06179_amd", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per forward pass from the committed counter summary, or None
    when it is missing or was taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_pass")


def traffic_reference(mib=512, reps=8):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"traffic_reference_copy_bytes": n * 4, "launches": reps}), flush=True)


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------
def timed_fwd_bwd(s, dl, steps, warmup):
    """Times `steps` forward + backward solves of the plan; returns (per-step
    wall ms, forward ms per step, backward ms per step, sol, grad).  The
    events are recorded on the caller's stream, which the plan's launch
    groups fork from and join back into."""
    import torch
    sol = s.sol0.clone()
    adj = torch.zeros_like(sol)
    grad = torch.zeros_like(s.data)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]

    def step(e=None):
        sol.copy_(s.sol0)
        if e:
            e[0].record()
        s.solve(sol=sol)
        if e:
            e[1].record()
        s.solve_backward(dl, adj=adj, grad=grad)
        if e:
            e[2].record()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(ev[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd = [e[0].elapsed_time(e[1]) for e in ev]
    bwd = [e[1].elapsed_time(e[2]) for e in ev]
    return 1000.0 * wall / steps, fwd, bwd, sol, grad


def dl_arena(s, cots):
    import torch
    from paper_2510_06179_amd import batch
    return torch.from_numpy(batch.sol_like(s.packed, [(c["gx"], c["gu"], c["glam"])
                                                      for c in cots])).to(s.device)


def solver_stats(s):
    from paper_2510_06179_amd import _lib
    status = s.status.cpu().numpy()
    info = s.info.cpu().numpy()
    return {"fwd_pcg_iters_mean": float(info[:, 0].mean()),
            "bwd_pcg_iters_mean": float(info[:, 1].mean()),
            # per-problem PCG iterations per solve: p10, p50, p90, p99, max
            "fwd_pcg_iters_pct": [float(v) for v in np.percentile(info[:, 0], [10, 50, 90, 99, 100])],
            "bwd_pcg_iters_pct": [float(v) for v in np.percentile(info[:, 1], [10, 50, 90, 99, 100])],
            "nonpd_or_nonfinite": int(np.count_nonzero(status & (_lib.PROB_NONPD | _lib.PROB_NONFINITE))),
            "fwd_pcg_capped": int(np.count_nonzero(status & _lib.PROB_PCG_MAXITER)),
            "bwd_pcg_capped": int(np.count_nonzero(status & _lib.PROB_BWD_PCG_MAXITER)),
            "ls_fallback_last_iter": int(np.count_nonzero(status & _lib.PROB_LS_FALLBACK)),
            # last QP / adjoint solve ended above the internal KKT target (1e-6)
            "fwd_kkt_target_unmet": int(np.count_nonzero(status & _lib.PROB_KKT_UNMET)),
            "bwd_kkt_target_unmet": int(np.count_nonzero(status & _lib.PROB_BWD_KKT_UNMET))}


def plain_gpu(s, probs, dl, per_class, batched_value):
    """The plain one-problem-per-launch form (dmpc_solve_one +
    dmpc_solve_backward_one, serial on one stream) on a stratified sample,
    extrapolated to the batch per (T, nx, nu) class."""
    import torch
    cls = shape_classes(probs)
    sol = s.sol0.clone()
    adj = torch.zeros_like(sol)
    grad = torch.zeros_like(s.data)
    for k in (0, 1):
        s.solve_one(k, sol=sol)
        s.solve_backward_one(k, dl, adj=adj, grad=grad)
    torch.cuda.synchronize()
    total = 0.0
    n = 0
    for key, ks in cls.items():
        pick = ks[:per_class]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in pick:
            s.solve_one(k, sol=sol)
            s.solve_backward_one(k, dl, adj=adj, grad=grad)
        torch.cuda.synchronize()
        total += len(ks) * (time.perf_counter() - t0) / len(pick)
        n += len(pick)
    value = len(probs) / total
    return {"value": value, "unit": "solves/s", "sample": n,
            "sample_kind": f"{per_class} per (T, nx, nu) class, extrapolated per class",
            "speedup_batched": batched_value / value}


def cartpole_leg(steps=10, warmup=2):
    """The cart-pole SQP batch: 1024 OCPs, nx=4, nu=1, T=50, 10 SQP
    iterations, fwd + bwd; with the fused forward kernel's FLOP rate."""
    from paper_2510_06179_amd.solver import BatchSolver
    probs = W.cartpole_batch(0, batch=1024)
    s = BatchSolver(probs, sqp_iters=10, pcg_tol=PCG_TOL, bwd_pcg_tol=PCG_TOL)
    dl = dl_arena(s, W.loss_cotangents(probs, seed=0))
    ms, fwd, bwd, _, _ = timed_fwd_bwd(s, dl, steps, warmup)
    info = s.info.cpu().numpy()
    flops = float(info[:, 0].sum()) * pcg_flops(51, 4) + 1024 * 10 * qp_flops(50, 4, 1)
    out = {"solves_per_s": 1024 / (ms / 1e3), "ms_per_step": ms, "fwd_ms": float(np.mean(fwd)),
           "bwd_ms": float(np.mean(bwd)), "sqp_iters": 10,
           "fwd_kernel_tflops": flops / (np.mean(fwd) / 1e3) / 1e12,
           "fwd_kernel_frac_fp32_peak": flops / (np.mean(fwd) / 1e3) / FP32_VECTOR_PEAK,
           "launch": s.describe(), "solver": solver_stats(s)}
    s.close()
    return out


def extra_workloads(steps=5, warmup=1):
    """The bicycle differentiation batch (512 OCPs, nx=8, nu=2, T=64, 10 SQP
    iterations, softplus cost weights; nominal weights, and the better
    conditioned variant), and the forward-mode sensitivity: the cart-pole
    batch, fwd + one JVP per OCP."""
    import torch
    from paper_2510_06179_amd import batch
    from paper_2510_06179_amd.solver import BatchSolver

    out = {}
    # nominal weights: condition ~4e5, so up to eight refinement passes of
    # 1e-2 each (the same KKT target); the conditioned variant: the defaults
    for name, variant, ref in (("bicycle_b512_fwd_bwd", "nominal", dict(refine_steps=8,
                                                                         refine_tol=1e-2)),
                               ("bicycle_conditioned_b512_fwd_bwd", "conditioned", {})):
        probs = W.bicycle_batch(0, batch=512, variant=variant)
        s = BatchSolver(probs, sqp_iters=10, pcg_tol=PCG_TOL, bwd_pcg_tol=PCG_TOL, **ref)
        dl = dl_arena(s, W.loss_cotangents(probs, seed=0))
        ms, fwd, bwd, _, _ = timed_fwd_bwd(s, dl, steps, warmup)
        out[name] = {"solves_per_s": len(probs) / (ms / 1e3), "fwd_ms": float(np.mean(fwd)),
                     "bwd_ms": float(np.mean(bwd)), "sqp_iters": 10, "weights": variant,
                     "refinement": ref or "default", "solver": solver_stats(s)}
        s.close()
    probs = W.cartpole_batch(0, batch=1024)
    s = BatchSolver(probs, sqp_iters=10, pcg_tol=PCG_TOL, bwd_pcg_tol=PCG_TOL)
    rng = np.random.default_rng(0)
    tps = []
    for p in probs:
        q = dict(p)
        for k in ("x0", "Qd", "q", "Rd", "r"):
            q[k] = W.f32(rng.standard_normal(np.shape(p[k])))
        q["params"] = np.zeros_like(np.asarray(p["params"]))
        tps.append(q)
    tan = torch.from_numpy(batch.pack(tps).data).to(s.device)
    sol = s.sol0.clone()
    jout = torch.zeros_like(sol)
    rhs = torch.empty_like(sol)
    grad = torch.empty_like(s.data)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for i in range(warmup + steps):
        e = ev[i - warmup] if i >= warmup else None
        sol.copy_(s.sol0)
        if e:
            e[0].record()
        s.solve(sol=sol)
        if e:
            e[1].record()
        s.solve_jvp(tan, out=jout, rhs=rhs, grad=grad)
        if e:
            e[2].record()
    torch.cuda.synchronize()
    fwd = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    jv = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    info = s.info.cpu().numpy()
    out["cartpole_b1024_fwd_jvp"] = {"solves_per_s": len(probs) / ((fwd + jv) / 1e3), "fwd_ms": fwd,
                                     "jvp_ms": jv, "jvp_pcg_iters_mean": float(info[:, 1].mean())}
    s.close()
    return out


def serve_load(seconds, rate_hz=20000.0, sessions=4096, p_bwd=0.3, p_large=0.05, seed=0):
    """Poisson arrivals of solve and solve+backward requests.  Sessions: 95%
    drawn from the uneven LTV mix, 5% large (nx=32, nu=8, T=256); a request
    picks a session uniformly (so about 5% of the requests are large) and
    perturbs its x_s by N(0, 0.01^2)."""
    import ctypes
    import threading

    from paper_2510_06179_amd.serving import Server

    rng = np.random.default_rng(seed)
    large = rng.random(sessions) < p_large
    probs = [W.ltv_problem(rng, 256, 32, 8) if big else
             W.ltv_problem(rng, int(rng.choice([16, 32, 64, 128])), int(rng.choice([4, 8, 12, 16])),
                           int(rng.choice([2, 4]))) for big in large]
    cots = W.loss_cotangents(probs, seed=seed)
    srv = Server(max_sessions=sessions, max_T=256, max_nx=32, max_nu=8, max_batch=1024,
                 max_inflight=4, hbm_budget=32 << 30, sqp_iters=1, alphas=(1.0,), pcg_tol=1e-6,
                 bwd_pcg_tol=1e-6, bwd_warm_start=True)
    t_setup = time.perf_counter()
    for k, p in enumerate(probs):
        srv.add_session(k, p, dl=(cots[k]["gx"], cots[k]["gu"], cots[k]["glam"]))
    t_setup = time.perf_counter() - t_setup
    lib, h = srv.lib, srv._h
    x0s = np.zeros((sessions, 32), np.float32)
    for k, p in enumerate(probs):
        x0s[k, :p["nx"]] = p["x0"]
    # warm every session once (cold starts are not the steady state)
    for k in range(sessions):
        srv.submit(k, bool(k % 3 == 0))
    srv.drain(timeout=300)
    srv.reset_stats()
    arr = W.poisson_arrivals(seed + 1, rate_hz, seconds)
    n = len(arr)
    sess = rng.integers(0, sessions, size=n)
    bwd = rng.random(n) < p_bwd
    xs = x0s[sess] + rng.normal(0.0, 0.01, size=(n, 32)).astype(np.float32)
    xs = np.ascontiguousarray(xs, np.float32)
    base = xs.ctypes.data
    tickets = []
    done = threading.Event()
    sent = [0]

    def reap():
        st, ps = ctypes.c_int32(), ctypes.c_int32()
        i = 0
        while True:
            if i < len(tickets):
                lib.dmpc_server_wait(h, tickets[i], -1.0, None, None, None, ctypes.byref(st),
                                     ctypes.byref(ps))
                i += 1
            elif done.is_set():
                break
            else:
                time.sleep(0.0005)

    th = threading.Thread(target=reap, daemon=True)
    th.start()
    tk = ctypes.c_int64()
    submit = lib.dmpc_server_submit
    lag = []
    t0 = time.perf_counter()
    for i in range(n):
        while True:
            now = time.perf_counter() - t0
            if now >= arr[i]:
                break
            if arr[i] - now > 0.002:
                time.sleep(0.0005)
        lag.append(now - arr[i])
        rc = submit(h, int(sess[i]), int(bwd[i]), base + 128 * i, None, ctypes.byref(tk))
        if rc == 0:
            tickets.append(tk.value)
            sent[0] += 1
    srv.drain(timeout=300)
    done.set()
    th.join()
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return {
        "arrivals": "poisson", "rate_hz": rate_hz, "seconds": seconds, "sessions": sessions,
        "requests_sent": sent[0], "large_fraction": float(large[sess].mean()) if n else 0.0,
        "backward_fraction": float(bwd.mean()) if n else 0.0,
        "completed": st["completed"], "rejected": st["rejected"], "failed": st["failed"],
        "throughput_rps": st["throughput"], "p50_latency_ms": 1e3 * st["p50_latency_s"],
        "p99_latency_ms": 1e3 * st["p99_latency_s"], "max_latency_ms": 1e3 * st["max_latency_s"],
        "light": {"completed": st["completed"] - st["heavy_completed"],
                  "p50_latency_ms": 1e3 * st["light_p50_latency_s"],
                  "p99_latency_ms": 1e3 * st["light_p99_latency_s"]},
        "large": {"completed": st["heavy_completed"],
                  "p50_latency_ms": 1e3 * st["heavy_p50_latency_s"],
                  "p99_latency_ms": 1e3 * st["heavy_p99_latency_s"]},
        "mean_group_size": st["mean_group_size"], "max_group_size": st["max_group_size"],
        "max_queue_depth": st["max_pending_seen"], "groups": st["groups"],
        "submit_lag_p99_ms": 1e3 * float(np.quantile(lag, 0.99)) if lag else 0.0,
        "wall_s": wall, "setup_s": t_setup,
        "server": {"max_batch": 1024, "max_inflight": 4, "hbm_budget_gib": 32,
                   "sqp_iters": 1, "pcg_tol": 1e-6},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle leg (CPU baseline and the sampled accuracy check)")
    ap.add_argument("--plain-sample", type=int, default=2,
                    help="problems per (T, nx, nu) class for the plain one-problem-per-launch form "
                         "(0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="duration of the serving load (0: skip)")
    ap.add_argument("--block-threads", type=int, default=0,
                    help="force the threads per workgroup (0: the library's choice)")
    ap.add_argument("--no-extra", dest="extra", action="store_false",
                    help="skip the cart-pole, bicycle and JVP throughput lines")
    ap.add_argument("--traffic-reference", action="store_true",
                    help="only run a plain 512 MiB device copy (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); "
              "the problems are independent, so a batch would shard across GPUs by problems "
              "with no exchange in either pass", file=sys.stderr)
        sys.exit(2)
    if args.traffic_reference:
        traffic_reference()
        return

    probs = headline_batch()
    cots = W.loss_cotangents(probs, seed=0)
    base = None
    cpu = None
    if not args.no_cpu:
        base = CpuBaseline(probs, cots)
        cpu = base.run()

    import torch  # noqa: F401
    from paper_2510_06179_amd.solver import BatchSolver

    s = BatchSolver(probs, sqp_iters=SQP, pcg_tol=PCG_TOL, bwd_pcg_tol=PCG_TOL,
                    block_threads=args.block_threads)
    dl = dl_arena(s, cots)
    ms_per_step, fwd_ms, bwd_ms, sol, grad = timed_fwd_bwd(s, dl, args.steps, args.warmup)
    value = B / (ms_per_step / 1e3)
    stats = solver_stats(s)
    accuracy = base.check(s, sol.cpu().numpy(), grad.cpu().numpy()) if base else None

    # roofline of the dominant kernel: the forward pass, every launch group of
    # the batch running concurrently between the fork and the join on the
    # caller's stream
    info = s.info.cpu().numpy()
    flops = sum(float(info[k, 0]) * pcg_flops(p["T"] + 1, p["nx"])
                + qp_flops(p["T"], p["nx"], p["nu"]) for k, p in enumerate(probs))
    fwd_s = float(np.mean(fwd_ms)) / 1e3
    achieved = flops / fwd_s
    nbytes = sum(ltv_bytes(p["T"], p["nx"], p["nu"]) for p in probs)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK,
            "traffic": measured_traffic(),
            "kernel": "forward pass: the fused forward_kernel of every launch group (QP data, "
                      "Schur assembly, preconditioner, PCG with double-residual refinement, "
                      "recovery, line search), all SQP iterations inside",
            "flops_per_launch": flops,
            "algorithmic_flops": "sum over problems of fwd PCG iterations x (12 N n^2 + 10 N n) "
                                 "plus one QP formation T(2n^3+2n^2 m) + N n^3/3 + 4T n^3 + "
                                 "T(2n^2+2nm)",
            "hbm_view": {"algorithmic_bytes": nbytes, "achieved_GBps": nbytes / fwd_s / 1e9,
                         "frac": nbytes / fwd_s / HBM_PEAK},
            "launch": s.describe(),
            "kernel_ms": float(np.mean(fwd_ms)), "backward_kernel_ms": float(np.mean(bwd_ms)),
            "kernel_source_hash": kernel_source_hash()}

    plain = plain_gpu(s, probs, dl, args.plain_sample, value) if args.plain_sample > 0 else None
    s.close()

    extra = None
    if args.extra:
        extra = {"cartpole_b1024_fwd_bwd": cartpole_leg()}
        extra.update(extra_workloads())
    serving = serve_load(args.serve_seconds) if args.serve_seconds > 0 else None

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"uneven LTV batch fwd+bwd in one call: B={B} OCPs, T in "
                               "{16,32,64,128}, nx in {4,8,12,16}, nu in {2,4}, A_t = I + "
                               "N(0,0.05^2), B_t ~ N(0,0.3^2), Q, R log-uniform [1e-2,1e1], "
                               f"{SQP} SQP iters, 5 step sizes, PCG rel tol {PCG_TOL:g}",
                   "global_batch": B, "seq_len": "16-128", "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "plain_gpu": plain,
        "solver": stats,
        "other_workloads": extra,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
