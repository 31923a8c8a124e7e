"""Throughput benchmark of the batched differentiable-MPC hot path on one GPU.

One step = one forward solve (Alg. sqp, 10 SQP iterations with the line
search, PCG inside) plus one backward solve (Alg. backward: adjoint PCG + VJP)
of the whole batch of 1024 cart-pole OCPs (nx=4, nu=1, T=50, dt=0.05), inputs
resident in HBM.  Beside it: the plain one-problem-per-launch GPU form, the
FP64 oracle on the host cores, and the continuous-batching server under
Poisson arrivals (p50/p99 latency).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu] [--plain-sample 64]
                    [--serve-seconds 60] [--no-extra] [--traffic-reference]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2510_06179_amd import workloads as W  # noqa: E402

METRIC = "OCP solves/s fwd+bwd @1e-5 KKT resid vs plain GPU; p50/p99 serve latency"
B, T, NX, NU, SQP = 1024, 50, 4, 1, 10
PCG_TOL = 1e-6
FP32_VECTOR_PEAK = 157.3e12   # MI355X published FP32 vector peak (FLOP/s)


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on the host cores (run before the GPU is touched)
# ---------------------------------------------------------------------------
def _oracle_fwd_bwd(args):
    seed, k = args
    from threadpoolctl import threadpool_limits

    import oracle
    with threadpool_limits(limits=1):
        p = W.cartpole_batch(seed, batch=k + 1)[k]
        c = W.loss_cotangents([p], seed=seed)[0]
        x, u, lam, hist = oracle.sqp.sqp(p, SQP)
        h = hist[-1]   # VJP of the last QP's solution map at its linearisation point
        oracle.backward.vjp(p, h["xbar"], h["ubar"], h["qp"], h["sol"], c["gx"], c["gu"])
    return k


def cpu_baseline(budget_s=15.0):
    cores = min(os.cpu_count() or 1, 16)
    _oracle_fwd_bwd((0, 0))               # imports and first-call costs
    t0 = time.perf_counter()
    _oracle_fwd_bwd((0, 1))
    t1 = time.perf_counter() - t0
    n = int(min(B, max(cores, budget_s * cores / max(t1, 1e-3))))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        list(pool.imap_unordered(_oracle_fwd_bwd, [(0, k) for k in range(n)], chunksize=1))
    wall = time.perf_counter() - t0
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": n / wall, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} of the {B} cart-pole OCPs, fwd ({SQP} SQP iters, dense LU) + "
                      f"IFT VJP, FP64, {cores} worker processes x 1 thread on {cpu}; "
                      f"{wall:.1f} s wall"}


# ---------------------------------------------------------------------------
# GPU
# ---------------------------------------------------------------------------
def pcg_flops(N, n):
    """Algorithmic FLOPs of one PCG iteration on one problem: two
    block-tridiagonal row products (3n FMAs per row each) over N*n rows plus
    five vector updates/dot products."""
    return 12 * N * n * n + 10 * N * n


def sqp_iter_flops(T, n, m):
    """Schur assembly T(2n^3 + 2n^2 m) plus preconditioner (Gauss-Jordan of
    every diagonal block and the two off-diagonal products per row) 12 N n^3."""
    return T * (2 * n ** 3 + 2 * n * n * m) + 12 * (T + 1) * n ** 3


KERNEL_SOURCES = ("dmpc_device.h", "dmpc_internal.h", "dmpc_k4.hip", "dmpc_launch.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "forward_kernel_cartpole_traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_06179_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per forward launch from the committed counter summary, or
    None when it is missing or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


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


def extra_workloads(steps=5, warmup=1):
    """Throughput of the other two batch workloads, fwd+bwd per step: the
    bicycle differentiation batch (512 OCPs, nx=8, nu=2, T=64, 10 SQP
    iterations, softplus cost weights) and the uneven LTV batch (4096 OCPs,
    T in {16..128}, nx in {4..16}, nu in {2,4}, 8 SQP iterations); and the
    forward-mode sensitivity: the cart-pole batch, fwd + one JVP per OCP."""
    import torch
    from paper_2510_06179_amd import batch
    from paper_2510_06179_amd.solver import BatchSolver

    out = {}
    for name, probs, sqp in (("bicycle_b512_fwd_bwd", W.bicycle_batch(0, batch=512), 10),
                             ("uneven_ltv_b4096_fwd_bwd", W.ltv_uneven_batch(0, batch=4096), 8)):
        cots = W.loss_cotangents(probs, seed=0)
        s = BatchSolver(probs, sqp_iters=sqp, pcg_tol=PCG_TOL, bwd_pcg_tol=PCG_TOL)
        dl = torch.from_numpy(batch.sol_like(s.packed, [(c["gx"], c["gu"], c["glam"])
                                                        for c in cots])).to(s.device)
        sol = s.sol0.clone()
        adj = torch.zeros_like(sol)
        grad = torch.zeros_like(s.data)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        for i in range(warmup + steps):
            e = ev[i - warmup] if i >= warmup else None
            sol.copy_(s.sol0)
            if e:
                e[0].record()
            s.solve(sol=sol)
            if e:
                e[1].record()
            s.solve_backward(dl, adj=adj, grad=grad)
            if e:
                e[2].record()
        torch.cuda.synchronize()
        fwd = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
        bwd = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
        info = s.info.cpu().numpy()
        status = s.status.cpu().numpy()
        out[name] = {"solves_per_s": len(probs) / ((fwd + bwd) / 1e3), "fwd_ms": fwd, "bwd_ms": bwd,
                     "sqp_iters": sqp, "fwd_pcg_iters_mean": float(info[:, 0].mean()),
                     "bwd_pcg_iters_mean": float(info[:, 1].mean()),
                     "pcg_capped": int(np.count_nonzero(status & 1)),
                     "launch_groups": len(s.describe())}
        s.close()
    # forward-mode sensitivities: the benchmark's cart-pole batch, forward plus
    # one JVP per problem (a seeded tangent of the cost data and x_s)
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

    from paper_2510_06179_amd import _lib
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
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-sample", type=int, default=64)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="duration of the serving load (0: skip)")
    ap.add_argument("--block-threads", type=int, default=0,
                    help="force the threads per workgroup (0: the library's choice)")
    ap.add_argument("--no-extra", dest="extra", action="store_false",
                    help="skip the bicycle and uneven-LTV throughput lines")
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

    cpu = None if args.no_cpu else cpu_baseline()

    import torch
    from paper_2510_06179_amd import _lib, batch
    from paper_2510_06179_amd.solver import BatchSolver

    probs = W.cartpole_batch(0, batch=B, T=T)
    cots = W.loss_cotangents(probs, seed=0)
    s = BatchSolver(probs, sqp_iters=SQP, pcg_tol=PCG_TOL, bwd_pcg_tol=PCG_TOL,
                    block_threads=args.block_threads)
    dl = torch.from_numpy(batch.sol_like(s.packed, [(c["gx"], c["gu"], c["glam"]) for c in cots])).to(s.device)
    sol = s.sol0.clone()
    adj = torch.zeros_like(sol)
    grad = torch.zeros_like(s.data)
    # events on the stream the kernels are launched on (torch's current stream)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]

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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(ev[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = [e[0].elapsed_time(e[1]) for e in ev]
    bwd_ms = [e[1].elapsed_time(e[2]) for e in ev]
    ms_per_step = 1000.0 * wall / args.steps
    value = B / (wall / args.steps)

    status = s.status.cpu().numpy()
    info = s.info.cpu().numpy()
    bad = int(np.count_nonzero(status & (_lib.PROB_NONPD | _lib.PROB_NONFINITE)))
    capped_f = int(np.count_nonzero(status & _lib.PROB_PCG_MAXITER))
    capped_b = int(np.count_nonzero(status & _lib.PROB_BWD_PCG_MAXITER))
    ls_fb = int(np.count_nonzero(status & _lib.PROB_LS_FALLBACK))

    # roofline of the dominant kernel (the fused forward SQP kernel)
    N = T + 1
    fwd_flops = float(info[:, 0].sum()) * pcg_flops(N, NX) + B * SQP * sqp_iter_flops(T, NX, NU)
    fwd_s = float(np.mean(fwd_ms)) / 1000.0
    achieved = fwd_flops / fwd_s
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK,
            "traffic": measured_traffic(),
            "kernel": "forward_kernel (fused SQP: QP data, Schur assembly, preconditioner, "
                      "PCG with double-residual refinement, recovery, line search)",
            "flops_per_launch": fwd_flops,
            "launch": s.describe(),
            "kernel_ms": float(np.mean(fwd_ms)), "backward_kernel_ms": float(np.mean(bwd_ms)),
            "kernel_source_hash": kernel_source_hash()}

    # plain one-problem-per-launch GPU form on a sample of the same batch
    P = min(args.plain_sample, B)
    plain = None
    if P > 0:
        for i in range(2):  # warm the per-problem path
            s.solve_one(i, sol=sol)
            s.solve_backward_one(i, dl, adj=adj, grad=grad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol.copy_(s.sol0)
        for i in range(P):
            s.solve_one(i, sol=sol)
            s.solve_backward_one(i, dl, adj=adj, grad=grad)
        torch.cuda.synchronize()
        plain_value = P / (time.perf_counter() - t0)
        plain = {"value": plain_value, "unit": "solves/s", "sample": P,
                 "speedup_batched": value / plain_value}
    s.close()

    extra = extra_workloads() if args.extra else None
    serving = serve_load(args.serve_seconds) if args.serve_seconds > 0 else None

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"cartpole SQP fwd+bwd: B={B} nx={NX} nu={NU} T={T} dt=0.05, "
                               f"{SQP} SQP iters, 5 step sizes, PCG rel tol {PCG_TOL:g}",
                   "global_batch": B, "seq_len": T, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "plain_gpu": plain,
        "other_workloads": extra,
        "serving": serving,
        "solver": {"fwd_pcg_iters_mean": float(info[:, 0].mean()),
                   "bwd_pcg_iters_mean": float(info[:, 1].mean()),
                   # per-problem PCG iterations per solve: p10, p50, p90, p99, max
                   "fwd_pcg_iters_pct": [float(v) for v in
                                         np.percentile(info[:, 0], [10, 50, 90, 99, 100])],
                   "bwd_pcg_iters_pct": [float(v) for v in
                                         np.percentile(info[:, 1], [10, 50, 90, 99, 100])],
                   "nonpd_or_nonfinite": bad, "fwd_pcg_capped": capped_f,
                   "bwd_pcg_capped": capped_b, "ls_fallback_last_iter": ls_fb},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
