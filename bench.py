"""Throughput benchmark of the batched differentiable-MPC hot path on one GPU.

One step = one forward solve (Alg. sqp, 10 SQP iterations with the line
search, PCG inside) plus one backward solve (Alg. backward: adjoint PCG + VJP)
of the whole batch of 1024 cart-pole OCPs (nx=4, nu=1, T=50, dt=0.05), inputs
resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu] [--plain-sample 64]
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
    t0 = time.perf_counter()
    _oracle_fwd_bwd((0, 0))
    t1 = time.perf_counter() - t0
    n = max(cores, int(budget_s / max(t1, 1e-3)) * cores // max(cores, 1))
    n = min(n, B)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-sample", type=int, default=64)
    ap.add_argument("--block-threads", type=int, default=0,
                    help="force the threads per workgroup (0: the library's choice)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); "
              "problems are independent, see DESIGN.md for how the batch shards", file=sys.stderr)
        sys.exit(2)

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
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd_ms, bwd_ms = [], []

    def step(record):
        sol.copy_(s.sol0)
        ev[0].record()
        s.solve(sol=sol)
        ev[1].record()
        s.solve_backward(dl, adj=adj, grad=grad)
        ev[2].record()
        if record:
            torch.cuda.synchronize()
            fwd_ms.append(ev[0].elapsed_time(ev[1]))
            bwd_ms.append(ev[1].elapsed_time(ev[2]))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for _ in range(min(args.steps, 10)):
        step(True)
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
            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK, "traffic": None,
            "kernel": "forward_kernel (fused SQP: QP data, Schur assembly, preconditioner, "
                      "PCG with double-residual refinement, recovery, line search)",
            "launch": s.describe(),
            "kernel_ms": float(np.mean(fwd_ms)), "backward_kernel_ms": float(np.mean(bwd_ms))}

    # plain one-problem-per-launch GPU form on a sample of the same batch
    P = min(args.plain_sample, B)
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
    plain_wall = time.perf_counter() - t0
    plain_value = P / plain_wall

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
        "plain_gpu": {"value": plain_value, "unit": "solves/s", "sample": P,
                      "speedup_batched": value / plain_value},
        "solver": {"fwd_pcg_iters_mean": float(info[:, 0].mean()),
                   "bwd_pcg_iters_mean": float(info[:, 1].mean()),
                   "nonpd_or_nonfinite": bad, "fwd_pcg_capped": capped_f,
                   "bwd_pcg_capped": capped_b, "ls_fallback_last_iter": ls_fb},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
