"""Autotuner of the kernel mapping (rows per thread, threads per workgroup,
register- or workspace-resident rows) for gfx950.

For every tuned shape it times each instantiated variant that can hold the
problem's rows -- at the smallest workgroup that holds them and at twice that
-- on a full synthetic batch of that shape (forward + backward solve, the
benchmark's options), keeps the fastest, and writes the table that
``_lib.load()`` installs (``dmpc_set_tuning``): one row per (nx, T range).

    python -m paper_2510_06179_amd.tune [--out FILE] [--reps 3]

Runs on the GPU; the committed ``tuning_gfx950.json`` was produced by it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import _lib, batch
from . import workloads as W

# (label, nx, T, batch builder, SQP iterations)
def _shapes():
    out = []
    for nx in (4, 8, 12, 16):
        for T in (16, 32, 64, 128):
            def mk(nx=nx, T=T):
                rng = np.random.default_rng(1000 * nx + T)
                return [W.ltv_problem(rng, T, nx, 4 if nx >= 12 else 2) for _ in range(1024)]
            out.append((f"ltv nx={nx} T={T}", nx, T, mk, 8))
    def big():
        rng = np.random.default_rng(32256)
        return [W.ltv_problem(rng, 256, 32, 8) for _ in range(256)]
    out.append(("ltv nx=32 T=256", 32, 256, big, 1))
    out.append(("cartpole nx=4 T=50", 4, 50, lambda: W.cartpole_batch(0, batch=1024), 10))
    out.append(("bicycle nx=8 T=64", 8, 64, lambda: W.bicycle_batch(0, batch=512), 10))
    return out


def _candidates(nx, T):
    R = (T + 1) * nx
    out = []
    for (vnx, slots, maxbt, reg) in _lib.variants():
        if vnx != nx:
            continue
        bt0 = -(-R // (64 * slots)) * 64
        for bt in (bt0, 2 * bt0):
            if bt <= maxbt and (bt == bt0 or bt0 >= 128):
                out.append((slots, maxbt, reg, bt))
    return out


def _time(probs, sqp, row, reps):
    import torch
    from .solver import BatchSolver

    _lib.install_tuning([row])
    s = BatchSolver(probs, sqp_iters=sqp, pcg_tol=1e-6, bwd_pcg_tol=1e-6)
    d = s.describe()
    assert len(d) == 1 and d[0]["slots"] == row[3] and d[0]["block_threads"] == row[6], d
    cots = W.loss_cotangents(probs, seed=0)
    dl = torch.from_numpy(batch.sol_like(s.packed, [(c["gx"], c["gu"], c["glam"])
                                                    for c in cots])).to(s.device)
    sol = s.sol0.clone()
    adj = torch.zeros_like(sol)
    grad = torch.zeros_like(s.data)
    times = []
    for i in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        sol.copy_(s.sol0)
        e0.record()
        s.solve(sol=sol)
        s.solve_backward(dl, adj=adj, grad=grad)
        e1.record()
        torch.cuda.synchronize()
        if i:
            times.append(e0.elapsed_time(e1))
    s.close()
    return float(np.median(times))


def _ranges(Ts):
    """Split T axis between neighbouring tuned horizons."""
    Ts = sorted(Ts)
    lo = [1] + [(a + b) // 2 + 1 for a, b in zip(Ts, Ts[1:])]
    hi = [(a + b) // 2 for a, b in zip(Ts, Ts[1:])] + [1000000]
    return list(zip(Ts, lo, hi))


def tune(reps=3, log=print):
    best = {}
    meas = {}
    for label, nx, T, mk, sqp in _shapes():
        probs = mk()
        res = []
        for slots, maxbt, reg, bt in _candidates(nx, T):
            row = (nx, T, T, slots, maxbt, reg, bt)
            ms = _time(probs, sqp, row, reps)
            res.append((ms, row))
            log(f"{label}: slots={slots} launch_bound={maxbt} reg={reg} bt={bt}: {ms:.3f} ms",
                flush=True)
        res.sort()
        best[(nx, T)] = res[0][1]
        meas[label] = [{"ms": ms, "slots": r[3], "launch_bound": r[4], "register_rows": r[5],
                        "block_threads": r[6]} for ms, r in res]
    _lib.install_tuning([])
    rows = []
    for nx in sorted({k[0] for k in best}):
        Ts = [T for (n, T) in best if n == nx]
        for T, lo, hi in _ranges(Ts):
            r = best[(nx, T)]
            rows.append([nx, lo, hi, r[3], r[4], r[5], r[6]])
    return {"arch": "gfx950", "rows": rows, "measurements_ms_fwd_bwd": meas,
            "note": "forward + backward solve of the whole batch, median of the timed "
                    "repetitions; rows map nx and a range of T to the fastest variant"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=_lib.TUNING_PATH)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    os.environ["DMPC_NO_TUNING"] = "1"
    t0 = time.time()
    out = tune(args.reps)
    out["seconds"] = time.time() - t0
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
