"""The QP data (diagonals, inverses, linear terms, dynamics and cost blocks)
is read from an LDS copy when the workgroup's LDS with it fits the share of a
CU that the batch leaves each problem, else from the workspace.  Where it
lives must not change a single bit of the results: the same problems solved
in a small batch (copy in LDS) and inside a large one (copy in the
workspace), forward and backward."""
import numpy as np
import pytest
import torch

from paper_2510_06179_amd import batch
from paper_2510_06179_amd import workloads as W
from _parity import gpu_only, gpu_solve

pytestmark = [pytest.mark.gpu, gpu_only]


def _fwd_bwd(probs, n_keep):
    s, res, status, info = gpu_solve(probs, sqp_iters=2, pcg_tol=1e-6, bwd_pcg_tol=1e-6)
    cots = W.loss_cotangents(probs, seed=4)
    dl = torch.from_numpy(batch.sol_like(s.packed, [(c["gx"], c["gu"], c["glam"]) for c in cots]))
    adj, grad = s.solve_backward(dl.to(s.device))
    torch.cuda.synchronize()
    grad = grad.cpu().numpy()
    lds = [d["lds_bytes"] for d in s.describe()]
    out = [(res[k], batch.split_grad(s.packed, grad, k)) for k in range(n_keep)]
    s.close()
    return lds, out


def test_qp_data_in_lds_or_workspace_gives_the_same_bits():
    rng = np.random.default_rng(11)
    probs = [W.ltv_problem(rng, 48, 8, 2) for _ in range(8)]
    filler = [W.ltv_problem(rng, 48, 8, 2) for _ in range(1100)]
    lds_small, small = _fwd_bwd(probs, len(probs))
    lds_large, large = _fwd_bwd(probs + filler, len(probs))
    # (nx = 8, T = 48: about 53 KB with the copy -- within a whole CU's LDS
    # for 8 problems, over a quarter of it for 1108)
    assert max(lds_small) > max(lds_large), (lds_small, lds_large)
    for k in range(len(probs)):
        (xs, gs), (xl, gl) = small[k], large[k]
        for a, b in zip(xs, xl):
            assert np.array_equal(a, b), k
        for key in gs:
            assert np.array_equal(gs[key], gl[key]), (k, key)
