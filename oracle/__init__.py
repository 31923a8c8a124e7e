"""FP64 CPU oracle for the batched SQP/PCG hot path of Differentiable MPC.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check and
the benchmark's CPU-baseline leg may import or run anything in this package.
The product path (the HIP library and its Python binding) never calls it and
shares no code with it.

What it computes, each step citing the paper's passage it follows:

* ``qp``       -- QP data at a linearisation point (Eq. QPmatrices, with the
                  positive-definite projection of Sec. 3.1), the dense KKT
                  matrix and right-hand side (Eq. KKTmatrix, Eq. ocp:KKT), and
                  its solution by LU with partial pivoting.  No Schur
                  complement and no conjugate gradient: the QP solution is
                  *defined* by the KKT system, so the oracle solves it densely.
* ``sqp``      -- the forward pass (Alg. sqp) with the merit line search of
                  App. A.3 (Alg. linesearch, Eqs. linesearch:merit/penalty/
                  decrease/descent).
* ``backward`` -- the implicit-function-theorem VJP (Eq. IFT, Eq. loss_gradient,
                  Eq. ocp:backward, Alg. backward) through the same dense KKT
                  matrix, expressed as cotangents of the QP data and chained to
                  the cost parameters by complex-step differentiation.
* ``exact``    -- the exact-Hessian (Newton) variant of the KKT system and
                  its gradient of the fully converged solution map (Sec. 3.4,
                  "Exact SQP vs iLQR"); reported beside Gauss-Newton, never gated.
* ``models``/``costs`` -- the dynamics and costs of the benchmark problems,
                  written so that complex arguments propagate (complex-step
                  Jacobians, Squire & Trapp 1998).

Sign convention.  Problems give explicit dynamics x_{t+1} = phi_t(x_t, u_t).
The oracle forms the paper's implicit constraint f_t(x_{t+1}, x_t, u_t) =
x_{t+1} - phi_t(x_t, u_t) and takes (A+_t, A_t, B_t) as its Jacobians (Eq.
QPmatrices), so every KKT block is exactly the paper's.

Parity status per function is listed in each module header.
"""
from . import models, costs, qp, sqp, backward, exact  # noqa: F401
