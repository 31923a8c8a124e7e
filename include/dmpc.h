/*
 * dmpc.h -- C ABI of the batched differentiable-MPC solver for AMD MI355X (gfx950).
 *
 * The library solves batches of optimal control problems (the OCP of Sec. 3 of
 * "Differentiable Model Predictive Control on the GPU"):
 *
 *   min_{x,u}  sum_{t=0}^{T} c_t^x(x_t) + sum_{t=0}^{T-1} c_t^u(u_t)
 *   s.t.       x_{t+1} = phi_t(x_t, u_t),   x_0 = x_s
 *
 * by SQP (Alg. sqp) whose QP (Sec. 3.1) is solved through the Schur complement
 * of its KKT system (Eq. shurcomplement, Eq. schur) with preconditioned
 * conjugate gradients (Alg. pcg) and the symmetric stair preconditioner
 * (Eq. S_Phiinv), followed by the merit line search (App. A.3).  The backward
 * pass (Alg. backward, Eq. ocp:backward, Eq. loss_gradient) reuses the same
 * Schur blocks and PCG for the adjoint solve and writes the vector-Jacobian
 * product with respect to every differentiable input.
 *
 * Conventions
 *   - Every pointer argument is a DEVICE pointer unless documented as host.
 *   - All floating point data is float32, row-major, stage-major.
 *   - The caller owns every buffer (arenas, workspace, status arrays).  The
 *     library allocates device memory only in dmpc_plan_create (the plan's
 *     descriptor table) and dmpc_server_create, never in a solve call; the
 *     static workspace of dmpc_solve_static is a device array that exists
 *     from the library's load on.
 *   - Calls return a dmpc_status; they never throw.  Numeric trouble of a
 *     single problem is reported in its per-problem status word, not as a call
 *     failure.  Solve calls are asynchronous on the given stream.
 *   - A handle and its plans may be used from one host thread at a time.
 */
#ifndef DMPC_H
#define DMPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------ */
/* Return codes of the API calls                                            */
/* ------------------------------------------------------------------------ */
typedef enum dmpc_status {
  DMPC_OK = 0,
  DMPC_ERR_INVALID_ARG = 1,   /* a descriptor, offset, size or option is invalid */
  DMPC_ERR_UNSUPPORTED = 2,   /* valid but not built (e.g. a state size without a kernel) */
  DMPC_ERR_HIP = 3,           /* a HIP runtime call failed */
  DMPC_ERR_NOMEM = 4          /* plan allocation failed, or a buffer is too small */
} dmpc_status;

/* Per-problem status bits written by the kernels (0 = converged normally). */
enum {
  DMPC_PROB_PCG_MAXITER = 1,      /* forward PCG hit its iteration cap before its tolerance */
  DMPC_PROB_NONPD = 2,            /* a Schur diagonal block had a non-positive pivot, or p'Sp <= 0 */
  DMPC_PROB_NONFINITE = 4,        /* NaN/Inf met in the iterate or in PCG scalars */
  DMPC_PROB_LS_FALLBACK = 8,      /* no step size passed the decrease test; the smallest was taken */
  DMPC_PROB_BWD_PCG_MAXITER = 16, /* backward PCG hit its iteration cap */
  DMPC_PROB_KKT_UNMET = 32,       /* the last QP's refinement ended with its residual above
                                     kkt_tol x its right-hand side (a pass no longer halved it:
                                     the float32 floor of an ill-conditioned system) */
  DMPC_PROB_BWD_KKT_UNMET = 64    /* the same for the backward pass's adjoint solve */
};

/* Dynamics x_{t+1} = phi_t(x_t, u_t) of a problem.  The data block at dyn_off holds:
 *   LTV      : A [T][nx][nx], B [T][nx][nu], c [T][nx]    (phi_t = A_t x + B_t u + c_t)
 *   CARTPOLE : (m_c, m_p, L, g, dt): the cart-pole of App. B.2 as printed, explicit
 *              Euler; nx = 4, nu = 1
 *   BICYCLE  : 16 parameters (a, b, m, Iz, rw, Iw, Bf, Cf, Df, Br, Cr, Dr, Cx, kappa,
 *              dt, vmin): a dynamic single-track model with Pacejka-type lateral tyre
 *              forces, explicit Euler; state (r, v, beta, omega, dpsi, e, delta, tau),
 *              input (ddelta, dtau); nx = 8, nu = 2 */
typedef enum dmpc_dyn_kind { DMPC_DYN_LTV = 0, DMPC_DYN_CARTPOLE = 1, DMPC_DYN_BICYCLE = 2 } dmpc_dyn_kind;

/* Costs.  The data block at cost_off holds:
 *   DIAG     : Qd [T+1][nx], q [T+1][nx], Rd [T][nu], r [T][nu]
 *              c_t^x = 1/2 x'diag(Qd_t)x + q_t'x, c_t^u = 1/2 u'diag(Rd_t)u + r_t'u
 *   SOFTPLUS : theta [P][nw+nu], wscale [nw+nu], wfix [nx-nw], xref [nx]
 *              (P = cost_phases, nw = cost_nw).  Stage t uses phase
 *              k = min(P*t/T, P-1) (integer division); its weights are
 *              wscale*softplus(theta[k]) for the first nw states and all inputs,
 *              wfix for the remaining states:
 *              c_t^x = 1/2 sum_i w_i (x_i - xref_i)^2, c_t^u = 1/2 sum_j w_j u_j^2
 * Cost Hessians are projected onto {H >= 1e-6 I} when the QP is formed (Sec. 3.1). */
typedef enum dmpc_cost_kind { DMPC_COST_DIAG = 0, DMPC_COST_SOFTPLUS = 1 } dmpc_cost_kind;

/* Initial guess of the SQP (Alg. sqp inputs). */
typedef enum dmpc_init_kind {
  DMPC_INIT_GIVEN = 0,   /* (x, u, lambda) from the solution arena; x_0 is reset to x_s */
  DMPC_INIT_ROLLOUT = 1  /* u from the solution arena, x rolled out from x_s, lambda = 0 */
} dmpc_init_kind;

/* One problem of a batch (host struct, 64 bytes).  Offsets are in floats.
 * Kernels are built for nx in {2, 3, 4, 8, 12, 16, 32} and nu <= 16; other
 * state sizes are UNSUPPORTED. */
typedef struct dmpc_problem {
  int32_t T;            /* horizon, >= 1 */
  int32_t nx, nu;       /* state and input sizes */
  int32_t dyn;          /* dmpc_dyn_kind */
  int32_t cost;         /* dmpc_cost_kind */
  int32_t cost_phases;  /* SOFTPLUS: number of phases P (>= 1); else 0 */
  int32_t cost_nw;      /* SOFTPLUS: number of leading states with learned weights; else 0 */
  int32_t reserved;     /* must be 0 */
  int64_t dyn_off;      /* data arena: dynamics block */
  int64_t cost_off;     /* data arena: cost block */
  int64_t x0_off;       /* data arena: x_s [nx] */
  int64_t sol_off;      /* solution arena: x [T+1][nx], u [T][nu], lambda [T+1][nx] */
} dmpc_problem;

/* Solver options (host struct). */
typedef struct dmpc_opts {
  int32_t sqp_iters;        /* fixed SQP iteration count, 1..1000 */
  int32_t pcg_max_iter;     /* forward PCG cap; 0 = N*nx + 10 */
  float pcg_tol;            /* stop when ||r||_{Phi^-1} <= pcg_tol * ||g||_{Phi^-1} */
  float pcg_abs_tol;        /* also stop when r'Phi^-1 r <= pcg_abs_tol (0 = off) */
  int32_t n_alphas;         /* number of line-search candidates, 1..8 */
  float alphas[8];          /* candidates in decreasing order, in (0, 1] */
  float ls_eta;             /* decrease parameter eta of Eq. linesearch:decrease, in (0, 1) */
  int32_t init;             /* dmpc_init_kind */
  int32_t bwd_warm_start;   /* 1: start the adjoint PCG from lambda~ in the adjoint arena */
  int32_t bwd_pcg_max_iter; /* backward PCG cap; 0 = N*nx + 10 */
  float bwd_pcg_tol;        /* backward relative tolerance (as pcg_tol) */
  int32_t block_threads;    /* threads per workgroup; 0 = chosen by the library */
  int32_t refine_steps;     /* refinement passes after each PCG solve, 0..8.  Every pass
                               re-assembles the Schur residual in double and solves the
                               correction with the float PCG; the first residual is that of
                               the warm start */
  float refine_tol;         /* relative tolerance of each refinement correction, relative
                               to the residual it corrects (0 = the pass's tol; default 1e-1) */
  float kkt_tol;            /* refinement stops once ||residual||_2 <= kkt_tol * ||KKT
                               right-hand side||_2 (default 1e-6); a warm start that
                               already meets it is kept without a PCG pass */
  int32_t graph;            /* 1 (default): a batched call replays a HIP graph of the
                               plan's launch groups (built at the plan's first batched
                               call, its kernel arguments updated when the buffers
                               change); 0: the groups are launched one by one on side
                               streams forked from and joined into the caller's stream */
} dmpc_opts;

/* Fills *o with the defaults: 1 SQP iteration, PCG tol 1e-6, up to three
 * refinement passes (tol 1e-1, KKT target 1e-6), candidates {1, 0.7, 0.3, 0.1, 0.01}
 * (App. A.3), eta = 0.4, INIT_GIVEN, graph replay on. Host only. */
void dmpc_default_opts(dmpc_opts* o);

typedef struct dmpc_handle dmpc_handle;
typedef struct dmpc_plan dmpc_plan;

/* Handle bound to a HIP device. */
dmpc_status dmpc_create(dmpc_handle** h, int device);
dmpc_status dmpc_destroy(dmpc_handle* h);

/* Host-only validation of a batch (no GPU needed).  problems: HOST array of
 * count descriptors; data_len / sol_len: arena lengths in floats.  On an
 * invalid problem, *bad_index (host, may be NULL) receives its index. */
dmpc_status dmpc_validate(const dmpc_problem* problems, int32_t count, int64_t data_len,
                          int64_t sol_len, const dmpc_opts* opts, int32_t* bad_index);

/* Host-only workspace size in bytes for a batch (no GPU needed). */
dmpc_status dmpc_workspace_size(const dmpc_problem* problems, int32_t count,
                                const dmpc_opts* opts, size_t* bytes);

/* Validates the batch and uploads its descriptor table to the handle's device
 * (the only device allocation of the library).  problems is a HOST array; the
 * plan keeps its own copy.  The plan fixes the problem shapes and offsets; the
 * arenas passed to the solve calls may change between calls. */
dmpc_status dmpc_plan_create(dmpc_handle* h, const dmpc_problem* problems, int32_t count,
                             int64_t data_len, int64_t sol_len, const dmpc_opts* opts,
                             dmpc_plan** plan);
dmpc_status dmpc_plan_workspace_size(const dmpc_plan* plan, size_t* bytes);
dmpc_status dmpc_plan_destroy(dmpc_plan* plan);

/* Forward pass: Alg. sqp for every problem of the plan.
 *   data      [data_len]  problem data (read only)
 *   sol       [sol_len]   in: initial guess per opts->init; out: x, u after the last
 *                         line search and lambda of the last QP
 *   workspace [plan_workspace_size bytes]; holds what the backward pass reuses
 *             (the last QP's data, its solution and the Schur/preconditioner
 *             blocks); must stay untouched until dmpc_solve_backward
 *   status    [count] int32 per-problem status bits (DMPC_PROB_*)
 *   info      [count][4] int32: forward PCG iterations (sum over SQP iterations),
 *             backward PCG iterations, index of the last accepted step size,
 *             SQP iterations run
 *   stream    a hipStream_t (NULL = default stream) */
dmpc_status dmpc_solve(dmpc_plan* plan, const float* data, float* sol, void* workspace,
                       int32_t* status, int32_t* info, void* stream);

/* dmpc_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same forward pass with its workspace in the library's own static device
 * buffer of DMPC_STATIC_WORKSPACE_BYTES (64 MiB) instead of a caller buffer.
 * The buffer is a file-scope device array, one per device, kept until the
 * process ends; the call itself allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).
 *   data, sol, status, info, stream  as for dmpc_solve (caller-owned)
 * Returns DMPC_ERR_NOMEM, with nothing launched, when the plan's workspace
 * (dmpc_plan_workspace_size) exceeds DMPC_STATIC_WORKSPACE_BYTES.  Every call
 * on a device shares that device's buffer and leaves its contents there:
 * calls that overlap on one device (other streams, other threads, other
 * plans) race and must be ordered by the caller.  The buffer is not a
 * workspace for dmpc_solve_backward (which takes its own). */
#define DMPC_STATIC_WORKSPACE_BYTES (64ull << 20)
dmpc_status dmpc_solve_static(dmpc_plan* plan, const float* data, float* sol, int32_t* status,
                              int32_t* info, void* stream);

/* Backward pass (Alg. backward): VJP of the last QP's solution map with the
 * linearisation point held fixed.
 *   dl_dsol [sol_len]  cotangent laid out like the solution arena: dl/dx, dl/du and
 *                      dl/dlambda (the paper's pass uses dl/dlambda = 0)
 *   adj     [sol_len]  out: x~, u~, lambda~ of Eq. ocp:backward; in: lambda~ as the
 *                      PCG warm start when opts->bwd_warm_start
 *   grad    [data_len] out: dl/d(data), laid out like the data arena: A, B, c (LTV),
 *                      Qd, q, Rd, r (DIAG), theta, xref (SOFTPLUS; wscale, wfix get 0),
 *                      x_s; parameters of CARTPOLE/BICYCLE dynamics get 0.  Floats of
 *                      the arena outside the problems' blocks are not written. */
dmpc_status dmpc_solve_backward(dmpc_plan* plan, const float* data, const float* dl_dsol,
                                float* adj, float* grad, void* workspace, int32_t* status,
                                int32_t* info, void* stream);

/* Forward-mode sensitivity (JVP) of the last QP's solution map, the
 * linearisation point held fixed (as for the backward pass): the derivative
 * of the last QP's x, u and lambda along a tangent of the inputs, from
 * differentiating Eq. ocp:KKT (K dw = d rhs - dK w; K is symmetric, so the
 * same adjoint PCG solves it, reusing the stored Schur and preconditioner
 * blocks).  Needs the workspace of a dmpc_solve on the same plan.  Problems
 * with SOFTPLUS costs: UNSUPPORTED.
 *   tangent [data_len]  tangent laid out like the data arena; read: A, B, c
 *                       (LTV), Qd, q, Rd, r (DIAG), x_s; the parameters of
 *                       CARTPOLE/BICYCLE dynamics are not read (tangent 0)
 *   rhs     [sol_len]   scratch: the right-hand side of the tangent system
 *   out     [sol_len]   out: dx, du, dlambda laid out like the solution arena;
 *                       in: the PCG warm start when opts->bwd_warm_start
 *   grad    [data_len]  scratch (the backward kernel's VJP of rhs lands here)
 * status / info as for dmpc_solve_backward (info[1]: PCG iterations). */
dmpc_status dmpc_solve_jvp(dmpc_plan* plan, const float* data, const float* tangent, float* rhs,
                           float* out, float* grad, void* workspace, int32_t* status,
                           int32_t* info, void* stream);

/* The same two passes for problem `index` of the plan alone, one launch each
 * (the plain one-problem-per-launch form). */
dmpc_status dmpc_solve_one(dmpc_plan* plan, int32_t index, const float* data, float* sol,
                           void* workspace, int32_t* status, int32_t* info, void* stream);
dmpc_status dmpc_solve_backward_one(dmpc_plan* plan, int32_t index, const float* data,
                                    const float* dl_dsol, float* adj, float* grad,
                                    void* workspace, int32_t* status, int32_t* info,
                                    void* stream);

/* Float offsets, inside the workspace, of what the forward pass keeps for the
 * backward pass of problem `index` (host only; no GPU work):
 *   out[0] x at the last linearisation point [T+1][nx]   out[1] u there [T][nu]
 *   out[2] x of the last QP solution [T+1][nx]           out[3] its u [T][nu]
 *   out[4] its multipliers [T+1][nx]
 *   out[5] projected cost Hessian diagonal Qd [T+1][nx]  out[6] projected Rd [T][nu]
 * Used to inspect the last QP (Alg. sqp returns the QP matrices). */
dmpc_status dmpc_workspace_offsets(const dmpc_plan* plan, int32_t index, int64_t* out);

/* Writes a NUL-terminated JSON description of the plan's launch groups (state
 * size, rows per thread, threads per workgroup, register residency, problem
 * count) into the host buffer buf of size len (truncated if too small). */
dmpc_status dmpc_plan_describe(const dmpc_plan* plan, char* buf, size_t len);


/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of solve and solve+backward requests        */
/* ------------------------------------------------------------------------ */
/* A server keeps, per session, one problem's data, its warm start (x, u,
 * lambda of the last solve, lambda~ of the last backward pass) and its current
 * loss cotangent in device memory (the warm-started reuse of Sec. 4).  A
 * request names a session, may bring a new initial state x_s and a new
 * cotangent, and asks for the forward pass (Alg. sqp, started from the
 * session's last solution: INIT_GIVEN) or the forward and backward passes
 * (Alg. sqp then Alg. backward).
 *
 * A dispatcher thread forms a launch group from the requests pending at that
 * moment, first come first served, while the group holds at most max_batch
 * requests and its per-problem workspaces fit one in-flight share of the
 * memory budget (hbm_budget / max_inflight).  Up to max_inflight groups run
 * at once, each on its own stream, so requests that arrive while others are
 * on the GPU are taken by the next group as soon as a share frees up, and
 * their kernels overlap on the device.  A session has at most one request in
 * flight; its later requests wait and run in submission order.  A result does
 * not depend on which other requests share its group.  Sessions too large for
 * a workgroup's LDS are "heavy": their requests form groups of their own, and
 * at most max(1, max_inflight / 2) heavy groups run at once, so that they
 * never hold up the other requests.
 *
 * Device memory is allocated in dmpc_server_create only: per-session stores
 * (max_sessions blocks sized for the largest shape max_T, max_nx, max_nu),
 * the in-flight workspaces and staging buffers (pinned host + device).
 * Calls are thread safe.  Results are copied into host memory when a group
 * finishes and stay there until dmpc_server_wait returns them. */
typedef struct dmpc_server dmpc_server;

typedef struct dmpc_server_config {
  int32_t device;           /* HIP device */
  int32_t max_sessions;     /* sessions 0..max_sessions-1, >= 1 */
  int32_t max_batch;        /* requests per launch group, 1..65536 */
  int32_t max_inflight;     /* launch groups running at once (one stream each), 1..8 */
  int32_t max_T, max_nx, max_nu;   /* largest session shape */
  int32_t max_pending;      /* submissions beyond this many waiting requests are
                               rejected (0 = no limit) */
  int32_t batch_window_us;  /* a free share waits up to this long for max_batch requests
                               before launching what is pending (0 = launch at once) */
  int32_t dry_run;          /* 1: no device work at all -- groups are formed and
                               "complete" after dry_run_us with zero outputs; for
                               testing the admission logic without a GPU */
  int32_t dry_run_us;
  int32_t reserved;         /* must be 0 */
  int64_t hbm_budget;       /* bytes of workspace for the in-flight groups (split evenly) */
  int64_t staging_bytes;    /* per in-flight group, for its inputs and again for its
                               results, pinned host + device (0 = 64 MiB); a group also
                               stops admitting when these would overflow */
  dmpc_opts opts;           /* solver options of every request; init must be GIVEN */
} dmpc_server_config;

typedef struct dmpc_server_stats {
  int64_t submitted;        /* accepted submissions */
  int64_t rejected;         /* refused submissions (queue full) */
  int64_t completed;        /* finished requests (of which backward_completed had a backward pass) */
  int64_t backward_completed;
  int64_t failed;           /* requests whose group failed to launch */
  int64_t groups;           /* launch groups run */
  double mean_group_size;
  int64_t max_group_size;
  int64_t max_pending_seen; /* deepest admission queue seen */
  double p50_latency_s, p99_latency_s, max_latency_s;  /* submit -> results on the host */
  double throughput;        /* completed / (last completion - first submission), per second */
  int64_t heavy_completed;  /* of completed: requests of heavy sessions (see below) */
  double light_p50_latency_s, light_p99_latency_s;   /* the same percentiles per class */
  double heavy_p50_latency_s, heavy_p99_latency_s;
} dmpc_server_stats;

/* Request states reported by dmpc_server_wait */
enum { DMPC_REQ_PENDING = 0, DMPC_REQ_RUNNING = 1, DMPC_REQ_DONE = 2, DMPC_REQ_FAILED = 3 };

dmpc_status dmpc_server_create(const dmpc_server_config* cfg, dmpc_server** srv);
/* Finishes the requests already launched, fails the pending ones, joins the
 * threads and frees everything. */
dmpc_status dmpc_server_destroy(dmpc_server* srv);

/* Registers (or replaces) session `session`.  problem: HOST descriptor whose
 * dyn_off, cost_off and x0_off index the HOST block data[data_len] (sol_off is
 * ignored); its shape must fit max_T, max_nx, max_nu.  sol0: HOST warm start
 * [sol block] or NULL (zeros); dl: HOST cotangent [sol block] or NULL (zeros).
 * The adjoint warm start starts at zero.  Fails with INVALID_ARG while the
 * session has requests pending or in flight. */
dmpc_status dmpc_server_add_session(dmpc_server* srv, int32_t session, const dmpc_problem* problem,
                                    const float* data, int64_t data_len, const float* sol0,
                                    const float* dl);

/* Queues a request.  x0: HOST x_s [nx] (NULL keeps the session's current one);
 * dl: HOST cotangent [sol block] that becomes the session's current one (NULL
 * keeps it).  *ticket identifies the request.  Returns NOMEM when max_pending
 * requests are already waiting (the request is not queued). */
dmpc_status dmpc_server_submit(dmpc_server* srv, int32_t session, int32_t backward,
                               const float* x0, const float* dl, int64_t* ticket);

/* Waits up to timeout_s seconds (< 0: no limit) for a request to finish and
 * copies its results into HOST buffers (each may be NULL): sol [sol block] (x,
 * u after the last line search, lambda), grad [data_len of the session]
 * (backward requests; laid out like the session's data block), info [4] (as
 * dmpc_solve).  *state receives DMPC_REQ_*, *prob_status the per-problem
 * status bits.  Once a finished request's results are returned its ticket is
 * forgotten.  An unknown ticket gives INVALID_ARG. */
dmpc_status dmpc_server_wait(dmpc_server* srv, int64_t ticket, double timeout_s, float* sol,
                             float* grad, int32_t* info, int32_t* state, int32_t* prob_status);

/* Waits until every accepted request has finished (or timeout_s passed:
 * returns INVALID_ARG then). */
dmpc_status dmpc_server_drain(dmpc_server* srv, double timeout_s);
dmpc_status dmpc_server_get_stats(dmpc_server* srv, dmpc_server_stats* out);
/* Clears the latency samples and counters (between warm-up and measurement). */
dmpc_status dmpc_server_reset_stats(dmpc_server* srv);

/* JSON array describing the last (up to 1024) launch groups: tickets, slot,
 * workspace bytes, launch and completion times (s since creation).  Written
 * into the HOST buffer buf[len] (truncated if too small). */
dmpc_status dmpc_server_trace(dmpc_server* srv, char* buf, size_t len);

/* ------------------------------------------------------------------------ */
/* Kernel mapping: instantiated variants and the tuning table                */
/* ------------------------------------------------------------------------ */
/* A problem's rows (T+1)*nx are spread over the threads of one workgroup,
 * `slots` rows per thread, with the Schur and preconditioner rows held in
 * registers (register_rows = 1) or read from the workspace (0); variants
 * with register_rows = 3 keep the Schur rows in registers and the inverted
 * diagonal blocks in LDS and apply the preconditioner of Eq. S_Phiinv in
 * factored form (half the registers); register_rows = 4 is the same with the
 * Schur rows of the last slot (those past (slots - 1) * block_threads) in
 * LDS; variants with register_rows = 2 run one wave per problem with a lane per stage block
 * (rows (T+1)*nx <= 64 * slots) and exchange neighbouring blocks between lanes
 * without LDS; register_rows = 5 (nx 8, 12, 16) runs the PCG on the system
 * scaled by the Cholesky factors of its diagonal blocks (the same iterates in
 * other variables, Eq. S_Phiinv's preconditioner becoming I - E~), with the
 * rows of its two off-diagonal blocks in registers, and applies only where
 * block_threads is a multiple of nx (whole stages per group of rows).  Without a
 * tuning-table entry the library picks the instantiated variant with the
 * lowest modelled cost.
 *
 * dmpc_list_variants writes up to max_rows rows of 4 int32 (nx, slots,
 * launch_bound, register_rows) of the instantiated kernels into the HOST array
 * out and returns how many exist.  Host only. */
int32_t dmpc_list_variants(int32_t* out, int32_t max_rows);

/* Installs the process-wide tuning table: n_rows HOST rows of 7 int32
 * (nx, T_min, T_max, slots, launch_bound, register_rows, block_threads).  A
 * problem with that nx and T_min <= T <= T_max uses the first matching row
 * whose variant is instantiated and holds its rows (slots * block_threads >=
 * (T+1)*nx, block_threads a multiple of 64 not above launch_bound, the
 * problem's LDS regions within a workgroup's LDS); otherwise
 * the cost model decides.  Replaces the previous table; n_rows = 0 clears it.
 * Affects plans and sessions created afterwards.  INVALID_ARG on a malformed
 * row (nothing is installed then); a row with register_rows = 2 must have
 * launch_bound 64 and slots a multiple of nx; one with register_rows = 4
 * launch_bound and block_threads 512 and slots >= 2; register_rows is at
 * most 5, and a register_rows = 5 row is passed over for a problem whose nx
 * does not divide block_threads.  Host only; thread safe. */
dmpc_status dmpc_set_tuning(const int32_t* rows, int32_t n_rows);

/* Copies up to max_rows rows of the installed table into the HOST array rows
 * and returns the number of rows installed. */
int32_t dmpc_get_tuning(int32_t* rows, int32_t max_rows);

/* The mapping a plan would give `problem` (HOST descriptor) under `opts`:
 * out[0..3] = slots, launch_bound, register_rows, block_threads.  UNSUPPORTED
 * when no instantiated variant holds it.  Host only. */
dmpc_status dmpc_choose_mapping(const dmpc_problem* problem, const dmpc_opts* opts, int32_t* out);

/* Human-readable name of a return code (static string). */
const char* dmpc_status_string(dmpc_status s);

/* Library version as major*10000 + minor*100 + patch. */
int32_t dmpc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DMPC_H */
