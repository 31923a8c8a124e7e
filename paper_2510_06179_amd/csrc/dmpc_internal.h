// Internal declarations shared by the host runtime (dmpc_host.cpp) and the
// device code (dmpc_kernels.hip).  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "dmpc.h"

#if defined(__HIP__)
#define DMPC_HD __host__ __device__
#else
#define DMPC_HD
#endif

namespace dmpc {

constexpr float kPdEps = 1e-6f;   // eigenvalue floor of the PD projection (Sec. 3.1)
constexpr int kMaxAlphas = 8;
constexpr int kMaxNu = 16;
constexpr int kMaxNx = 32;
constexpr int kCartpoleParams = 5;
constexpr int kBicycleParams = 16;
constexpr int kAlignFloats = 64;  // per-problem workspace alignment (256 B)
// Dynamic LDS of one workgroup: gfx950's 160 KiB less 1 KiB kept for the
// kernels' static LDS (up to 256 bytes); a launch over the total fails.
constexpr int kLdsBytes = 159 * 1024;

// ProbRec::flags
constexpr int kRecRegRows = 1;   // the kernel keeps the Schur rows in registers
constexpr int kRecBulkWs = 2;    // iterate, QP solution, multipliers and the line-search
                                 // region live in the workspace (too large for LDS)
constexpr int kRecLinLds = 4;    // the QP data (see lin_floats) is read from an LDS copy
constexpr int kRecDinvLds = 8;   // the inverted diagonal Schur blocks live in LDS (the kernel
                                 // applies the preconditioner in factored form)
constexpr int kRecTailLds = 16;  // with kRecDinvLds: the Schur rows of a thread's last value
                                 // slot live in LDS (rows past the register slots)
constexpr int kTailThreads = 512; // workgroup size of the kRecTailLds kernels
constexpr int kRecScaled = 32;   // the kernel runs the PCG on the Schur system scaled by the
                                 // Cholesky factors of its diagonal blocks (register rows of
                                 // the scaled off-diagonal blocks only)
constexpr int kComputeUnits = 256;   // CUs of an MI355X

// Device record of one problem (96 bytes).
struct ProbRec {
  int32_t T, nx, nu, dyn, cost, phases, nw, index;  // index: slot in status/info
  int64_t dyn_off, cost_off, x0_off, sol_off;
  int64_t ws_off;                                   // float offset into the workspace
  int32_t slots;                                    // rows per thread of its kernel
  int32_t flags;                                    // kRec* bits
  int64_t pad[2];
};

// Per-problem workspace layout (float offsets from ProbRec::ws_off).
struct WsLayout {
  int64_t Qd, iQ, q, Rd, iR, r;   // projected Hessian diagonals, inverses, linear terms
  int64_t iQd, iRd;               // the inverses in double (float offsets, 8-byte aligned)
  int64_t A, B, c;                // linearised dynamics (nonlinear models only)
  int64_t Ad, Bd, cd;             // the same in double (float offsets, 8-byte aligned)
  int64_t Dinv;                   // diagonal Schur blocks inverted [N][nx][nx]
  int64_t blk;                    // saved rows of S^ and Phi^-1: [N*nx][6*nx]
  int64_t xp, up, lam;            // last QP solution and multipliers
  int64_t xlin, ulin;             // last linearisation point
  int64_t g;                      // right-hand side of the Schur system [N*nx]
  int64_t bulk;                   // kRecBulkWs: the regions that do not fit LDS (-1 if unused)
  int64_t stash;                  // kRecTailLds: the multipliers (hi, lo) during a PCG [2][N*nx]
  int64_t Lid;                    // kRecScaled: the inverses of the Cholesky factors L_t of
                                  // the diagonal blocks [N][nx][nx], in double (float
                                  // offset, 8-byte aligned)
  int64_t total;
};

DMPC_HD inline int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

DMPC_HD inline int64_t bulk_floats(int64_t N, int64_t R, int64_t TM);

DMPC_HD inline WsLayout ws_layout(int T, int nx, int nu, int dyn, int flags) {
  const int64_t N = T + 1, R = N * nx, TM = (int64_t)T * nu;
  WsLayout L;
  int64_t o = 0;
  L.Qd = o; o += R;
  L.iQ = o; o += R;
  L.q = o; o += R;
  L.Rd = o; o += TM;
  L.iR = o; o += TM;
  L.r = o; o += TM;
  o = align_up(o, 4);
  L.iQd = o; o += 2 * R;
  L.iRd = o; o += 2 * TM;
  o = align_up(o, 4);
  if (dyn != DMPC_DYN_LTV) {
    L.A = o; o += (int64_t)T * nx * nx;
    L.B = o; o += (int64_t)T * nx * nu;
    L.c = o; o += (int64_t)T * nx;
    o = align_up(o, 4);
    L.Ad = o; o += 2 * (int64_t)T * nx * nx;
    L.Bd = o; o += 2 * (int64_t)T * nx * nu;
    L.cd = o; o += 2 * (int64_t)T * nx;
  } else {
    L.A = L.B = L.c = L.Ad = L.Bd = L.cd = -1;
  }
  o = align_up(o, 4);
  L.Dinv = o; o += N * nx * nx;
  o = align_up(o, 4);
  L.blk = o; o += R * 6 * nx;
  L.xp = o; o += R;
  L.up = o; o += TM;
  L.lam = o; o += R;
  L.xlin = o; o += R;
  L.ulin = o; o += TM;
  L.g = o; o += R;
  if (flags & kRecBulkWs) {
    o = align_up(o, 4);
    L.bulk = o; o += bulk_floats(N, R, TM);
  } else {
    L.bulk = -1;
  }
  if (flags & kRecTailLds) {
    o = align_up(o, 4);
    L.stash = o; o += 2 * R;
  } else {
    L.stash = -1;
  }
  if (flags & kRecScaled) {
    o = align_up(o, 4);
    L.Lid = o; o += 2 * N * nx * nx;
  } else {
    L.Lid = -1;
  }
  L.total = align_up(o, kAlignFloats);
  return L;
}

// Sizes (floats) of the data blocks of a problem.
DMPC_HD inline int64_t dyn_block_len(int T, int nx, int nu, int dyn) {
  if (dyn == DMPC_DYN_LTV) return (int64_t)T * (nx * nx + nx * nu + nx);
  if (dyn == DMPC_DYN_CARTPOLE) return kCartpoleParams;
  return kBicycleParams;
}
DMPC_HD inline int64_t cost_block_len(int T, int nx, int nu, int cost, int phases, int nw) {
  if (cost == DMPC_COST_DIAG) return 2 * (int64_t)(T + 1) * nx + 2 * (int64_t)T * nu;
  return (int64_t)phases * (nw + nu) + (nw + nu) + (nx - nw) + nx;
}
DMPC_HD inline int64_t sol_block_len(int T, int nx, int nu) {
  return 2 * (int64_t)(T + 1) * nx + (int64_t)T * nu;
}

// LDS floats a workgroup needs for a problem (forward and backward kernels).
// (must match the device-side carve in dmpc_device.h: every region rounded up
// to 4 floats)
DMPC_HD inline int64_t a4h(int64_t v) { return (v + 3) / 4 * 4; }
// Shared region used by the line search (stage costs and defects of every
// candidate, per-candidate sums) and, during a QP solve, by the refinement
// residual (the primal point of the current multipliers): doubles.
DMPC_HD inline int64_t ls_floats(int64_t N, int64_t R, int64_t TM) {
  const int64_t a = 4 * (kMaxAlphas + 1) * N + 4 * (kMaxAlphas + 1);
  const int64_t b = 2 * (R + TM);
  return a > b ? a : b;
}
// Regions that may live in LDS or in the workspace: iterate, QP solution
// (x, u each), multipliers, line-search / refinement region.
DMPC_HD inline int64_t bulk_floats(int64_t N, int64_t R, int64_t TM) {
  return 3 * a4h(R) + 2 * a4h(TM) + a4h(ls_floats(N, R, TM));
}
// Length of one vector window: a zero pad of nx, an entry per row (per row of
// every slot when the rows are in registers: those PCG loops have no row
// guard), and 2 nx of zero pad.
DMPC_HD inline int64_t win_floats(int64_t R, int nx, int bt, int slots, int flags) {
  if (flags & kRecTailLds) {   // register slots unguarded, the LDS slot up to R
    const int64_t reg = (int64_t)(slots - 1) * bt;
    return a4h((R > reg ? R : reg) + 3 * nx);
  }
  return a4h(((flags & kRecRegRows) ? (int64_t)slots * bt : R) + 3 * nx);
}
// Rows held in LDS under kRecTailLds (those past the register slots) and the
// LDS stride of one such row: its 3 nx Schur coefficients padded to a
// multiple of four floats with an odd number of 16-byte words, so that the
// 16-byte reads of consecutive lanes fall on distinct banks.
DMPC_HD inline int64_t tail_rows(int64_t R, int bt, int slots, int flags) {
  if (!(flags & kRecTailLds)) return 0;
  const int64_t t = R - (int64_t)(slots - 1) * bt;
  return t > 0 ? t : 0;
}
DMPC_HD constexpr int tail_stride(int nx) {
  return ((3 * nx + 3) / 4) % 2 == 1 ? (3 * nx + 3) / 4 * 4 : (3 * nx + 3) / 4 * 4 + 4;
}
// QP data read by every phase of an SQP iteration, copied to LDS under
// kRecLinLds (one region after the reductions): an image of the workspace
// span [Qd, lin_span) -- diagonals, inverses (float and double), linear terms
// and, for nonlinear models, the linearised dynamics in float and double --
// then, for LTV problems, the dynamics block (A, B, c as in the data arena),
// then the cost block.  Offsets of the image equal the workspace offsets.
DMPC_HD inline int64_t lin_span(int T, int nx, int nu, int dyn) {
  const WsLayout L = ws_layout(T, nx, nu, dyn, 0);
  return dyn != DMPC_DYN_LTV ? L.cd + 2 * (int64_t)T * nx : L.iRd + 2 * (int64_t)T * nu;
}
DMPC_HD inline int64_t lin_floats(int T, int nx, int nu, int dyn, int64_t cost_len) {
  int64_t n = a4h(lin_span(T, nx, nu, dyn));
  if (dyn == DMPC_DYN_LTV) n += a4h(dyn_block_len(T, nx, nu, dyn));
  return n + a4h(cost_len);
}
inline int64_t lin_floats_of(const dmpc_problem& p) {
  return lin_floats(p.T, p.nx, p.nu, p.dyn,
                    cost_block_len(p.T, p.nx, p.nu, p.cost, p.cost_phases, p.cost_nw));
}
DMPC_HD inline int64_t piv_floats(int64_t R, int nx, int bt, int flags) {
  int64_t v = 4 * (int64_t)bt;
  if ((flags & kRecDinvLds) && R * nx > v) v = R * nx;
  if ((flags & kRecScaled) && 2 * R > v) v = 2 * R;
  return v;
}
DMPC_HD inline int64_t lds_floats(int T, int nx, int nu, int bt, int slots, int flags,
                                  int64_t lin) {
  const int64_t N = T + 1, R = N * nx, TM = (int64_t)T * nu;
  return ((flags & kRecBulkWs) ? 0 : bulk_floats(N, R, TM))
         + 3 * win_floats(R, nx, bt, slots, flags)   // three padded windows
         // Gauss-Jordan pivot rows, double buffered (kRecDinvLds: the rows of
         // the inverted diagonal blocks share the region; kRecScaled: the
         // Cholesky exchange, one double row per stage)
         + piv_floats(R, nx, bt, flags)
         + 128                           // reductions
         + tail_rows(R, bt, slots, flags) * tail_stride(nx)   // kRecTailLds rows
         + ((flags & kRecLinLds) ? lin : 0);
}
// Record flags of a problem run by a kernel variant: register rows as the
// variant has them; the bulk regions go to the workspace when LDS is too
// small; the QP data (lin floats) is copied to LDS when the workgroup's LDS
// stays within lin_budget bytes (0: never).
DMPC_HD inline int rec_flags(int T, int nx, int nu, int bt, int slots, int reg, int64_t lin,
                             int64_t lin_budget) {
  const int f = (reg ? kRecRegRows : 0) | ((reg == 3 || reg == 4) ? kRecDinvLds : 0) |
                (reg == 4 ? kRecTailLds : 0) | (reg == 5 ? kRecScaled : 0);
  if (lds_floats(T, nx, nu, bt, slots, f, 0) * 4 > kLdsBytes) return f | kRecBulkWs;
  if (lds_floats(T, nx, nu, bt, slots, f | kRecLinLds, lin) * 4 <= lin_budget) return f | kRecLinLds;
  return f;
}
// LDS budget for the QP-data copy when `resident` problems share the chip at
// once: the LDS of a CU divided among the problems each CU then holds (at
// most four, the one-wave-per-SIMD case of the one-wave kernels).
DMPC_HD inline int64_t lin_budget(int64_t resident) {
  int64_t per_cu = (resident + kComputeUnits - 1) / kComputeUnits;
  per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
  return kLdsBytes / per_cu;
}

// Launch-time arguments of the kernels.
struct KArgs {
  const ProbRec* recs;
  int32_t count;
  int32_t first;        // first record of this launch (plain mode uses count = 1)
  const float* data;
  float* sol;
  float* ws;
  const float* dl;
  float* adj;
  float* grad;
  int32_t* status;
  int32_t* info;
  int32_t sqp_iters, pcg_max_iter, n_alphas, init;
  int32_t bwd_warm, bwd_max_iter, refine_steps;
  float pcg_tol, pcg_abs_tol, ls_eta, bwd_tol, refine_tol, kkt_tol;
  float alphas[kMaxAlphas];
};

// One launch group: problems sharing a kernel instantiation.
struct LaunchCfg {
  int nx;          // template state size
  int slots;       // rows per thread
  int maxbt;       // launch bound of the instantiation
  int reg;         // 1: Schur/preconditioner rows kept in registers
  int bt;          // threads per workgroup
  int grid;        // workgroups
  size_t lds_bytes;
};

// Implemented in dmpc_host.cpp (shared with the serving runtime).
bool nx_supported(int nx);
dmpc_status check_opts(const dmpc_opts* o);
dmpc_status check_problem(const dmpc_problem& p, int64_t data_len, int64_t sol_len);
bool choose_cfg(const dmpc_problem& p, int force_bt, LaunchCfg* c);
int problem_flags(const dmpc_problem& p, int force_bt);   // ProbRec::flags under choose_cfg
// Right-hand side of the JVP system for every record (dmpc_jvp.hip); 0 or -2.
int launch_jvp_rhs(const ProbRec* recs, int count, const float* data, const float* tangent,
                   const float* ws, float* rhs, void* stream);

KArgs make_kargs(const dmpc_opts& o, const ProbRec* recs, const float* data, float* sol, void* ws,
                 const float* dl, float* adj, float* grad, int32_t* status, int32_t* info);

// A copy of len 32-bit words between two device addresses (serving scatter
// and gather).
struct Seg {
  const uint32_t* src;
  uint32_t* dst;
  int64_t len;
};

// Implemented in dmpc_serve.hip: copies every segment of segs[n] (device).
int launch_seg_copy(const Seg* segs, int n, void* stream);

// Implemented in dmpc_launch.hip.
bool kernel_available(int nx, int slots, int maxbt, int reg);
int launch_forward(const LaunchCfg& cfg, const KArgs& a, void* stream);
int launch_backward(const LaunchCfg& cfg, const KArgs& a, void* stream);
// The kernel of a launch group (with its dynamic-LDS limit raised as the
// launch functions do), for graph nodes; nullptr if not instantiated or the
// limit cannot be set.
const void* kernel_function(const LaunchCfg& cfg, bool fwd);

}  // namespace dmpc
