// Right-hand side of the forward-mode sensitivity (JVP) of the last QP's
// solution map, the linearisation point held fixed.
#include <hip/hip_runtime.h>

#include "dmpc_internal.h"

namespace dmpc {

// Differentiating the KKT system K w = rhs (Eq. ocp:KKT) along a tangent v
// of the inputs gives K dw = d rhs - dK w.  With the user signs (A+ = I, the
// paper's A and B are -A_t and -B_t, C_t = c_t) its blocks, laid out like the
// solution arena, are
//   x_t:       -(dQ_t x_t + dq_t - dA_t' lambda_{t+1})    (no dA term at t = T)
//   u_t:       -(dR_t u_t + dr_t - dB_t' lambda_{t+1})
//   lambda_0:  dx_s,   lambda_{t+1}:  dA_t x_t + dB_t u_t + dc_t
// with (x, u, lambda) the last QP's solution.  A diagonal Hessian entry held
// at the PD floor does not move; its linear term moves by dQd times the
// linearisation point (q = grad c(xbar) - Q xbar).  dA, dB, dc exist for
// linear dynamics only (a tangent of nonlinear model parameters is not read).
// K is symmetric, so the adjoint solve of the backward pass with this vector
// as its cotangent returns dw.  One workgroup per problem, double
// accumulation, rounded to float.
__global__ __launch_bounds__(256) void jvp_rhs_kernel(const ProbRec* recs, int count,
                                                      const float* data, const float* tangent,
                                                      const float* ws, float* rhs) {
  for (int pi = blockIdx.x; pi < count; pi += gridDim.x) {
    const ProbRec& rc = recs[pi];
    const int T = rc.T, nx = rc.nx, nu = rc.nu, N = T + 1;
    const int R = N * nx, TM = T * nu;
    const WsLayout L = ws_layout(T, nx, nu, rc.dyn, rc.flags);
    const float* W = ws + rc.ws_off;
    const float* xs = W + L.xp;      // last QP solution
    const float* us = W + L.up;
    const float* lam = W + L.lam;    // its multipliers
    const float* xl = W + L.xlin;    // linearisation point
    const float* ul = W + L.ulin;
    const float* cost = data + rc.cost_off;   // Qd [N][nx], q [N][nx], Rd [T][nu], r [T][nu]
    const float* dcost = tangent + rc.cost_off;
    const bool ltv = rc.dyn == DMPC_DYN_LTV;
    const float* dA = tangent + rc.dyn_off;   // LTV: A [T][nx][nx], B [T][nx][nu], c [T][nx]
    const float* dB = dA + (int64_t)T * nx * nx;
    const float* dc = dB + (int64_t)T * nx * nu;
    const float* dx0 = tangent + rc.x0_off;
    float* out = rhs + rc.sol_off;
    for (int idx = threadIdx.x; idx < R; idx += blockDim.x) {
      const int t = idx / nx, i = idx - t * nx;
      const double dh = dcost[idx];
      double v = (cost[idx] >= kPdEps ? dh * (double)xs[idx] : dh * (double)xl[idx]) +
                 (double)dcost[R + idx];
      if (ltv && t < T)
        for (int k = 0; k < nx; ++k)
          v -= (double)dA[(int64_t)t * nx * nx + k * nx + i] * (double)lam[(t + 1) * nx + k];
      out[idx] = (float)(-v);
    }
    for (int idx = threadIdx.x; idx < TM; idx += blockDim.x) {
      const int t = idx / nu, l = idx - t * nu;
      const double dh = dcost[2 * R + idx];
      double v = (cost[2 * R + idx] >= kPdEps ? dh * (double)us[idx] : dh * (double)ul[idx]) +
                 (double)dcost[2 * R + TM + idx];
      if (ltv)
        for (int k = 0; k < nx; ++k)
          v -= (double)dB[(int64_t)t * nx * nu + k * nu + l] * (double)lam[(t + 1) * nx + k];
      out[R + idx] = (float)(-v);
    }
    for (int idx = threadIdx.x; idx < R; idx += blockDim.x) {
      const int t = idx / nx, i = idx - t * nx;
      double v = 0.0;
      if (t == 0) {
        v = dx0[i];
      } else if (ltv) {
        const int tt = t - 1;
        v = dc[tt * nx + i];
        for (int j = 0; j < nx; ++j)
          v += (double)dA[(int64_t)tt * nx * nx + i * nx + j] * (double)xs[tt * nx + j];
        for (int l = 0; l < nu; ++l)
          v += (double)dB[(int64_t)tt * nx * nu + i * nu + l] * (double)us[tt * nu + l];
      }
      out[R + TM + idx] = (float)v;
    }
  }
}

int launch_jvp_rhs(const ProbRec* recs, int count, const float* data, const float* tangent,
                   const float* ws, float* rhs, void* stream) {
  if (count <= 0) return 0;
  const int grid = count < 65536 ? count : 65536;
  hipLaunchKernelGGL(jvp_rhs_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, recs, count,
                     data, tangent, ws, rhs);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace dmpc
