// Device templates of the batched differentiable-MPC solver for gfx950 (CDNA4).
// Instantiated per state size in dmpc_k<nx>.hip; launched from dmpc_launch.hip.
//
// One workgroup owns one OCP at a time (persistent grid-stride loop over the
// problems of a launch).  Thread <-> scalar row of the multiplier vector:
// row rho = t*nx + i (stage t, component i) lives in thread rho % BT, slot
// rho / BT.  The thread keeps its row of the Schur complement S^ = H G^-1 H'
// and of the preconditioner Phi^-1 in registers as 3*nx contiguous
// coefficients [lower block | diagonal block | upper block]; both matrices
// are block-tridiagonal (Eq. S_Phiinv), so a row product only needs the
// 3*nx-long window of the vector around block t, which the workgroup shares
// through LDS.  Dot products are wave butterflies plus one LDS exchange, in a
// fixed order (bitwise reproducible, identical in every thread).
//
// Sign convention: the user's explicit dynamics x_{t+1} = phi_t(x_t, u_t)
// linearise to x_{t+1} = A_t x_t + B_t u_t + c_t.  In the paper's notation
// this is A+_t = I, A^paper_t = -A_t, B^paper_t = -B_t, C_t = c_t.  The PCG
// runs on S^ = -S (symmetric positive definite) with right-hand side
// g = -gamma (Eq. shurcomplement), which gives the same lambda as S lambda =
// gamma; Phi^-1 is the block matrix displayed in Eq. S_Phiinv, whose general
// block is  diag: D_t^-1,  off-diagonal: -D_t^-1 E_{t,t+-1} D_{t+-1}^-1,
// with D_t, E the diagonal and off-diagonal blocks of S^.
#pragma once
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>


#include "dmpc_internal.h"

namespace dmpc {

// ===========================================================================
// Forward-mode dual numbers (Jacobians of the nonlinear models), base type R
// ===========================================================================
template <typename T>
struct Ident {
  typedef T type;
};

template <int K, typename R>
struct Dual {
  R v;
  R d[K];
};

template <int K, typename R>
__device__ __forceinline__ Dual<K, R> mkconst(R a) {
  Dual<K, R> r;
  r.v = a;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = R(0);
  return r;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator+(const Dual<K, R>& a, const Dual<K, R>& b) {
  Dual<K, R> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator-(const Dual<K, R>& a, const Dual<K, R>& b) {
  Dual<K, R> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator-(const Dual<K, R>& a) {
  Dual<K, R> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator*(const Dual<K, R>& a, const Dual<K, R>& b) {
  Dual<K, R> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator/(const Dual<K, R>& a, const Dual<K, R>& b) {
  Dual<K, R> r;
  const R ib = R(1) / b.v;
  r.v = a.v * ib;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator+(const Dual<K, R>& a, typename Ident<R>::type b) {
  Dual<K, R> r = a;
  r.v += b;
  return r;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator+(typename Ident<R>::type b, const Dual<K, R>& a) {
  return a + b;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator-(const Dual<K, R>& a, typename Ident<R>::type b) {
  Dual<K, R> r = a;
  r.v -= b;
  return r;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator-(typename Ident<R>::type b, const Dual<K, R>& a) {
  Dual<K, R> r = -a;
  r.v += b;
  return r;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator*(const Dual<K, R>& a, typename Ident<R>::type b) {
  Dual<K, R> r;
  r.v = a.v * b;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b;
  return r;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator*(typename Ident<R>::type b, const Dual<K, R>& a) {
  return a * b;
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> operator/(const Dual<K, R>& a, typename Ident<R>::type b) {
  return a * (R(1) / b);
}

template <int K, typename R>
__device__ __forceinline__ Dual<K, R> chain(const Dual<K, R>& a, R fv, R dfv) {
  Dual<K, R> r;
  r.v = fv;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = dfv * a.d[k];
  return r;
}
// Sine and cosine in double, branch free, from one argument reduction
// (Cody and Waite): x = k pi/2 + r with k = rint(2x/pi) and pi/2 split into
// its leading 33 bits, the next 33 bits and the rounded remainder (so k P1
// and k P2 are exact for |k| < 2^20), |r| <= pi/4; then the Taylor series of
// sin r to r^19 and cos r to r^18 (truncation below 2^-70 relative), and the
// quadrant k mod 4 selects and negates.  Within a few ulp of the exact values
// for |x| < 2^20 pi/2 (the models' angles are far smaller); NaN for a
// non-finite x.  Coefficients (-1)^k/(2k+1)! and (-1)^k/(2k)!, rounded.
__device__ __forceinline__ void sincos_cw(double x, double& sn, double& cs) {
  constexpr double kInvPio2 = 0x1.45f306dc9c883p-1;
  constexpr double kP1 = 0x1.921fb54400000p+0, kP2 = 0x1.0b4611a600000p-34,
                   kP3 = 0x1.3198a2e037073p-69;
  const double k = rint(x * kInvPio2);
  const double r = ((x - k * kP1) - k * kP2) - k * kP3;
  const double z = r * r;
  double ps = -0x1.2f49b46814157p-57;   // 1/19!
  ps = fma(ps, z, 0x1.952c77030ad4ap-49);
  ps = fma(ps, z, -0x1.ae7f3e733b81fp-41);
  ps = fma(ps, z, 0x1.6124613a86d09p-33);
  ps = fma(ps, z, -0x1.ae64567f544e4p-26);
  ps = fma(ps, z, 0x1.71de3a556c734p-19);
  ps = fma(ps, z, -0x1.a01a01a01a01ap-13);
  ps = fma(ps, z, 0x1.1111111111111p-7);
  ps = fma(ps, z, -0x1.5555555555555p-3);   // -1/3!
  const double sr = fma(ps * z, r, r);
  double pc = -0x1.6827863b97d97p-53;   // -1/18!
  pc = fma(pc, z, 0x1.ae7f3e733b81fp-45);
  pc = fma(pc, z, -0x1.93974a8c07c9dp-37);
  pc = fma(pc, z, 0x1.1eed8eff8d898p-29);
  pc = fma(pc, z, -0x1.27e4fb7789f5cp-22);
  pc = fma(pc, z, 0x1.a01a01a01a01ap-16);
  pc = fma(pc, z, -0x1.6c16c16c16c17p-10);
  pc = fma(pc, z, 0x1.5555555555555p-5);
  pc = fma(pc, z, -0.5);
  const double cr = fma(pc, z, 1.0);
  const int q = (int)(k - 4.0 * floor(k * 0.25));   // k mod 4 in 0..3
  const double s0 = (q & 1) ? cr : sr;
  const double c0 = (q & 1) ? sr : cr;
  sn = (q & 2) ? -s0 : s0;
  cs = ((q + 1) & 2) ? -c0 : c0;
}
__device__ __forceinline__ double sin_(double a) {
  double s, c;
  sincos_cw(a, s, c);
  return s;
}
__device__ __forceinline__ double cos_(double a) {
  double s, c;
  sincos_cw(a, s, c);
  return c;
}
__device__ __forceinline__ double atan_(double a) { return atan(a); }
__device__ __forceinline__ double tanh_(double a) { return tanh(a); }
__device__ __forceinline__ double sqrt_(double a) { return sqrt(a); }
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> sin_(const Dual<K, R>& a) {
  return chain(a, sin_(a.v), cos_(a.v));
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> cos_(const Dual<K, R>& a) {
  return chain(a, cos_(a.v), -sin_(a.v));
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> atan_(const Dual<K, R>& a) {
  return chain(a, atan_(a.v), R(1) / (R(1) + a.v * a.v));
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> tanh_(const Dual<K, R>& a) {
  const R t = tanh_(a.v);
  return chain(a, t, R(1) - t * t);
}
template <int K, typename R>
__device__ __forceinline__ Dual<K, R> sqrt_(const Dual<K, R>& a) {
  const R q = sqrt_(a.v);
  return chain(a, q, R(0.5) / q);
}

// ===========================================================================
// Models (explicit dynamics phi_t; scalar type S = float or Dual<K>)
// ===========================================================================
// Cart-pole of App. B.2 as printed (cart acceleration without the input,
// pole acceleration with the unsquared rate), explicit Euler.
// par = (m_c, m_p, L, g, dt)
template <typename S>
__device__ __forceinline__ void cartpole_step(const float* par, const S* x, const S* u, S* xn) {
  const float mc = par[0], mp = par[1], L = par[2], g = par[3], dt = par[4];
  const float M = mp + mc;
  const S s = sin_(x[2]);
  const S c = cos_(x[2]);
  const S den = M + mp * (1.0 - c * c);
  const S d2 = ((mp * g) * s * c - (mp * L) * s * x[3] * x[3]) / (den * L);
  const S d4 = ((mp * g) * s * c - (mp * L) * s * x[3] + u[0]) / den;
  xn[0] = x[0] + dt * x[1];
  xn[1] = x[1] + dt * d2;
  xn[2] = x[2] + dt * x[3];
  xn[3] = x[3] + dt * d4;
}

// Dynamic single-track model with Pacejka-type lateral tyre forces and a
// saturating rear longitudinal force, path-relative coordinates, actuator
// states (delta, tau) driven by their rates; explicit Euler.
// par = (a, b, m, Iz, rw, Iw, Bf, Cf, Df, Br, Cr, Dr, Cx, kappa, dt, vmin)
template <typename S>
__device__ __forceinline__ void bicycle_step(const float* p, const S* x, const S* u, S* xn) {
  const float a = p[0], b = p[1], m = p[2], Iz = p[3], rw = p[4], Iw = p[5];
  const float Bf = p[6], Cf = p[7], Df = p[8], Br = p[9], Cr = p[10], Dr = p[11];
  const float Cx = p[12], kap = p[13], dt = p[14], vmin = p[15];
  const S r = x[0], v = x[1], beta = x[2], om = x[3], dpsi = x[4], e = x[5];
  const S delta = x[6], tau = x[7];
  const S cb = cos_(beta), sb = sin_(beta);
  const S vx = v * cb, vy = v * sb;
  const S vxs = sqrt_(vx * vx + vmin * vmin);
  const S vs = sqrt_(v * v + vmin * vmin);
  const S af = atan_((vy + a * r) / vxs) - delta;
  const S ar = atan_((vy - b * r) / vxs);
  const S Fyf = -Df * sin_(Cf * atan_(Bf * af));
  const S Fyr = -Dr * sin_(Cr * atan_(Br * ar));
  const S slip = (om * rw - vx) / vxs;
  const S Fxr = Dr * tanh_((Cx / Dr) * slip);
  const S cd = cos_(delta), sd = sin_(delta);
  const S Fx = Fxr - Fyf * sd;
  const S Fy = Fyf * cd + Fyr;
  const S d_r = (a * Fyf * cd - b * Fyr) / Iz;
  const S d_v = (Fx * cb + Fy * sb) / m;
  const S d_beta = (Fy * cb - Fx * sb) / (m * vs) - r;
  const S d_om = (tau - rw * Fxr) / Iw;
  const S d_psi = r - kap * v * cos_(dpsi + beta) / (1.0 - kap * e);
  const S d_e = v * sin_(dpsi + beta);
  xn[0] = r + dt * d_r;
  xn[1] = v + dt * d_v;
  xn[2] = beta + dt * d_beta;
  xn[3] = om + dt * d_om;
  xn[4] = dpsi + dt * d_psi;
  xn[5] = e + dt * d_e;
  xn[6] = delta + dt * u[0];
  xn[7] = tau + dt * u[1];
}

// ===========================================================================
// Reductions (fixed order: every thread obtains the same bits)
// ===========================================================================
// Wave sum with DPP: xor-1 and xor-2 quad permutations, half-row and row
// mirrors (each lane pairs with a distinct partner, so every lane of a row of
// 16 holds the same bits), then row broadcasts: each row adds the last lane
// of the row before it, then rows 2 and 3 add lane 31, so lane 63 holds
// (r3 + r2) + (r1 + r0) (the other lanes hold partial sums), which is read
// into a scalar (the same bits in every lane).
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);        // row_half_mirror
  v += dpp<0x140>(v);        // row_mirror
  v += dpp<0x142>(v);        // row_bcast:15
  v += dpp<0x143>(v);        // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)u, l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Double wave sum, the same pattern on the two halves of each double.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_d(double v) {
  // (bound_ctrl: lanes without a source read zero, so no old value is needed)
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)u, CTRL, ROWS, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, ROWS, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// K independent double wave sums, step-major so that the K DPP exchanges of a
// step are in flight together (the same pattern and order as wave_sum_d).
template <int K>
__device__ __forceinline__ void wave_sum_d_multi(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0xB1>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x4E>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x141>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x140>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x142>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_d<0x143>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = readlane_d(v[k], 63);
}
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  v += dpp_d<0x142>(v);
  v += dpp_d<0x143>(v);
  return readlane_d(v, 63);
}
__device__ __forceinline__ double block_sum_d(double v, double* red, int nwv) {
  v = wave_sum_d(v);
  if (nwv == 1) return v;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nwv; ++w) s += red[w];
  return s;
}

// Block sum: wave sums, then (several waves) one LDS exchange read in order.
__device__ __forceinline__ float block_sum(float v, float* red, int nwv) {
  v = wave_sum(v);
  if (nwv == 1) return v;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.f;
  for (int w = 0; w < nwv; ++w) s += red[w];
  return s;
}

// ===========================================================================
// LDS carve
// ===========================================================================
struct Carve {
  int xbar, ubar, xp, up, lam, w0, w1, w2, piv, red, dinv, tail, ls, lin;
};
__device__ __forceinline__ int a4(int v) { return (v + 3) & ~3; }
// Offsets: the bulk regions (iterate, QP solution, multipliers, line-search
// region) from the bulk base -- the start of LDS, or the workspace's bulk
// region for problems too large for LDS -- and the windows, pivot rows,
// reduction slots and the QP-data copy in LDS after them (or from the start
// of LDS).
__device__ __forceinline__ Carve carve(int R, int TM, int N, int nx, int bt, int slots,
                                       int flags) {
  Carve C;
  int o = 0;
  C.xbar = o;  o += a4(R);            // forward: iterate;     backward: x~
  C.ubar = o;  o += a4(TM);           //                                   u~
  C.xp = o;    o += a4(R);            // QP solution
  C.up = o;    o += a4(TM);
  C.lam = o;   o += a4(R);            // backward: forward multipliers
  C.ls = o;    o += a4((int)ls_floats(N, R, TM));   // doubles
  if (flags & kRecBulkWs) o = 0;
  const int wl = (int)win_floats(R, nx, bt, slots, flags);
  C.w0 = o;    o += wl;
  C.w1 = o;    o += wl;
  C.w2 = o;    o += wl;               // low part of a double-float vector in w0
  // Gauss-Jordan pivot rows (assembly only); kRecDinvLds: the rows of the
  // inverted diagonal blocks share the region (staged after the assembly)
  C.piv = o;
  C.dinv = o;
  o += (int)piv_floats(R, nx, bt, flags);
  C.red = o;   o += 128;
  C.tail = o;                         // kRecTailLds: Schur rows past the register slots
  o += (int)tail_rows(R, bt, slots, flags) * tail_stride(nx);
  C.lin = o;                          // kRecLinLds: the QP-data copy (lin_floats)
  return C;
}
// ===========================================================================
// Per-problem context
// ===========================================================================
struct Prob {
  int T, N, m, R, TM, dyn, cost, phases, nw, slots, flags;
  const float* dynp;   // dynamics block in the data arena
  const float* costp;  // cost block in the data arena
  const float* x0;
  const float* A;      // linearised dynamics (arena for LTV, workspace otherwise)
  const float* B;
  const float* c;
  const double* Ad;    // the same in double (nonlinear models; null for LTV)
  const double* Bd;
  const double* cd;
  float* W;            // problem workspace base
  float* Wq;           // QP data (Qd .. cd at workspace offsets): W, or its LDS copy
  WsLayout L;
};

template <int NX>
__device__ __forceinline__ Prob make_prob(const ProbRec& pr, const float* data, float* ws) {
  Prob P;
  P.T = pr.T;
  P.N = pr.T + 1;
  P.m = pr.nu;
  P.R = P.N * NX;
  P.TM = pr.T * pr.nu;
  P.dyn = pr.dyn;
  P.cost = pr.cost;
  P.phases = pr.phases;
  P.nw = pr.nw;
  P.slots = pr.slots;
  P.flags = pr.flags;
  P.dynp = data + pr.dyn_off;
  P.costp = data + pr.cost_off;
  P.x0 = data + pr.x0_off;
  P.W = ws + pr.ws_off;
  P.L = ws_layout(pr.T, NX, pr.nu, pr.dyn, pr.flags);
  if (pr.dyn == DMPC_DYN_LTV) {
    P.A = P.dynp;
    P.B = P.A + pr.T * NX * NX;
    P.c = P.B + pr.T * NX * pr.nu;
    P.Ad = P.Bd = P.cd = nullptr;
  } else {
    P.A = P.W + P.L.A;
    P.B = P.W + P.L.B;
    P.c = P.W + P.L.c;
    P.Ad = (const double*)(P.W + P.L.Ad);
    P.Bd = (const double*)(P.W + P.L.Bd);
    P.cd = (const double*)(P.W + P.L.cd);
  }
  P.Wq = P.W;
  if (pr.flags & kRecLinLds) {
    // QP data, dynamics and costs from the LDS copy (staged by the kernels)
    extern __shared__ float smem[];
    const Carve C = carve(P.R, P.TM, P.N, NX, blockDim.x, P.slots, P.flags);
    float* b = smem + C.lin;
    P.Wq = b;
    const int span = (int)a4h(lin_span(P.T, NX, P.m, P.dyn));
    if (P.dyn == DMPC_DYN_LTV) {
      P.A = b + span;
      P.B = P.A + P.T * NX * NX;
      P.c = P.B + P.T * NX * P.m;
      P.costp = b + span + (int)a4h(dyn_block_len(P.T, NX, P.m, P.dyn));
    } else {
      P.A = b + P.L.A;
      P.B = b + P.L.B;
      P.c = b + P.L.c;
      P.Ad = (const double*)(b + P.L.Ad);
      P.Bd = (const double*)(b + P.L.Bd);
      P.cd = (const double*)(b + P.L.cd);
      P.costp = b + span;
    }
  }
  return P;
}

// Workgroup copy of n floats, four loads in flight per thread before their
// stores (the copies below are latency bound).  VEC: both ends 16-byte
// aligned and n a multiple of 4.
template <bool VEC>
__device__ __forceinline__ void copy_block(float* dst, const float* src, int n) {
  const int BT = blockDim.x;
  int i = threadIdx.x;
  if constexpr (VEC) {
    const float4* s4 = reinterpret_cast<const float4*>(src);
    float4* d4 = reinterpret_cast<float4*>(dst);
    const int n4 = n >> 2;
    for (; i + 3 * BT < n4; i += 4 * BT) {
      const float4 a = s4[i], b = s4[i + BT], c = s4[i + 2 * BT], e = s4[i + 3 * BT];
      d4[i] = a;
      d4[i + BT] = b;
      d4[i + 2 * BT] = c;
      d4[i + 3 * BT] = e;
    }
    for (; i < n4; i += BT) d4[i] = s4[i];
  } else {
    for (; i + 3 * BT < n; i += 4 * BT) {
      const float a = src[i], b = src[i + BT], c = src[i + 2 * BT], e = src[i + 3 * BT];
      dst[i] = a;
      dst[i + BT] = b;
      dst[i + 2 * BT] = c;
      dst[i + 3 * BT] = e;
    }
    for (; i < n; i += BT) dst[i] = src[i];
  }
}

// kRecLinLds staging (whole workgroup; the caller synchronises): the cost
// block and, for LTV problems, the dynamics block from the data arena into
// the LDS copy; with `qp` also the QP data span from the workspace.
template <int NX>
__device__ __forceinline__ void stage_lin(const Prob& P, const ProbRec& pr, const float* data,
                                          bool qp) {
  copy_block<false>(const_cast<float*>(P.costp), data + pr.cost_off,
                    (int)cost_block_len(P.T, NX, P.m, P.cost, P.phases, P.nw));
  if (P.dyn == DMPC_DYN_LTV)
    copy_block<false>(const_cast<float*>(P.A), data + pr.dyn_off,
                      (int)dyn_block_len(P.T, NX, P.m, P.dyn));
  // (the span rounded up to 4 floats stays inside both regions)
  if (qp) copy_block<true>(P.Wq, P.W, (int)a4h(lin_span(P.T, NX, P.m, P.dyn)));
}

// Linearised dynamics entries in precision R: the double copy where one
// exists (nonlinear models), else the float data (exact for LTV inputs).
template <typename R>
__device__ __forceinline__ R ldA(const Prob& P, int idx) {
  if constexpr (sizeof(R) == sizeof(double)) {
    if (P.Ad) return P.Ad[idx];
  }
  return (R)P.A[idx];
}
template <typename R>
__device__ __forceinline__ R ldB(const Prob& P, int idx) {
  if constexpr (sizeof(R) == sizeof(double)) {
    if (P.Bd) return P.Bd[idx];
  }
  return (R)P.B[idx];
}
template <typename R>
__device__ __forceinline__ R ldc(const Prob& P, int idx) {
  if constexpr (sizeof(R) == sizeof(double)) {
    if (P.cd) return P.cd[idx];
  }
  return (R)P.c[idx];
}

// Row passes over the Schur rows: the entries of A a row needs, for U rows
// rho = base + u BT of a thread at once, every load issued before any is
// used (the passes are bound by the latency of these loads, and a row at a
// time leaves one row's loads in flight).  Row index r = rho - off of the
// stacked blocks A_t (row-major [T][NX][NX]): COL takes column i of block t
// = r / NX (entries A_t[k][i]), else row r (entries A_t[i][k]); rows outside
// [0, lim) read block 0 and the caller discards them.  Float data (LTV).
template <int NX, int U, bool COL>
__device__ __forceinline__ void gather_A(const float* A, int base, int BT, int off, int lim,
                                         float (&a)[U][NX]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = base + u * BT - off;
    const bool ok = r >= 0 && r < lim;
    const int t = r / NX, i = r - t * NX;
    const float* s = A + (ok ? (COL ? t * NX * NX + i : r * NX) : 0);
#pragma unroll
    for (int k = 0; k < NX; ++k) a[u][k] = s[COL ? k * NX : k];
  }
}
// rows gathered at once: at most 32 floats of A per thread (the passes are
// calls with at most 128 registers; one row at nx = 32)
template <int NX>
constexpr int gather_rows() { return NX >= 32 ? 1 : (NX >= 12 ? 2 : (NX >= 8 ? 4 : 8)); }

__device__ __forceinline__ float softplusf(float v) {
  return v > 20.f ? v : log1pf(expf(v));
}
__device__ __forceinline__ float sigmoidf(float v) { return 1.f / (1.f + expf(-v)); }

// Softplus cost: index of theta/wscale for stage t, component j of the
// weight vector (j < nw: state j; nw <= j < nw+m: input j-nw).
__device__ __forceinline__ int sp_phase(const Prob& P, int t) {
  const int k = (P.phases * t) / P.T;
  return k < P.phases - 1 ? k : P.phases - 1;
}
// learned weight j of stage t
__device__ __forceinline__ float sp_weight(const Prob& P, int t, int j) {
  const int K = P.nw + P.m;
  const float* th = P.costp;
  const float* ws = th + P.phases * K;
  return ws[j] * softplusf(th[sp_phase(P, t) * K + j]);
}
// state weight of stage t (learned or fixed)
template <int NX>
__device__ __forceinline__ float sp_wx(const Prob& P, int t, int i) {
  if (i < P.nw) return sp_weight(P, t, i);
  const int K = P.nw + P.m;
  const float* wfix = P.costp + P.phases * K + K;
  return wfix[i - P.nw];
}
template <int NX>
__device__ __forceinline__ const float* sp_xref(const Prob& P) {
  const int K = P.nw + P.m;
  return P.costp + P.phases * K + K + (NX - P.nw);
}

// Stage costs at a point (the true costs, as used by the merit function),
// evaluated in double.
template <int NX>
__device__ __forceinline__ double cost_x(const Prob& P, int t, const double* x, int cost_kind) {
  double s = 0.0;
  if (cost_kind == DMPC_COST_DIAG) {
    const float* Qd = P.costp + t * NX;
    const float* q = P.costp + P.N * NX + t * NX;
#pragma unroll
    for (int i = 0; i < NX; ++i) s += 0.5 * (double)Qd[i] * x[i] * x[i] + (double)q[i] * x[i];
  } else {
    const float* xr = sp_xref<NX>(P);
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const double d = x[i] - (double)xr[i];
      s += 0.5 * (double)sp_wx<NX>(P, t, i) * d * d;
    }
  }
  return s;
}
template <int NX>
__device__ __forceinline__ double cost_u1(const Prob& P, int t, int l, double u, int cost_kind) {
  if (cost_kind == DMPC_COST_DIAG) {
    const float* Rd = P.costp + 2 * P.N * NX + t * P.m;
    const float* r = Rd + P.TM;
    return 0.5 * (double)Rd[l] * u * u + (double)r[l] * u;
  }
  return 0.5 * (double)sp_weight(P, t, P.nw + l) * u * u;
}
// directional derivative of the stage costs: grad c(xb)'(xq - xb)
template <int NX>
__device__ __forceinline__ double dcost_x(const Prob& P, int t, const float* xb, const float* xq,
                                          int cost_kind) {
  double s = 0.0;
  if (cost_kind == DMPC_COST_DIAG) {
    const float* Qd = P.costp + t * NX;
    const float* q = P.costp + P.N * NX + t * NX;
#pragma unroll
    for (int i = 0; i < NX; ++i)
      s += ((double)Qd[i] * xb[i] + (double)q[i]) * ((double)xq[i] - (double)xb[i]);
  } else {
    const float* xr = sp_xref<NX>(P);
#pragma unroll
    for (int i = 0; i < NX; ++i)
      s += (double)sp_wx<NX>(P, t, i) * ((double)xb[i] - (double)xr[i]) *
           ((double)xq[i] - (double)xb[i]);
  }
  return s;
}
template <int NX>
__device__ __forceinline__ double dcost_u1(const Prob& P, int t, int l, float ub, float uq,
                                           int cost_kind) {
  if (cost_kind == DMPC_COST_DIAG) {
    const float* Rd = P.costp + 2 * P.N * NX + t * P.m;
    const float* r = Rd + P.TM;
    return ((double)Rd[l] * ub + (double)r[l]) * ((double)uq - (double)ub);
  }
  return (double)sp_weight(P, t, P.nw + l) * ub * ((double)uq - (double)ub);
}

// State cost of one row (t, i) and its directional derivative: the stage
// costs above are sums of these over i.
template <int NX>
__device__ __forceinline__ double cost_x1(const Prob& P, int t, int i, double x, int cost_kind) {
  if (cost_kind == DMPC_COST_DIAG) {
    const double qd = P.costp[t * NX + i], q = P.costp[P.N * NX + t * NX + i];
    return 0.5 * qd * x * x + q * x;
  }
  const double d = x - (double)sp_xref<NX>(P)[i];
  return 0.5 * (double)sp_wx<NX>(P, t, i) * d * d;
}
template <int NX>
__device__ __forceinline__ double dcost_x1(const Prob& P, int t, int i, double xb, double dx,
                                           int cost_kind) {
  if (cost_kind == DMPC_COST_DIAG) {
    const double qd = P.costp[t * NX + i], q = P.costp[P.N * NX + t * NX + i];
    return (qd * xb + q) * dx;
  }
  return (double)sp_wx<NX>(P, t, i) * (xb - (double)sp_xref<NX>(P)[i]) * dx;
}

// Parameters of a nonlinear model, loaded once per phase into registers
// (through the scalar unit: the block is the same for the whole workgroup).
struct ModelPar {
  float v[kBicycleParams];
};
__device__ __forceinline__ ModelPar load_par(const Prob& P) {
  ModelPar mp;
  const uint64_t a = (uint64_t)P.dynp;
  const float* dp = (const float*)(((uint64_t)__builtin_amdgcn_readfirstlane((int)(a >> 32)) << 32) |
                                   (uint32_t)__builtin_amdgcn_readfirstlane((int)a));
#pragma unroll
  for (int i = 0; i < kBicycleParams; ++i) mp.v[i] = 0.f;
  // (whole blocks of unconditional loads: one wait for all of them)
  if (P.dyn == DMPC_DYN_CARTPOLE) {
#pragma unroll
    for (int i = 0; i < kCartpoleParams; ++i) mp.v[i] = dp[i];
  } else if (P.dyn == DMPC_DYN_BICYCLE) {
#pragma unroll
    for (int i = 0; i < kBicycleParams; ++i) mp.v[i] = dp[i];
  }
  return mp;
}

// Next state of the true dynamics, in double (rollout and merit function).
template <int NX>
__device__ __forceinline__ void dyn_step(const Prob& P, const ModelPar& mp, int t,
                                         const double* x, const double* u, double* xn,
                                         int dyn_kind) {
  if (dyn_kind == DMPC_DYN_LTV) {
    const float* At = P.A + t * NX * NX;
    const float* Bt = P.B + t * NX * P.m;
    const float* ct = P.c + t * NX;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      double s = ct[i];
#pragma unroll
      for (int j = 0; j < NX; ++j) s += (double)At[i * NX + j] * x[j];
      for (int l = 0; l < P.m; ++l) s += (double)Bt[i * P.m + l] * u[l];
      xn[i] = s;
    }
    return;
  }
  if constexpr (NX == 4) {
    if (dyn_kind == DMPC_DYN_CARTPOLE) {
      cartpole_step<double>(mp.v, x, u, xn);
      return;
    }
  }
  if constexpr (NX == 8) {
    if (dyn_kind == DMPC_DYN_BICYCLE) {
      bicycle_step<double>(mp.v, x, u, xn);
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < NX; ++i) xn[i] = __builtin_nan("");
}

// Jacobians of a nonlinear model at (xb, ub) by forward-mode duals in double;
// writes A_t [NX][NX], B_t [NX][MU] and the offset c_t = phi(xb, ub) - A xb
// - B ub (so that the affine model passes through phi at the linearisation
// point), each in double and rounded to float; c_t is formed in double with
// the double Jacobians.
template <int NX, int MU, typename F>
__device__ __forceinline__ void linearize_model(F step, const float* par, const float* xb,
                                                const float* ub, float* A, float* B, float* c,
                                                double* Ad, double* Bd, double* cd) {
  constexpr int K = NX + MU;
  typedef Dual<K, double> D;
  D x[NX], u[MU], xn[NX];
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    x[j] = mkconst<K, double>((double)xb[j]);
    x[j].d[j] = 1.0;
  }
#pragma unroll
  for (int l = 0; l < MU; ++l) {
    u[l] = mkconst<K, double>((double)ub[l]);
    u[l].d[NX + l] = 1.0;
  }
  step(par, x, u, xn);
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    double s = xn[i].v;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      A[i * NX + j] = (float)xn[i].d[j];
      Ad[i * NX + j] = xn[i].d[j];
      s -= xn[i].d[j] * (double)xb[j];
    }
#pragma unroll
    for (int l = 0; l < MU; ++l) {
      B[i * MU + l] = (float)xn[i].d[NX + l];
      Bd[i * MU + l] = xn[i].d[NX + l];
      s -= xn[i].d[NX + l] * (double)ub[l];
    }
    c[i] = (float)s;
    cd[i] = s;
  }
}

template <int NX>
struct CartpoleStepF {
  template <typename S>
  __device__ __forceinline__ void operator()(const float* p, const S* x, const S* u, S* xn) const {
    cartpole_step<S>(p, x, u, xn);
  }
};
template <int NX>
struct BicycleStepF {
  template <typename S>
  __device__ __forceinline__ void operator()(const float* p, const S* x, const S* u, S* xn) const {
    bicycle_step<S>(p, x, u, xn);
  }
};

// ===========================================================================
// QP data (Eq. QPmatrices) at the iterate held in LDS
// ===========================================================================
template <int NX>
__device__ __forceinline__ void form_qp(const Prob& P, const float* xbar, const float* ubar,
                                        bool first) {
  const int tid = threadIdx.x, BT = blockDim.x;
  float* W = P.Wq;
  float* Qd = W + P.L.Qd;
  float* iQ = W + P.L.iQ;
  float* q = W + P.L.q;
  float* Rd = W + P.L.Rd;
  float* iR = W + P.L.iR;
  float* r = W + P.L.r;
  double* iQd = (double*)(W + P.L.iQd);
  double* iRd = (double*)(W + P.L.iRd);
  // cost Hessians projected onto {H >= eps I} and linear terms
  // q = grad c(xb) - Q_proj xb  (written so that q = q_raw exactly when no clamp)
  if (P.cost == DMPC_COST_DIAG && !first) {
    // diagonal costs: the Hessians (and their reciprocals) do not depend on
    // the iterate and stay from the first SQP iteration; only the linear
    // terms of clamped entries do
    for (int idx = tid; idx < P.R; idx += BT)
      q[idx] = P.costp[P.R + idx] + (P.costp[idx] - Qd[idx]) * xbar[idx];
    for (int idx = tid; idx < P.TM; idx += BT)
      r[idx] = P.costp[2 * P.R + P.TM + idx] + (P.costp[2 * P.R + idx] - Rd[idx]) * ubar[idx];
  } else {
  for (int idx = tid; idx < P.R; idx += BT) {
    const int t = idx / NX, i = idx - t * NX;
    float h, qq;
    if (P.cost == DMPC_COST_DIAG) {
      h = P.costp[idx];
      qq = P.costp[P.R + idx];
    } else {
      h = sp_wx<NX>(P, t, i);
      qq = -h * sp_xref<NX>(P)[i];
    }
    const float hp = fmaxf(h, kPdEps);
    Qd[idx] = hp;
    iQ[idx] = 1.f / hp;
    iQd[idx] = 1.0 / (double)hp;
    q[idx] = qq + (h - hp) * xbar[idx];
  }
  for (int idx = tid; idx < P.TM; idx += BT) {
    const int t = idx / P.m, l = idx - t * P.m;
    float h, rr;
    if (P.cost == DMPC_COST_DIAG) {
      h = P.costp[2 * P.R + idx];
      rr = P.costp[2 * P.R + P.TM + idx];
    } else {
      h = sp_weight(P, t, P.nw + l);
      rr = 0.f;
    }
    const float hp = fmaxf(h, kPdEps);
    Rd[idx] = hp;
    iR[idx] = 1.f / hp;
    iRd[idx] = 1.0 / (double)hp;
    r[idx] = rr + (h - hp) * ubar[idx];
  }
  }
  // dynamics Jacobians for nonlinear models, one thread per stage
  if (P.dyn != DMPC_DYN_LTV) {
    float* A = W + P.L.A;
    float* B = W + P.L.B;
    float* c = W + P.L.c;
    double* Ad = (double*)(W + P.L.Ad);
    double* Bd = (double*)(W + P.L.Bd);
    double* cd = (double*)(W + P.L.cd);
    const ModelPar mp = load_par(P);
    for (int t = tid; t < P.T; t += BT) {
      if constexpr (NX == 4) {
        if (P.dyn == DMPC_DYN_CARTPOLE)
          linearize_model<4, 1>(CartpoleStepF<4>(), mp.v, xbar + t * 4, ubar + t, A + t * 16,
                                B + t * 4, c + t * 4, Ad + t * 16, Bd + t * 4, cd + t * 4);
      }
      if constexpr (NX == 8) {
        if (P.dyn == DMPC_DYN_BICYCLE)
          linearize_model<8, 2>(BicycleStepF<8>(), mp.v, xbar + t * 8, ubar + t * 2,
                                A + t * 64, B + t * 16, c + t * 8, Ad + t * 64, Bd + t * 16,
                                cd + t * 8);
      }
    }
  }
}

// ===========================================================================
// Schur rows (Eq. shurcomplement, Eq. S_Phiinv; user signs), float or double
//   D_0 = Q_0^-1,  D_{t+1} = A_t Q_t^-1 A_t' + B_t R_t^-1 B_t' + Q_{t+1}^-1
//   E_{t+1,t} = -A_t Q_t^-1,  E_{t,t+1} = E_{t+1,t}'
//   g = -gamma:  g_0 = -(x_s + Q_0^-1 q_0),
//   g_{t+1} = -(c_t - A_t Q_t^-1 q_t - B_t R_t^-1 r_t + Q_{t+1}^-1 q_{t+1})
// S[0:NX] = E_{t,t-1}[i,:], S[NX:2NX] = D_t[i,:], S[2NX:3NX] = E_{t,t+1}[i,:]
// Both versions read the reciprocals of the projected Hessian diagonal that
// form_qp stores, in float and in double.
// ===========================================================================
template <typename R>
__device__ __forceinline__ R rinv(const float* ih, const double* ihd, int idx) {
  if constexpr (sizeof(R) == sizeof(float)) {
    return ih[idx];
  } else {
    return ihd[idx];
  }
}

template <int NX, typename R, bool SKIP_D = false>
__device__ __forceinline__ void schur_row(const Prob& P, int t, int i, R* S, R& g) {
  const float* W = P.Wq;
  const float* iQ = W + P.L.iQ;
  const float* q = W + P.L.q;
  const float* iR = W + P.L.iR;
  const float* r = W + P.L.r;
  const double* iQd = (const double*)(W + P.L.iQd);
  const double* iRd = (const double*)(W + P.L.iRd);
  const int m = P.m;
#pragma unroll
  for (int j = 0; j < 3 * NX; ++j) S[j] = R(0);
  if (t == 0) {
    const R d = rinv<R>(iQ, iQd, i);
#pragma unroll
    for (int j = 0; j < NX; ++j) S[NX + j] = (j == i) ? d : R(0);
    g = -((R)P.x0[i] + (R)q[i] * d);
  } else {
    const int tt = t - 1;
    const int a0 = tt * NX * NX, b0 = tt * NX * m;
    R ai[NX];
    R gs = R(0);
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      ai[j] = ldA<R>(P, a0 + i * NX + j) * rinv<R>(iQ, iQd, tt * NX + j);
      gs += ai[j] * (R)q[tt * NX + j];
      S[j] = -ai[j];
    }
    if constexpr (!SKIP_D) {
#pragma unroll
      for (int k = 0; k < NX; ++k) {
        R acc = R(0);
#pragma unroll
        for (int j = 0; j < NX; ++j) acc += ai[j] * ldA<R>(P, a0 + k * NX + j);
        S[NX + k] = acc;
      }
    }
    for (int l = 0; l < m; ++l) {
      const R bi = ldB<R>(P, b0 + i * m + l) * rinv<R>(iR, iRd, tt * m + l);
      gs += bi * (R)r[tt * m + l];
      if constexpr (!SKIP_D) {
#pragma unroll
        for (int k = 0; k < NX; ++k) S[NX + k] += bi * ldB<R>(P, b0 + k * m + l);
      }
    }
    const R dq = rinv<R>(iQ, iQd, t * NX + i);
    if constexpr (!SKIP_D) {
#pragma unroll
      for (int k = 0; k < NX; ++k) S[NX + k] += (k == i) ? dq : R(0);
    }
    g = -(ldc<R>(P, tt * NX + i) - gs + (R)q[t * NX + i] * dq);
  }
  if (t < P.T) {
    const int a0 = t * NX * NX;
    const R d = rinv<R>(iQ, iQd, t * NX + i);
#pragma unroll
    for (int k = 0; k < NX; ++k) S[2 * NX + k] = -ldA<R>(P, a0 + k * NX + i) * d;
  }
}

// The right-hand side entry g (row (t, i)) of schur_row alone: for problems
// whose QP matrices do not change between SQP iterations only the linear
// terms (and with them g) move.  Ai: row i of A_{t-1} (t > 0), gathered by
// the caller.
template <int NX>
__device__ __forceinline__ float schur_rhs_row(const Prob& P, int t, int i, const float* Ai) {
  const float* W = P.Wq;
  const float* iQ = W + P.L.iQ;
  const float* q = W + P.L.q;
  const float* iR = W + P.L.iR;
  const float* r = W + P.L.r;
  const int m = P.m;
  if (t == 0) return -(P.x0[i] + q[i] * iQ[i]);
  const int tt = t - 1;
  const int b0 = tt * NX * m;
  float gs = 0.f;
#pragma unroll
  for (int j = 0; j < NX; ++j) gs += (Ai[j] * iQ[tt * NX + j]) * q[tt * NX + j];
  for (int l = 0; l < m; ++l) gs += (P.B[b0 + i * m + l] * iR[tt * m + l]) * r[tt * m + l];
  return -(P.c[tt * NX + i] - gs + q[t * NX + i] * iQ[t * NX + i]);
}

// Right-hand side of the adjoint Schur system (the first step of Alg. backward, with
// (-b, d) <- (dl/dz, dl/dlambda)):  g~ = H G^-1 dl/dz - dl/dlambda, row (t, i).
// Ai: row i of A_{t-1} gathered by the caller, or null to read it here.
template <int NX, typename R>
__device__ __forceinline__ R adjoint_rhs_row(const Prob& P, int t, int i, const float* dlx,
                                             const float* dlu, const float* dll,
                                             const float* Ai = nullptr) {
  const float* iQ = P.Wq + P.L.iQ;
  const float* iR = P.Wq + P.L.iR;
  const double* iQd = (const double*)(P.Wq + P.L.iQd);
  const double* iRd = (const double*)(P.Wq + P.L.iRd);
  const int m = P.m;
  const int rho = t * NX + i;
  R v = (R)dlx[rho] * rinv<R>(iQ, iQd, rho) - (R)dll[rho];
  if (t >= 1) {
    const int tt = t - 1;
    const int a0 = tt * NX * NX + i * NX, b0 = tt * NX * m + i * m;
#pragma unroll
    for (int j = 0; j < NX; ++j)
      v -= (Ai ? (R)Ai[j] : ldA<R>(P, a0 + j)) * ((R)dlx[tt * NX + j] * rinv<R>(iQ, iQd, tt * NX + j));
    for (int l = 0; l < m; ++l)
      v -= ldB<R>(P, b0 + l) * ((R)dlu[tt * m + l] * rinv<R>(iR, iRd, tt * m + l));
  }
  return v;
}

// Storage of the Schur and preconditioner rows in the workspace: row-major,
// 6 NX coefficients per row (S^ row, then Phi^-1 row).  (A layout in tiles of
// 64 rows, coefficient-major, made the wave's loads contiguous but measured
// two to four times slower on the workspace-row kernels.)
template <int NX>
__device__ __forceinline__ int64_t blk_at(int rho, int j) {
  return (int64_t)rho * (6 * NX) + j;
}

// Row product with a padded LDS window: sum_j coef[j] * win[j], win = w + t*NX.
// For NX a multiple of 4 the window is 16-byte aligned (windows start on
// 4-float boundaries) and is read with 128-bit LDS loads.
template <int NX>
__device__ __forceinline__ float row_dot(const float* coef, const float* win) {
  float wv[3 * NX];
  if constexpr (NX % 4 == 0) {
    const float4* w4 = reinterpret_cast<const float4*>(win);
#pragma unroll
    for (int j = 0; j < 3 * NX / 4; ++j) {
      const float4 v = w4[j];
      wv[4 * j] = v.x;
      wv[4 * j + 1] = v.y;
      wv[4 * j + 2] = v.z;
      wv[4 * j + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 3 * NX; ++j) wv[j] = win[j];
  }
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    a0 = fmaf(coef[j], wv[j], a0);
    a1 = fmaf(coef[NX + j], wv[NX + j], a1);
    a2 = fmaf(coef[2 * NX + j], wv[2 * NX + j], a2);
  }
  return (a0 + a1) + a2;
}
// Row product with the coefficients read from the workspace (row-major).  The coefficients do not change during the
// PCG, so the compiler hoists their loads out of the loop and keeps what it
// can in registers (the rest in AGPRs and swizzled scratch): measured faster
// than re-reading the rows for nx <= 16.  For nx = 32 that would keep
// 6 x 32 values per row live, so there the row address passes through an
// empty asm at each product and the rows are re-read every iteration.
template <int NX>
__device__ __forceinline__ float row_dot_ws(const float* coef, const float* win) {
  if constexpr (NX <= 16) {
    return row_dot<NX>(coef, win);
  }
  uint64_t a = (uint64_t)(uintptr_t)coef;
  asm volatile("" : "+v"(a));
  // rows are 6 NX floats and the workspace is 256-byte aligned: 16-byte loads
  const float4* c4 = (const float4*)(uintptr_t)a;
  const float4* w4 = reinterpret_cast<const float4*>(win);
  float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int b = 0; b < 3; ++b) {
#pragma unroll
    for (int j = 0; j < NX / 4; ++j) {
      const float4 c = c4[b * (NX / 4) + j];
      const float4 v = w4[b * (NX / 4) + j];
      acc[b] = fmaf(c.x, v.x, acc[b]);
      acc[b] = fmaf(c.y, v.y, acc[b]);
      acc[b] = fmaf(c.z, v.z, acc[b]);
      acc[b] = fmaf(c.w, v.w, acc[b]);
    }
  }
  return (acc[0] + acc[1]) + acc[2];
}

// Same with the window value taken as the double-float hi + lo.
template <int NX>
__device__ __forceinline__ double row_dot64(const double* coef, const float* hi, const float* lo) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    a0 = fma(coef[j], (double)hi[j] + (double)lo[j], a0);
    a1 = fma(coef[NX + j], (double)hi[NX + j] + (double)lo[NX + j], a1);
    a2 = fma(coef[2 * NX + j], (double)hi[2 * NX + j] + (double)lo[2 * NX + j], a2);
  }
  return (a0 + a1) + a2;
}

// ===========================================================================
// Shared-memory layout of a workgroup (float offsets)
// ===========================================================================
template <int NX>
__device__ __forceinline__ Carve carve_of(const Prob& P) {
  return carve(P.R, P.TM, P.N, NX, blockDim.x, P.slots, P.flags);
}
// Base of the bulk regions.
__device__ __forceinline__ float* bulk_base(float* smem, const Prob& P) {
  return (P.flags & kRecBulkWs) ? P.W + P.L.bulk : smem;
}

// Zeroes the pads of the three windows: [0, nx) and [R + nx, window end).
template <int NX>
__device__ __forceinline__ void zero_pads(float* smem, const Carve& C, const Prob& P) {
  const int wl = (int)win_floats(P.R, NX, blockDim.x, P.slots, P.flags);
  const int R = P.R;
  for (int i = threadIdx.x; i < NX + (wl - R - NX); i += blockDim.x) {
    const int o = i < NX ? i : R + i;
    smem[C.w0 + o] = 0.f;
    smem[C.w1 + o] = 0.f;
    smem[C.w2 + o] = 0.f;
  }
}

struct Lds {
  float* w0;   // padded windows: w[NX + rho] = v[rho], zero pads of NX at both ends
  float* w1;
  float* w2;   // low part of the vector in w0 (double-float multipliers)
  float* piv;  // Gauss-Jordan pivot rows, double buffered
  float* red;  // 2 x 64 floats for block reductions
  float* dinv; // kRecDinvLds: row rho of D_t^-1 at dinv + rho NX
  float* tail; // kRecTailLds: Schur row (s - 1) BT + k of the last slot s at tail + k stride
};

template <int NX>
__device__ __forceinline__ Lds lds_of(float* smem, const Prob& P) {
  const Carve C = carve_of<NX>(P);
  Lds sh;
  sh.w0 = smem + C.w0;
  sh.w1 = smem + C.w1;
  sh.w2 = smem + C.w2;
  sh.piv = smem + C.piv;
  sh.red = smem + C.red;
  sh.dinv = smem + C.dinv;
  sh.tail = smem + C.tail;
  return sh;
}

// Row guard of slot s.  With FULL (register-resident rows, which are zero
// past R, as is every vector entry there) every row of every slot runs, with
// no branch: rows past R compute zeros into the window's tail pad.
template <bool FULL>
__device__ __forceinline__ bool row_live(int s, int rho, int R, int BT) {
  if constexpr (FULL) return true;
  return rho < R;
}

// Row of the s-th value a thread holds.  Standard layout: rho = tid + s BT.
// Wave-block layout (one wave per problem, a lane per stage block): value
// s = b NX + i of lane l is row i of block l + 64 b.
template <int NX, bool WAVE>
__device__ __forceinline__ int row_of(int s, int tid, int BT) {
  if constexpr (WAVE) return (tid + 64 * (s / NX)) * NX + (s % NX);
  return tid + s * BT;
}

// Threads of the workgroup: LDS-row kernels (TAIL) run with kTailThreads, a
// compile-time constant there, so that per-slot row offsets are immediates.
template <bool TAIL>
__device__ __forceinline__ int block_threads() {
  if constexpr (TAIL) return kTailThreads;
  return blockDim.x;
}
// Thread index for the row products of the PCG loop.  TAIL: read through an
// empty asm, so that the LDS addresses derived from it are formed where they
// are used instead of being hoisted out of the loop and held (the rows need
// those registers).
template <bool TAIL>
__device__ __forceinline__ int loop_tid() {
  int tid = threadIdx.x;
  if constexpr (TAIL) asm volatile("" : "+v"(tid));
  return tid;
}

// (TAIL: the last slot's rows are in LDS and guarded, the others as FULL says)
template <int NX, int SLOTS, bool FULL = false, bool WAVE = false, bool TAIL = false>
__device__ __forceinline__ void publish(float* w, const float (&v)[SLOTS], int R) {
  const int tid = loop_tid<TAIL>(), BT = block_threads<TAIL>();
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int rho = row_of<NX, WAVE>(s, tid, BT);
    const bool full = FULL && !(TAIL && s == SLOTS - 1);
    if (full || rho < R) w[NX + rho] = v[s];
  }
}

// Orders a wave's LDS stores before its later LDS loads of other lanes' data
// (a wave executes its LDS instructions in order; this keeps the compiler
// from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Double-precision matrix-core product of 16 x 16 x 4 tiles: lane (q, c)
// (q = lane / 16, c = lane % 16) supplies A[c][k_q] and B[k_q][c], where k_q
// is the contraction index its lane group stands for in this step; item r of
// the result is D[4 r + q][c] (rows interleaved across the lane groups,
// unlike the single-precision 16 x 16 x 4 tile, whose item r is row 4 q + r).
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ mfma_d4 mfma16d(double a, double b, mfma_d4 acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

// Scaled off-diagonal blocks E~_{t,t-1} = L_t^-1 S_{t,t-1} L_{t-1}^-T for
// t = 1..T (nx <= 16, padded to 16 with zeros), one wave per stage:
// Y = S_{t,t-1} L_{t-1}^-T, then L_t^-1 Y.  Step s of either product lets
// lane group q stand for index 4 s + q, so that the B operand of the second
// product, Y[4 s + q][c], is item s of the lane's own result of the first.
// Writes E~_{t,t-1} to coefficients 3 nx .. 4 nx of the rows of stage t and
// its transpose E~_{t-1,t} to coefficients 4 nx .. 5 nx of the rows of stage
// t - 1.  Lid: L_t^-1, double, row-major per stage.
template <int NX>
__device__ __forceinline__ void mfma_scaled_offdiag(const Prob& P, float* blk, const double* Lid) {
  static_assert(NX <= 16, "one 16 x 16 tile per block");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const bool cin = c < NX;
  const int cc = cin ? c : 0;
  for (int t = 1 + w; t < P.N; t += W) {
    const float* St = blk + blk_at<NX>(t * NX + cc, 0);         // row c of S_{t,t-1}
    const double* Lp = Lid + ((int64_t)(t - 1) * NX + cc) * NX;  // row c of L_{t-1}^-1
    const double* Lt = Lid + ((int64_t)t * NX + cc) * NX;        // row c of L_t^-1
    mfma_d4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + q;
      const bool ok = cin && k < NX;
      y = mfma16d(ok ? (double)St[k] : 0.0, ok ? Lp[k] : 0.0, y);
    }
    mfma_d4 e = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + q;
      const bool ok = cin && k < NX;
      e = mfma16d(ok ? Lt[k] : 0.0, y[s], e);
    }
    if (cin) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * r + q;
        if (i < NX) {
          const float v = (float)e[r];
          blk[blk_at<NX>(t * NX + i, 3 * NX + c)] = v;
          blk[blk_at<NX>((t - 1) * NX + c, 4 * NX + i)] = v;
        }
      }
    }
  }
}

// ===========================================================================
// Scaled Schur system (kRecScaled).  With D_t = L_t L_t' (Cholesky, in double
// from the float blocks) and L = blkdiag(L_t), the PCG of Alg. pcg on S^
// with the stair preconditioner Phi^-1 = D^-1 - D^-1 E D^-1 (Eq. S_Phiinv)
// is the same iteration, in the variables x~ = L' x, as the PCG on
// L^-1 S^ L^-T = I + E~ with the preconditioner L' Phi^-1 L = I - E~, where
// E~_{t,t-1} = L_t^-1 S_{t,t-1} L_{t-1}^-T (and E~_{t-1,t} its transpose):
// the same step lengths and the same stopping test (r'Phi^-1 r is unchanged).
// A row then needs only its two scaled off-diagonal blocks.  Writes L_t^-1
// (double, row-major per stage) to the Lid region and row rho of E~ (the
// blocks at t-1 and t+1) to coefficients 3 nx .. 5 nx of the saved row.
// xch: LDS exchange of BT doubles.  Returns true (in every thread) on a
// non-positive pivot.
// ===========================================================================
template <int NX>
__device__ __forceinline__ bool scaled_blocks(const Prob& P, double* xch) {
  // a stage's NX rows are consecutive threads of one group of BT rows (the
  // host launches these kernels with BT a multiple of nx); when nx divides
  // the wave size they are lanes of one wave and exchange under wave-level
  // ordering, otherwise through workgroup barriers
  constexpr bool STAGE_IN_WAVE = 64 % NX == 0;
  auto sync = [] {
    if constexpr (STAGE_IN_WAVE) wave_sync();
    else __syncthreads();
  };
  const int tid = threadIdx.x, BT = blockDim.x, R = P.R;
  const int N = P.N;
  float* blk = P.W + P.L.blk;
  double* Lid = (double*)(P.W + P.L.Lid);
  double* xg = xch + (tid / NX) * NX;   // exchange row of this thread's stage group
  double* xr = xg + BT;                  // reciprocals of the pivots (the region holds 2 BT)
  int bad = 0;
  // (1), (2) per group of BT rows (whole stages); rows past R factor
  // identity blocks and store nothing
  for (int base = 0; base < R; base += BT) {
    const int rho = base + tid;
    const bool live = rho < R;
    const int t = rho / NX, i = rho - t * NX;
    double a[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j)
      a[j] = live ? (double)blk[blk_at<NX>(rho, NX + j)] : (j == i ? 1.0 : 0.0);
    // Cholesky, one column per step: lane i ends with row i of L_t in a[0..i];
    // the pivot lane publishes L_kk and 1 / L_kk, so that the column is a
    // product (the division leaves the step's dependent chain)
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      if (i == k) {
        if (!(a[k] > 0.0)) bad = 1;
        const double l = sqrt(a[k] > 0.0 ? a[k] : 1.0);
        xg[k] = l;
        xr[k] = 1.0 / l;
      }
      sync();
      const double lkk = xg[k];
      if (i == k) a[k] = lkk;
      if (i > k) {
        a[k] *= xr[k];
        xg[i] = a[k];
      }
      sync();
#pragma unroll
      for (int j = k + 1; j < NX; ++j)
        if (j <= i) a[j] -= a[k] * xg[j];
      sync();
    }
    // L_t^-1 by columns: lane i gets column i (x[m], zero for m < i); row m
    // of L_t comes from lane m through the exchange row
    double x[NX];
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      if (i == m) {
#pragma unroll
        for (int q = 0; q <= m; ++q) xg[q] = a[q];
      }
      sync();
      double acc = m == i ? 1.0 : 0.0;
#pragma unroll
      for (int q = 0; q < m; ++q) acc -= xg[q] * x[q];
      x[m] = m < i ? 0.0 : acc * xr[m];
      sync();
    }
    if (live) {
#pragma unroll
      for (int m = 0; m < NX; ++m) Lid[((int64_t)t * NX + m) * NX + i] = x[m];
    }
  }
  __syncthreads();
  // (3) E~_{t,t-1} = L_t^-1 S_{t,t-1} L_{t-1}^-T on the matrix cores, and
  // E~_{t-1,t} as its transpose; the blocks past either end are zero
  mfma_scaled_offdiag<NX>(P, blk, Lid);
  for (int rho = tid; rho < NX; rho += BT) {
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      blk[blk_at<NX>(rho, 3 * NX + j)] = 0.f;
      blk[blk_at<NX>((N - 1) * NX + rho, 4 * NX + j)] = 0.f;
    }
  }
  return __syncthreads_or(bad) != 0;
}

// ===========================================================================
// Symmetric stair preconditioner (Eq. S_Phiinv): Gauss-Jordan inversion of
// every D_t (rows of a block are handled by consecutive threads; the rows are
// processed in chunks of whole blocks), then the off-diagonal blocks
// -D_t^-1 E_{t,t-1} D_{t-1}^-1 and -D_t^-1 E_{t,t+1} D_{t+1}^-1.  Reads the
// diagonal-block rows from coefficients NX..2NX-1 of blk and writes the
// preconditioner rows to coefficients 3NX..6NX-1.  Returns true (in this
// thread) on a
// non-positive pivot.
// ===========================================================================
// Gauss-Jordan inversion of one diagonal block in registers: b = a^-1 (a is
// destroyed).  Returns true on a non-positive pivot (then taken as 1).
template <int NX>
__device__ __forceinline__ bool gj_invert(float (&a)[NX][NX], float (&b)[NX][NX]) {
  bool nonpd = false;
#pragma unroll
  for (int i = 0; i < NX; ++i)
#pragma unroll
    for (int j = 0; j < NX; ++j) b[i][j] = (i == j) ? 1.f : 0.f;
#pragma unroll
  for (int kk = 0; kk < NX; ++kk) {
    float pv = a[kk][kk];
    if (!(pv > 0.f)) {
      nonpd = true;
      pv = 1.f;
    }
    const float inv = 1.f / pv;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      a[kk][j] *= inv;
      b[kk][j] *= inv;
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      if (i == kk) continue;
      const float f = a[i][kk];
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        a[i][j] = fmaf(-f, a[kk][j], a[i][j]);
        b[i][j] = fmaf(-f, b[kk][j], b[i][j]);
      }
    }
  }
  return nonpd;
}

template <int NX>
__device__ __forceinline__ bool precond_rows(const Prob& P, float* piv) {
  const int tid = threadIdx.x, BT = blockDim.x;
  const int nb = BT / NX;        // whole blocks per chunk
  const int BTb = nb * NX;
  float* blk = P.W + P.L.blk;
  float* Dinv = P.W + P.L.Dinv;
  const float* iQ = P.Wq + P.L.iQ;
  bool nonpd = false;
  if constexpr (NX <= 8) {
    // small blocks: one thread inverts a whole D_t in registers (the same
    // operations in the same order as the row-parallel elimination below)
    for (int t = tid; t < P.N; t += BT) {
      float a[NX][NX], b[NX][NX];
#pragma unroll
      for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) a[i][j] = blk[blk_at<NX>(t * NX + i, NX + j)];
      if (gj_invert<NX>(a, b)) nonpd = true;
#pragma unroll
      for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) Dinv[(t * NX + i) * NX + j] = b[i][j];
    }
    __syncthreads();
  }
  for (int c0 = 0; NX > 8 && c0 < P.R; c0 += BTb) {
    const int rho = c0 + tid;
    const bool act = tid < BTb && rho < P.R;
    const int tl = tid / NX, i = tid - tl * NX;
    float ga[NX], gb[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      ga[j] = act ? blk[blk_at<NX>(rho, NX + j)] : 0.f;
      gb[j] = (j == i) ? 1.f : 0.f;
    }
#pragma unroll
    for (int kk = 0; kk < NX; ++kk) {
      float* buf = piv + (kk & 1) * (nb * 2 * NX) + tl * 2 * NX;
      if (act && i == kk) {
        float pv = ga[kk];
        if (!(pv > 0.f)) {
          nonpd = true;
          pv = 1.f;
        }
        const float inv = 1.f / pv;
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          ga[j] *= inv;
          gb[j] *= inv;
          buf[j] = ga[j];
          buf[NX + j] = gb[j];
        }
      }
      __syncthreads();
      if (act && i != kk) {
        const float f = ga[kk];
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          ga[j] = fmaf(-f, buf[j], ga[j]);
          gb[j] = fmaf(-f, buf[NX + j], gb[j]);
        }
      }
    }
    if (act) {
#pragma unroll
      for (int j = 0; j < NX; ++j) Dinv[rho * NX + j] = gb[j];
    }
    __syncthreads();
  }
  if constexpr (NX >= 16) {
    // the off-diagonal blocks come from the matrix cores (mfma_precond_blocks);
    // here only the diagonal block and the zero blocks at both ends
    for (int rho = tid; rho < P.R; rho += BT) {
      const int t = rho / NX;
      float* b = blk + blk_at<NX>(rho, 3 * NX);
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        b[NX + j] = Dinv[rho * NX + j];
        if (t == 0) b[j] = 0.f;
        if (t == P.T) b[2 * NX + j] = 0.f;
      }
    }
    return nonpd;
  }
  for (int rho = tid; rho < P.R; rho += BT) {
    const int t = rho / NX;
    const float* Dt = Dinv + rho * NX;   // row i of D_t^-1
    float lo[NX], up[NX], dr[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      lo[j] = 0.f;
      up[j] = 0.f;
      dr[j] = Dt[j];
    }
    if (t >= 1) {
      const float* Ap = P.A + (t - 1) * NX * NX;
      const float* iQp = iQ + (t - 1) * NX;
      const float* Dp = Dinv + (t - 1) * NX * NX;
#pragma unroll
      for (int k = 0; k < NX; ++k) {
        float w = 0.f;
#pragma unroll
        for (int j = 0; j < NX; ++j) w = fmaf(dr[j], Ap[j * NX + k], w);
        w *= iQp[k];   // (D_t^-1 E_{t,t-1})[i][k] = -w
#pragma unroll
        for (int j = 0; j < NX; ++j) lo[j] = fmaf(w, Dp[k * NX + j], lo[j]);
      }
    }
    if (t < P.T) {
      const float* At = P.A + t * NX * NX;
      const float* iQt = iQ + t * NX;
      const float* Dn = Dinv + (t + 1) * NX * NX;
      float bq[NX];
#pragma unroll
      for (int j = 0; j < NX; ++j) bq[j] = dr[j] * iQt[j];
#pragma unroll
      for (int k = 0; k < NX; ++k) {
        float w = 0.f;
#pragma unroll
        for (int j = 0; j < NX; ++j) w = fmaf(bq[j], At[k * NX + j], w);
        // (D_t^-1 E_{t,t+1})[i][k] = -w
#pragma unroll
        for (int j = 0; j < NX; ++j) up[j] = fmaf(w, Dn[k * NX + j], up[j]);
      }
    }
    float* b = blk + blk_at<NX>(rho, 3 * NX);
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      b[j] = lo[j];
      b[NX + j] = dr[j];
      b[2 * NX + j] = up[j];
    }
  }
  return nonpd;
}

// ===========================================================================
// Matrix-core assembly for nx >= 16 (Eq. shurcomplement, Eq. S_Phiinv)
// ===========================================================================
// The dense n x n x n contractions of the assembly -- the diagonal Schur
// blocks D_{t+1} = chi_t = A_t Q_t^-1 A_t' + B_t R_t^-1 B_t' + Q_{t+1}^-1 and
// the preconditioner's off-diagonal blocks
//   L_t := -D_t^-1 E_{t,t-1} D_{t-1}^-1 = D_t^-1 (A_{t-1} Q_{t-1}^-1) D_{t-1}^-1
// (and its transpose, the block -D_{t-1}^-1 E_{t-1,t} D_t^-1 of the row above)
// -- run on v_mfma_f32_16x16x4_f32 in 16 x 16 tiles, one wave per stage.
// Operand layout of one 16x16x4 step (lane l, q = l / 16, c = l % 16):
// lane l supplies a = A[c][4s + q] and b = B[4s + q][c]; the accumulator
// holds D[4q + r][c] in its register r.
typedef float mfma_v4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mfma_v4 mfma16(float a, float b, mfma_v4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

// Per-wave staging tile for a change of operand layout (16 x 16 floats in
// the pivot-row region, which the Gauss-Jordan inversion no longer needs):
// element (row, col) at row * 16 + (col ^ row), so that the transposed
// reads of a 16-lane group fall in distinct banks.
__device__ __forceinline__ int stg_at(int row, int col) { return row * 16 + (col ^ row); }

// Diagonal Schur blocks D_t, t = 1..T, into coefficients NX..2NX-1 of the
// rows (D_0 = Q_0^-1 comes from the row pass).  chi_{t-1} = F G' + Q_t^-1
// with G = [A_{t-1} B_{t-1}] and F = G diag(Q_{t-1}^-1, R_{t-1}^-1): tile
// (I, J) sums over the NX + m columns of F and G in steps of four.
template <int NX>
__device__ __forceinline__ void mfma_diag_blocks(const Prob& P, float* blk) {
  constexpr int TW = NX / 16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const float* iQ = P.Wq + P.L.iQ;
  const float* iR = P.Wq + P.L.iR;
  const int m = P.m;
  for (int t = 1 + w; t < P.N; t += W) {
    const int tt = t - 1;
    const float* At = P.A + tt * NX * NX;
    const float* Bt = P.B + tt * NX * m;
#pragma unroll
    for (int I = 0; I < TW; ++I) {
#pragma unroll
      for (int J = 0; J < TW; ++J) {
        mfma_v4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < NX / 4; ++s) {
          const int k = 4 * s + q;
          const float sc = iQ[tt * NX + k];
          acc = mfma16(At[(16 * I + c) * NX + k] * sc, At[(16 * J + c) * NX + k], acc);
        }
        for (int s = 0; 4 * s < m; ++s) {
          const int k = 4 * s + q;
          const bool ok = k < m;
          const float g1 = ok ? Bt[(16 * I + c) * m + k] * iR[tt * m + k] : 0.f;
          const float g2 = ok ? Bt[(16 * J + c) * m + k] : 0.f;
          acc = mfma16(g1, g2, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * I + 4 * q + r, col = 16 * J + c;
          const float d = (row == col) ? iQ[t * NX + row] : 0.f;
          blk[blk_at<NX>(t * NX + row, NX + col)] = acc[r] + d;
        }
      }
    }
  }
}

// Off-diagonal preconditioner blocks from the inverted diagonal blocks
// (Dinv, row-major [N][NX][NX]): for t = 1..T, M = D_t^-1 A_{t-1}
// Q_{t-1}^-1 tile by tile, staged through LDS into operand layout, then
// L_t = M D_{t-1}^-1.  L_t fills coefficients 3NX..4NX-1 of the rows of
// stage t and, transposed, coefficients 5NX..6NX-1 of the rows of stage t-1.
// The stage loop has the same trip count in every wave (barriers inside).
template <int NX>
__device__ __forceinline__ void mfma_precond_blocks(const Prob& P, float* blk, const float* Dinv,
                                                    float* stage_lds) {
  constexpr int TW = NX / 16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const float* iQ = P.Wq + P.L.iQ;
  float* stg = stage_lds + 256 * w;
  for (int t0 = 1; t0 < P.N; t0 += W) {
    const int t = t0 + w;
    const bool act = t < P.N;
    const int ts = act ? t : 1;   // idle waves compute a valid stage and store nothing
    const float* Dt = Dinv + ts * NX * NX;
    const float* Dp = Dinv + (ts - 1) * NX * NX;
    const float* Ap = P.A + (ts - 1) * NX * NX;
    const float* iQp = iQ + (ts - 1) * NX;
#pragma unroll
    for (int I = 0; I < TW; ++I) {
      mfma_v4 accL[TW];
#pragma unroll
      for (int J = 0; J < TW; ++J) accL[J] = mfma_v4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int K = 0; K < TW; ++K) {
        // tile (I, K) of M = D_t^-1 A_{t-1} Q_{t-1}^-1
        mfma_v4 accM = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < NX / 4; ++s) {
          const int k = 4 * s + q;
          accM = mfma16(Dt[(16 * I + c) * NX + k], Ap[k * NX + 16 * K + c], accM);
        }
        const float sc = iQp[16 * K + c];
#pragma unroll
        for (int r = 0; r < 4; ++r) stg[stg_at(4 * q + r, c)] = accM[r] * sc;
        __syncthreads();
        // L(I, J) += M(I, K) D_{t-1}^-1(K, J)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float a = stg[stg_at(c, 4 * s + q)];
#pragma unroll
          for (int J = 0; J < TW; ++J)
            accL[J] = mfma16(a, Dp[(16 * K + 4 * s + q) * NX + 16 * J + c], accL[J]);
        }
        __syncthreads();
      }
      if (act) {
#pragma unroll
        for (int J = 0; J < TW; ++J)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int a = 16 * I + 4 * q + r, b = 16 * J + c;
            blk[blk_at<NX>(t * NX + a, 3 * NX + b)] = accL[J][r];
            blk[blk_at<NX>((t - 1) * NX + b, 5 * NX + a)] = accL[J][r];
          }
      }
    }
  }
}

// ===========================================================================
// PCG (Alg. pcg) and its row products
// ===========================================================================
// Register copy of a thread's Schur / preconditioner rows; a placeholder of
// one float when the rows are read from the workspace.  With the last value
// slot's rows in LDS (TAIL) a thread holds SLOTS - 1 register rows.
template <int NX, int SLOTS, bool REG>
using RowRegs = float[REG ? SLOTS : 1][REG ? 3 * NX : 1];

// Schur row k of the LDS rows (kRecTailLds).
template <int NX>
__device__ __forceinline__ const float* tail_row(const float* tail, int k) {
  return tail + k * tail_stride(NX);
}
// Row product and off-diagonal part of an LDS row (16-byte aligned rows).
template <int NX>
__device__ __forceinline__ float tail_dot(const float* coef, const float* win) {
  static_assert(NX % 4 == 0, "LDS rows: nx a multiple of 4");
  const float4* c4 = reinterpret_cast<const float4*>(coef);
  const float4* w4 = reinterpret_cast<const float4*>(win);
  float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int j = 0; j < NX / 4; ++j) {
      const float4 c = c4[b * (NX / 4) + j], v = w4[b * (NX / 4) + j];
      acc[b] = fmaf(c.x, v.x, acc[b]);
      acc[b] = fmaf(c.y, v.y, acc[b]);
      acc[b] = fmaf(c.z, v.z, acc[b]);
      acc[b] = fmaf(c.w, v.w, acc[b]);
    }
  return (acc[0] + acc[1]) + acc[2];
}
template <int NX>
__device__ __forceinline__ float tail_offdiag(const float* coef, const float* win) {
  const float4* c4 = reinterpret_cast<const float4*>(coef);
  const float4* w4 = reinterpret_cast<const float4*>(win);
  float a0 = 0.f, a2 = 0.f;
#pragma unroll
  for (int j = 0; j < NX / 4; ++j) {
    const float4 c = c4[j], v = w4[j];
    const float4 e = c4[NX / 2 + j], u = w4[NX / 2 + j];
    a0 = fmaf(c.x, v.x, a0);
    a2 = fmaf(e.x, u.x, a2);
    a0 = fmaf(c.y, v.y, a0);
    a2 = fmaf(e.y, u.y, a2);
    a0 = fmaf(c.z, v.z, a0);
    a2 = fmaf(e.z, u.z, a2);
    a0 = fmaf(c.w, v.w, a0);
    a2 = fmaf(e.w, u.w, a2);
  }
  return a0 + a2;
}

// Scaled off-diagonal row product (kRecScaled rows: E~_{t,t-1}[i,:] at
// coef[0, nx), E~_{t,t+1}[i,:] at coef[nx, 2 nx)), window at block t-1.
template <int NX>
__device__ __forceinline__ float scaled_dot(const float* coef, const float* win) {
  float a0 = 0.f, a2 = 0.f;
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    a0 = fmaf(coef[j], win[j], a0);
    a2 = fmaf(coef[NX + j], win[2 * NX + j], a2);
  }
  return a0 + a2;
}

// nx = 16 with a stage per 16-lane row of the wave (rows tid + s BT with BT a
// multiple of 16): lane i of a row holds row i of stage t, so the products
// with the neighbouring stages need, per lane, only its own entry of p_{t-1}
// and of p_{t+1} from the window (two 4-byte reads); entry j then reaches
// every lane of the row through the multiply-add's DPP operand (row_newbcast:j
// reads lane j of the row), instead of every lane reading all 2 nx entries.
// (The compiler does not fold a broadcast into the multiply-add, hence the
// asm; s_nop 1 covers the wait states a DPP read needs after a vector ALU
// write of its source.)
__device__ __forceinline__ float bcast_dot16(const float* c, float x) {
  float a = 0.f;
  asm("s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %10 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %11 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %12 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %13 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %14 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %15 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %1, %17 row_newbcast:15 row_mask:0xf bank_mask:0xf"
      : "+v"(a)
      : "v"(x), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]),
        "v"(c[7]), "v"(c[8]), "v"(c[9]), "v"(c[10]), "v"(c[11]), "v"(c[12]), "v"(c[13]),
        "v"(c[14]), "v"(c[15]));
  return a;
}
// Scaled off-diagonal row product of row rho (window entry w[nx + rho] is
// row rho of the published vector).
__device__ __forceinline__ float scaled_dot_rows16(const float* coef, const float* wrow) {
  const float pv = wrow[-16], nv = wrow[16];
  return bcast_dot16(coef, pv) + bcast_dot16(coef + 16, nv);
}

// Ordering fence on a computed value: the value is complete before the fence
// and no memory access moves across it.  The LDS-row kernels hold four
// register rows per thread in a 256-register budget; fences after each slot's
// row product (and after each of the three blocks of a row) keep the
// compiler from issuing every slot's window reads at once, which would leave
// no room for the rows.
template <bool ON>
__device__ __forceinline__ void slot_fence(float& x) {
  if constexpr (ON) asm volatile("" : "+v"(x) : : "memory");
}
// Row product with the window read block by block (three blocks of nx).
template <int NX>
__device__ __forceinline__ float row_dot_blocks(const float* coef, const float* win) {
  static_assert(NX % 4 == 0, "block-wise row product: nx a multiple of 4");
  const float4* w4 = reinterpret_cast<const float4*>(win);
  float acc[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    float wv[NX];
#pragma unroll
    for (int j = 0; j < NX / 4; ++j) {
      const float4 v = w4[b * (NX / 4) + j];
      wv[4 * j] = v.x;
      wv[4 * j + 1] = v.y;
      wv[4 * j + 2] = v.z;
      wv[4 * j + 3] = v.w;
    }
    float a = 0.f;
#pragma unroll
    for (int j = 0; j < NX; ++j) a = fmaf(coef[b * NX + j], wv[j], a);
    slot_fence<true>(a);
    acc[b] = a;
  }
  return (acc[0] + acc[1]) + acc[2];
}

template <int NX, int SLOTS, bool REG>
__device__ __forceinline__ const float* coefS(const Prob& P, RowRegs<NX, SLOTS, REG>& S, int s,
                                              int rho) {
  if constexpr (REG) return S[s];
  return P.W + P.L.blk + blk_at<NX>(rho, 0);
}
template <int NX, int SLOTS, bool REG>
__device__ __forceinline__ const float* coefP(const Prob& P, RowRegs<NX, SLOTS, REG>& Ph, int s,
                                              int rho) {
  if constexpr (REG) return Ph[s];
  return P.W + P.L.blk + blk_at<NX>(rho, 3 * NX);
}

template <int NX, int SLOTS, bool REG>
__device__ __forceinline__ float rdot(const float* coef, const float* win) {
  if constexpr (REG) return row_dot<NX>(coef, win);
  return row_dot_ws<NX>(coef, win);
}

// Wave-block neighbour exchange: for each value s = b NX + j, the value of
// the previous and of the next stage block (lanes l - 1 and l + 1 through DPP
// wave shifts; across the 64-block boundary through lane 63 / lane 0).
// Blocks outside [0, N) read zeros (their entries are zero).
__device__ __forceinline__ float wave_prev(float x) {   // lane l <- lane l - 1, lane 0 <- 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float wave_next(float x) {   // lane l <- lane l + 1, lane 63 <- 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, true));
}
template <int NX, int SLOTS>
__device__ __forceinline__ void wave_neighbours(const float (&v)[SLOTS], float (&pv)[SLOTS],
                                                float (&nv)[SLOTS]) {
  constexpr int BPL = SLOTS / NX;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int b = 0; b < BPL; ++b)
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      float a = wave_prev(v[b * NX + j]);
      float c = wave_next(v[b * NX + j]);
      if (b > 0) {
        const float e = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[(b - 1) * NX + j]), 63));
        a = lane == 0 ? e : a;
      }
      if (b < BPL - 1) {
        const float e = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[(b + 1) * NX + j]), 0));
        c = lane == 63 ? e : c;
      }
      pv[b * NX + j] = a;
      nv[b * NX + j] = c;
    }
}

// out[s] = (row of value s) . [v_{t-1}; v_t; v_{t+1}] for the coefficient
// rows of S^ (PH = false) or Phi^-1 (PH = true): through an LDS window
// (publish, barrier, row products) or, in the wave-block layout, with the
// neighbour values in registers (same products in the same order).
// (TAIL: the last slot's rows are the LDS rows at `tail`.  SC: the scaled
// system, out = v + E~ v for the Schur product and v - E~ v for the
// preconditioner.)
template <int NX, int SLOTS, bool REG, bool WAVE, bool PH, bool TAIL = false, bool SC = false>
__device__ __forceinline__ void apply_rows(const Prob& P, float* win,
                                           RowRegs<NX, SLOTS - TAIL, REG>& M,
                                           const float (&v)[SLOTS], float (&out)[SLOTS],
                                           const float* tail = nullptr) {
  const int tid = loop_tid<TAIL>(), BT = block_threads<TAIL>(), R = P.R;
  if constexpr (WAVE) {
    float pv[SLOTS], nv[SLOTS];
    wave_neighbours<NX, SLOTS>(v, pv, nv);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      // one fused chain per row (the rows of a lane give independent chains)
      const int b = s / NX;
      float acc = M[s][0] * pv[b * NX];
#pragma unroll
      for (int j = 1; j < NX; ++j) acc = fmaf(M[s][j], pv[b * NX + j], acc);
#pragma unroll
      for (int j = 0; j < NX; ++j) acc = fmaf(M[s][NX + j], v[b * NX + j], acc);
#pragma unroll
      for (int j = 0; j < NX; ++j) acc = fmaf(M[s][2 * NX + j], nv[b * NX + j], acc);
      out[s] = acc;
    }
  } else {
    publish<NX, SLOTS, REG, false, TAIL>(win, v, R);
    __syncthreads();
    constexpr int RS = SLOTS - TAIL;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int rho = row_of<NX, false>(s, tid, BT);
      out[s] = 0.f;
      bool lds_row = false;
      if constexpr (TAIL) {
        if (s == SLOTS - 1) {
          lds_row = true;
          if (rho < R) out[s] = tail_dot<NX>(tail_row<NX>(tail, rho - RS * BT), win + (rho / NX) * NX);
        }
      }
      if constexpr (SC) {
        if (row_live<REG>(s, rho, R, BT)) {
          float e;
          if constexpr (NX == 16) e = scaled_dot_rows16(M[s], win + NX + rho);
          else e = scaled_dot<NX>(M[s], win + (rho / NX) * NX);
          out[s] = PH ? v[s] - e : v[s] + e;
        }
      } else if (!lds_row && row_live<REG>(s, rho, R, BT)) {
        const int t = rho / NX;
        const int sr = s < RS ? s : 0;   // (s < RS here)
        const float* coef = PH ? coefP<NX, RS, REG>(P, M, sr, rho) : coefS<NX, RS, REG>(P, M, sr, rho);
        if constexpr (TAIL) out[s] = row_dot_blocks<NX>(coef, win + t * NX);
        else out[s] = rdot<NX, RS, REG>(coef, win + t * NX);
      }
      slot_fence<TAIL>(out[s]);
    }
  }
}

// Workgroup sum of the PCG: one wave needs no LDS exchange.
template <bool WAVE>
__device__ __forceinline__ float pcg_sum(float part, const Lds& sh, int& redi, int nwv) {
  if constexpr (WAVE) return wave_sum(part);
  return block_sum(part, sh.red + 64 * (redi++ & 1), nwv);
}

// LDS layout of the inverted diagonal blocks: row rho of D_t^-1 at rho NX,
// its 16-byte chunks permuted by dinv_swz(rho) (chunk j at j ^ swz).  With an
// even number of chunks per row the 16-byte reads of consecutive rows (lanes)
// would fall on the same banks every few lanes; the permutation spreads the
// 16 lanes of a read over all banks.
template <int NX>
__device__ __forceinline__ int dinv_swz(int rho) {
  constexpr int C = NX / 4;
  if constexpr (NX % 4 != 0 || C % 2 == 1 || C > 16) return 0;
  else return (rho / (16 / C)) & (C - 1);
}

// Row product of the inverted diagonal block D_t^-1 (row rho, in LDS, chunks
// permuted by swz) with the window values of block t.
template <int NX>
__device__ __forceinline__ float dinv_dot(const float* drow, const float* wblk, int swz) {
  float a0 = 0.f, a1 = 0.f;
  if constexpr (NX % 4 == 0) {
    const float4* d4 = reinterpret_cast<const float4*>(drow);
    const float4* w4 = reinterpret_cast<const float4*>(wblk);
#pragma unroll
    for (int j = 0; j < NX / 4; ++j) {
      const float4 d = d4[j ^ swz], w = w4[j];
      a0 = fmaf(d.x, w.x, a0);
      a1 = fmaf(d.y, w.y, a1);
      a0 = fmaf(d.z, w.z, a0);
      a1 = fmaf(d.w, w.w, a1);
    }
  } else {
#pragma unroll
    for (int j = 0; j < NX; ++j) a0 = fmaf(drow[j], wblk[j], a0);
  }
  return a0 + a1;
}

// The off-diagonal part of a Schur row, E_{t,t-1}[i,:] v_{t-1} +
// E_{t,t+1}[i,:] v_{t+1}, with the window at block t-1.
template <int NX>
__device__ __forceinline__ float offdiag_dot(const float* coef, const float* win) {
  float a0 = 0.f, a2 = 0.f;
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    a0 = fmaf(coef[j], win[j], a0);
    a2 = fmaf(coef[2 * NX + j], win[2 * NX + j], a2);
  }
  return a0 + a2;
}

// z = Phi^-1 v with the preconditioner in factored form: the blocks of
// Eq. S_Phiinv are D_t^-1 on the diagonal and -D_t^-1 E_{t,t+-1} D_{t+-1}^-1
// off it, that is Phi^-1 = D^-1 - D^-1 E D^-1 with E the off-diagonal blocks
// of S^.  So w = D^-1 v, u = v - E w, z = D^-1 u: the inverted diagonal
// blocks from LDS, E from the Schur rows the thread holds, three exchanges
// through two windows (wa, wb).  Rows past R (register rows are zero there)
// give zeros.  When nx divides the wave size, the rows of a stage are
// consecutive lanes of one wave, so the two D^-1 products read only their own
// wave's values and need no workgroup barrier before them (wa is read only by
// the wave that wrote those entries).
template <int NX, int SLOTS, bool TAIL>
__device__ __forceinline__ void apply_precond_factored(const Prob& P, const Lds& sh, float* wa,
                                                       float* wb,
                                                       RowRegs<NX, SLOTS - TAIL, true>& S,
                                                       const float (&v)[SLOTS],
                                                       float (&z)[SLOTS]) {
  const int tid = loop_tid<TAIL>(), BT = block_threads<TAIL>(), R = P.R;
  constexpr int RS = SLOTS - TAIL;
  float w[SLOTS];
  constexpr bool STAGE_IN_WAVE = 64 % NX == 0;
  publish<NX, SLOTS, true, false, TAIL>(wa, v, R);
  if constexpr (STAGE_IN_WAVE) wave_sync();
  else __syncthreads();
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int rho = row_of<NX, false>(s, tid, BT);
    const int t = rho / NX;
    w[s] = rho < R ? dinv_dot<NX>(sh.dinv + rho * NX, wa + NX + t * NX, dinv_swz<NX>(rho)) : 0.f;
    slot_fence<TAIL>(w[s]);
  }
  publish<NX, SLOTS, true, false, TAIL>(wb, w, R);
  __syncthreads();
  float u[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int rho = row_of<NX, false>(s, tid, BT);
    const int t = rho / NX;
    if constexpr (TAIL) {
      if (s == SLOTS - 1)
        u[s] = rho < R ? v[s] - tail_offdiag<NX>(tail_row<NX>(sh.tail, rho - RS * BT), wb + t * NX)
                       : 0.f;
      else
        u[s] = v[s] - offdiag_dot<NX>(S[s < RS ? s : 0], wb + t * NX);
    } else {
      u[s] = v[s] - offdiag_dot<NX>(S[s], wb + t * NX);
    }
    slot_fence<TAIL>(u[s]);
  }
  // (every read of wa happened before the barrier above)
  publish<NX, SLOTS, true, false, TAIL>(wa, u, R);
  if constexpr (STAGE_IN_WAVE) wave_sync();
  else __syncthreads();
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int rho = row_of<NX, false>(s, tid, BT);
    const int t = rho / NX;
    z[s] = rho < R ? dinv_dot<NX>(sh.dinv + rho * NX, wa + NX + t * NX, dinv_swz<NX>(rho)) : 0.f;
    slot_fence<TAIL>(z[s]);
  }
}

// z = Phi^-1 v: the explicit preconditioner rows, or (DINV) the factored form.
template <int NX, int SLOTS, bool REG, bool WAVE, bool DINV, bool TAIL, bool SC = false>
__device__ __forceinline__ void apply_precond(const Prob& P, const Lds& sh,
                                              RowRegs<NX, SLOTS - TAIL, REG>& S,
                                              RowRegs<NX, SLOTS - TAIL, REG && !DINV>& Ph,
                                              const float (&v)[SLOTS], float (&z)[SLOTS]) {
  if constexpr (SC) {
    static_assert(REG && !WAVE && !DINV && !TAIL, "scaled system: register rows");
    apply_rows<NX, SLOTS, REG, WAVE, true, false, true>(P, sh.w1, S, v, z);
  } else if constexpr (DINV) {
    static_assert(REG && !WAVE, "factored preconditioner: register rows, workgroup layout");
    apply_precond_factored<NX, SLOTS, TAIL>(P, sh, sh.w1, sh.w2, S, v, z);
  } else {
    static_assert(!TAIL, "LDS rows: factored preconditioner only");
    apply_rows<NX, SLOTS, REG, WAVE, true>(P, sh.w1, Ph, v, z);
  }
}

// v' Phi^-1 v for a vector held in this thread's rows.
template <int NX, int SLOTS, bool REG, bool WAVE, bool DINV, bool TAIL, bool SC = false>
__device__ __forceinline__ float precond_norm(const Prob& P, const Lds& sh,
                                              RowRegs<NX, SLOTS - TAIL, REG>& S,
                                              RowRegs<NX, SLOTS - TAIL, REG && !DINV>& Ph,
                                              const float (&v)[SLOTS], int& redi) {
  const int nwv = (block_threads<TAIL>() + 63) >> 6;
  float z[SLOTS];
  apply_precond<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, sh, S, Ph, v, z);
  float part = 0.f;
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) part = fmaf(v[s], z[s], part);
  return pcg_sum<WAVE>(part, sh, redi, nwv);
}

// PCG (Alg. pcg) on S^ d = rhs from d = 0, preconditioner Phi^-1; rows live
// in registers (REG) or in the workspace.  Stops when eta = r'Phi^-1 r <=
// max(rel_tol^2 * rhs'Phi^-1 rhs, abs_thresh), or at the iteration cap.
// (The warm start of Alg. pcg enters through rhs = g - S^ lambda, which the
// caller computes in double.)  Returns the iteration count; ORs status bits.
// PCG of Alg. pcg on the scaled system (kRecScaled, register rows), with
// one barrier fewer per iteration: the Schur product is taken of z = Phi^-1 r
// instead of p, and y = S^ p follows from y <- S^ z + beta y (the same
// vectors in exact arithmetic), so that z's exchange and the reduction of
// eta' = r'z share one barrier: the wave sums of eta' are written before the
// barrier that publishes z, and beta is known before the row products.  Per
// iteration: the reduction of p'y, the exchange of r (preconditioner), the
// exchange of z with eta'.  Same stopping test, status bits and return as
// pcg below; the refinement passes check each result against the residual
// formed in double.  Used for nx >= 12.
template <int NX, int SLOTS, bool REG>
__device__ __forceinline__ int pcg_scaled(const Prob& P, const Lds& sh,
                                          RowRegs<NX, SLOTS, REG>& S, RowRegs<NX, SLOTS, REG>& Ph,
                                          const float (&rhs)[SLOTS], float (&d)[SLOTS], int maxit,
                                          float rel_tol, float abs_thresh, int& flags, int& redi,
                                          int maxit_flag) {
  static_assert(REG, "scaled system: register rows");
  const int tid = threadIdx.x, BT = blockDim.x, R = P.R;
  const int nwv = (BT + 63) >> 6;
  float r[SLOTS], p[SLOTS], z[SLOTS], y[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    r[s] = rhs[s];
    d[s] = 0.f;
  }
  apply_precond<NX, SLOTS, REG, false, false, false, true>(P, sh, S, Ph, r, z);
  float part = 0.f;
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    p[s] = z[s];
    part = fmaf(r[s], z[s], part);
  }
  float eta = pcg_sum<false>(part, sh, redi, nwv);
  const float thresh = fmaxf(rel_tol * rel_tol * eta, abs_thresh);
  int it = 0;
  if (!isfinite(eta)) {
    flags |= DMPC_PROB_NONFINITE;
    return 0;
  }
  if (eta > thresh) apply_rows<NX, SLOTS, REG, false, false, false, true>(P, sh.w0, S, p, y);
  while (it < maxit && eta > thresh) {
    part = 0.f;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) part = fmaf(p[s], y[s], part);
    const float v = pcg_sum<false>(part, sh, redi, nwv);
    if (!(v > 0.f)) {
      flags |= isfinite(v) ? DMPC_PROB_NONPD : DMPC_PROB_NONFINITE;
      break;
    }
    const float alpha = eta * __builtin_amdgcn_rcpf(v);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      d[s] = fmaf(alpha, p[s], d[s]);
      r[s] = fmaf(-alpha, y[s], r[s]);
    }
    apply_precond<NX, SLOTS, REG, false, false, false, true>(P, sh, S, Ph, r, z);
    part = 0.f;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) part = fmaf(r[s], z[s], part);
    // eta' and the exchange of z behind one barrier
    float* red = sh.red + 64 * (redi++ & 1);
    const float wpart = wave_sum(part);
    if ((tid & 63) == 0) red[tid >> 6] = wpart;
    publish<NX, SLOTS, REG, false, false>(sh.w0, z, R);
    __syncthreads();
    float etan = 0.f;
    for (int w = 0; w < nwv; ++w) etan += red[w];
    ++it;
    const float beta = etan * __builtin_amdgcn_rcpf(eta);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int rho = row_of<NX, false>(s, tid, BT);
      float e;
      if constexpr (NX == 16) e = scaled_dot_rows16(S[s], sh.w0 + NX + rho);
      else e = scaled_dot<NX>(S[s], sh.w0 + (rho / NX) * NX);
      y[s] = fmaf(beta, y[s], z[s] + e);
      p[s] = fmaf(beta, p[s], z[s]);
    }
    if (!isfinite(etan)) {
      flags |= DMPC_PROB_NONFINITE;
      break;
    }
    eta = etan;
  }
  if (it >= maxit && eta > thresh) flags |= maxit_flag;
  return it;
}

template <int NX, int SLOTS, bool REG, bool WAVE, bool DINV, bool TAIL, bool SC = false>
__device__ __forceinline__ int pcg(const Prob& P, const Lds& sh,
                                   RowRegs<NX, SLOTS - TAIL, REG>& S,
                                   RowRegs<NX, SLOTS - TAIL, REG && !DINV>& Ph,
                                   const float (&rhs)[SLOTS],
                                   float (&d)[SLOTS], int maxit, float rel_tol, float abs_thresh,
                                   int& flags, int& redi, int maxit_flag) {
  // (nx >= 12: on the bicycle (nx = 8, Schur condition numbers near 1e6)
  // the recurrence for y lengthened the slowest problem's PCG by a tenth)
  if constexpr (SC && NX >= 12 && !WAVE && !DINV && !TAIL)
    return pcg_scaled<NX, SLOTS, REG>(P, sh, S, Ph, rhs, d, maxit, rel_tol, abs_thresh, flags,
                                      redi, maxit_flag);
  const int nwv = (block_threads<TAIL>() + 63) >> 6;
  float r[SLOTS], p[SLOTS], z[SLOTS], y[SLOTS];
  // initial residual r = rhs (d = 0), r~ = Phi^-1 r, p = r~, eta = r'r~
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    r[s] = rhs[s];
    d[s] = 0.f;
  }
  apply_precond<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, sh, S, Ph, r, z);
  float part = 0.f;
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    p[s] = z[s];
    part = fmaf(r[s], z[s], part);
  }
  float eta = pcg_sum<WAVE>(part, sh, redi, nwv);
  const float thresh = fmaxf(rel_tol * rel_tol * eta, abs_thresh);
  int it = 0;
  if (!isfinite(eta)) {
    flags |= DMPC_PROB_NONFINITE;
    return 0;
  }
  while (it < maxit && eta > thresh) {
    // y = S^ p, v = p'y, alpha = eta / v
    apply_rows<NX, SLOTS, REG, WAVE, false, TAIL, SC>(P, sh.w0, S, p, y, sh.tail);
    part = 0.f;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) part = fmaf(p[s], y[s], part);
    const float v = pcg_sum<WAVE>(part, sh, redi, nwv);
    if (!(v > 0.f)) {
      flags |= isfinite(v) ? DMPC_PROB_NONPD : DMPC_PROB_NONFINITE;
      break;
    }
    // (alpha and beta with the hardware reciprocal: within about one ulp of
    // the quotient, and off the latency-bound critical path of a division)
    const float alpha = eta * __builtin_amdgcn_rcpf(v);
    // d += alpha p, r -= alpha y
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      d[s] = fmaf(alpha, p[s], d[s]);
      r[s] = fmaf(-alpha, y[s], r[s]);
    }
    // r~ = Phi^-1 r, eta' = r'r~
    apply_precond<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, sh, S, Ph, r, z);
    part = 0.f;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) part = fmaf(r[s], z[s], part);
    const float etan = pcg_sum<WAVE>(part, sh, redi, nwv);
    ++it;
    // beta, p = r~ + beta p, eta = eta'; (p is not used
    // after a non-finite eta', so it is updated before that exit)
    const float beta = etan * __builtin_amdgcn_rcpf(eta);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) p[s] = fmaf(beta, p[s], z[s]);
    if (!isfinite(etan)) {
      flags |= DMPC_PROB_NONFINITE;
      break;
    }
    eta = etan;
  }
  if (it >= maxit && eta > thresh) flags |= maxit_flag;
  return it;
}

// ===========================================================================
// Forward phases (not inlined: each keeps its registers to itself)
// ===========================================================================
struct LsParams {
  float alphas[kMaxAlphas];
  int n;
  float eta;
};
// alphas[a - 1] for a in 1..kMaxAlphas, 0 for a = 0: a select chain over
// the (uniform) parameters, so that a per-lane index does not put the array
// in scratch memory.
__device__ __forceinline__ float pick_alpha(const LsParams& lp, int a) {
  float v = 0.f;
#pragma unroll
  for (int i = 0; i < kMaxAlphas; ++i) v = (a == i + 1) ? lp.alphas[i] : v;
  return v;
}

// Line-search outcome: selected step and flag bits.
struct LsResult {
  int sel, flags;
};

// Initial guess (Alg. sqp inputs) into LDS; x_0 = x_s; rollout if asked.
template <int NX>
__device__ __noinline__ void fwd_begin(const ProbRec* rec, const float* data, const float* sol,
                                       float* ws, int init) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = blockDim.x;
  const Prob P = make_prob<NX>(*rec, data, ws);
  const Carve C = carve_of<NX>(P);
  float* xbar = bulk_base(smem, P) + C.xbar;
  float* ubar = bulk_base(smem, P) + C.ubar;
  const int T = P.T, m = P.m, R = P.R, TM = P.TM;
  const float* solx = sol + rec->sol_off;
  const float* solu = solx + R;
  for (int i = tid; i < R; i += BT) xbar[i] = (i < NX) ? P.x0[i] : solx[i];
  for (int i = tid; i < TM; i += BT) ubar[i] = solu[i];
  zero_pads<NX>(smem, C, P);
  if (P.flags & kRecLinLds) stage_lin<NX>(P, *rec, data, false);
  __syncthreads();
  if (init != DMPC_INIT_ROLLOUT) return;
  if (P.dyn == DMPC_DYN_LTV) {
    for (int t = 0; t < T; ++t) {
      if (tid < NX) {
        const float* At = P.A + t * NX * NX + tid * NX;
        const float* Bt = P.B + t * NX * m + tid * m;
        float s = P.c[t * NX + tid];
#pragma unroll
        for (int j = 0; j < NX; ++j) s = fmaf(At[j], xbar[t * NX + j], s);
        for (int l = 0; l < m; ++l) s = fmaf(Bt[l], ubar[t * m + l], s);
        xbar[(t + 1) * NX + tid] = s;
      }
      __syncthreads();
    }
  } else {
    const ModelPar mp = load_par(P);
    if (tid == 0) {
      double xc[NX], xn[NX], uc[2];
#pragma unroll
      for (int i = 0; i < NX; ++i) xc[i] = xbar[i];
      for (int t = 0; t < T; ++t) {
        uc[0] = ubar[t * m];
        uc[1] = (m > 1) ? ubar[t * m + 1] : 0.f;
        dyn_step<NX>(P, mp, t, xc, uc, xn, P.dyn);
#pragma unroll
        for (int i = 0; i < NX; ++i) {
          xbar[(t + 1) * NX + i] = (float)xn[i];
          xc[i] = (double)(float)xn[i];
        }
      }
    }
    __syncthreads();
  }
}

// QP data at the iterate (Eq. QPmatrices), Schur rows and right-hand side
// (Eq. shurcomplement) and preconditioner rows (Eq. S_Phiinv) into the
// workspace.  Returns non-zero (in every thread) on a non-positive pivot.
template <int NX>
__device__ __forceinline__ int fwd_blocks_body(const ProbRec* rec, const float* data, float* ws,
                                               int first) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = blockDim.x;
  const Prob P = make_prob<NX>(*rec, data, ws);
  const Carve C = carve_of<NX>(P);
  form_qp<NX>(P, bulk_base(smem, P) + C.xbar, bulk_base(smem, P) + C.ubar, first);
  __syncthreads();
  float* blk = P.W + P.L.blk;
  float* gv = P.W + P.L.g;
  if (!first && P.dyn == DMPC_DYN_LTV && P.cost == DMPC_COST_DIAG) {
    // linear dynamics and diagonal costs: the Schur and preconditioner blocks
    // depend on A, B and the projected Hessians only, which do not change
    // between SQP iterations; the rows of the first iteration stay, and only
    // the right-hand side follows the linear terms
    constexpr int U = gather_rows<NX>();
    for (int base = tid; base < P.R; base += U * BT) {
      float ag[U][NX];   // row i of A_{t-1}
      gather_A<NX, U, false>(P.A, base, BT, NX, P.T * NX, ag);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rho = base + u * BT;
        if (rho < P.R) gv[rho] = schur_rhs_row<NX>(P, rho / NX, rho % NX, ag[u]);
      }
    }
    __syncthreads();
    return 0;
  }
  // nx >= 16: the diagonal blocks of stages 1..T and the preconditioner's
  // off-diagonal blocks are dense contractions, formed on the matrix cores
  constexpr bool MX = NX >= 16;
  for (int rho = tid; rho < P.R; rho += BT) {
    const int t = rho / NX, i = rho - t * NX;
    float row[3 * NX], g;
    schur_row<NX, float, MX>(P, t, i, row, g);
#pragma unroll
    for (int j = 0; j < 3 * NX; ++j)
      if (!MX || t == 0 || j < NX || j >= 2 * NX) blk[blk_at<NX>(rho, j)] = row[j];
    gv[rho] = g;
  }
  if constexpr (MX) mfma_diag_blocks<NX>(P, blk);
  __syncthreads();
  if constexpr (NX == 8 || NX == 12 || NX == 16) {   // (nx with scaled-system kernels)
    if (P.flags & kRecScaled) return scaled_blocks<NX>(P, (double*)(smem + C.piv)) ? 1 : 0;
  }
  const bool bad = precond_rows<NX>(P, smem + C.piv);
  if constexpr (MX) mfma_precond_blocks<NX>(P, blk, P.W + P.L.Dinv, smem + C.piv);
  return __syncthreads_or(bad ? 1 : 0);
}

// QP data at the iterate (Eq. QPmatrices) only (the wave-block kernels
// assemble the rows in registers).
template <int NX>
__device__ __forceinline__ void fwd_form_body(const ProbRec* rec, const float* data, float* ws,
                                              int first) {
  extern __shared__ float smem[];
  const Prob P = make_prob<NX>(*rec, data, ws);
  const Carve C = carve_of<NX>(P);
  form_qp<NX>(P, bulk_base(smem, P) + C.xbar, bulk_base(smem, P) + C.ubar, first);
  __syncthreads();
}

// Squared norms that steer the refinement: of the residual and of the KKT
// right-hand side the residual is measured against.
struct ResNorms {
  float r2, rhs2;
};

__device__ __forceinline__ ResNorms block_sum2(float a, float b, float* red, int nwv) {
  a = wave_sum(a);
  b = wave_sum(b);
  ResNorms n{a, b};
  if (nwv == 1) return n;
  if ((threadIdx.x & 63) == 0) {
    const int w = threadIdx.x >> 6;
    red[2 * w] = a;
    red[2 * w + 1] = b;
  }
  __syncthreads();
  n = ResNorms{0.f, 0.f};
  for (int w = 0; w < nwv; ++w) {
    n.r2 += red[2 * w];
    n.rhs2 += red[2 * w + 1];
  }
  return n;
}

// Residual of the Schur system in double, r = g - S^ lambda with lambda = w0
// + w2 (double-float), in factored form: with the primal point of the
// multipliers (Eq. schur:xu)
//   x_t = -Q_t^-1 (q_t + lambda_t - A_t' lambda_{t+1}),  u_t = -R_t^-1 (r_t - B_t' lambda_{t+1}),
// the rows of g - S^ lambda are the dynamics defects of that point:
//   r_0 = x_0 - x_s,   r_{t+1} = x_{t+1} - A_t x_t - B_t u_t - c_t
// (expand S^ = H G^-1 H' and g = -gamma: the q, r terms cancel).  This needs
// O(nx + nu) work per row instead of re-assembling the rows of S^.  Result
// (rounded to float) to w1[NX + rho]; returns the norms of r and of the KKT
// right-hand side [-b; d] = [-(q, r); (x_s, c)] (Eq. ocp:KKT), identical in
// every thread.
// Scaled system (kRecScaled): r~ = L^-1 r, the right-hand side of the PCG on
// the scaled system, from the residual r in LDS (unpadded view) to out, at
// the end of the residual call, where the double rows of L^-1 of several
// rows can be loaded at once (in the PCG's context the rows of the Schur
// system hold the registers).  Row rho: the double row of L_t^-1 (zero
// above its diagonal) times the stage's residual, accumulated in double.
template <int NX>
__device__ __forceinline__ void scaled_rhs(const Prob& P, const float* r, float* out) {
  const int tid = threadIdx.x, BT = blockDim.x, R = P.R;
  const double* Li = (const double*)(P.W + P.L.Lid);
  constexpr int U = gather_rows<NX>();
  for (int base = tid; base < R; base += U * BT) {
    double l[U][NX];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int rho = base + u * BT;
      const double* row = Li + (int64_t)(rho < R ? rho : 0) * NX;
#pragma unroll
      for (int j = 0; j < NX; ++j) l[u][j] = row[j];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int rho = base + u * BT;
      if (rho < R) {
        const float* rt = r + (rho / NX) * NX;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < NX; ++j) acc = fma(l[u][j], (double)rt[j], acc);
        out[rho] = (float)acc;
      }
    }
  }
  __syncthreads();
}

// Scaled system: d = L^-T d~, the PCG's solution mapped back, from d~ in LDS
// (unpadded view of w1) to the line-search region (floats), in a call of its
// own for the same reason: column i of the double L_t^-1 (zero above its
// diagonal) times the stage's d~, accumulated in double.
template <int NX>
__device__ __noinline__ void scaled_solution_call(const ProbRec* rec, const float* data,
                                                  float* ws) {
  extern __shared__ float smem[];
  const Prob P = make_prob<NX>(*rec, data, ws);
  const Carve C = carve_of<NX>(P);
  const int tid = threadIdx.x, BT = blockDim.x, R = P.R;
  const float* dt = smem + C.w1 + NX;
  float* out = bulk_base(smem, P) + C.ls;
  const double* Li = (const double*)(P.W + P.L.Lid);
  constexpr int U = gather_rows<NX>();
  for (int base = tid; base < R; base += U * BT) {
    double l[U][NX];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int rho = base + u * BT;
      const int rr = rho < R ? rho : 0;
      const int t = rr / NX, i = rr - t * NX;
      const double* col = Li + (int64_t)t * NX * NX + i;
#pragma unroll
      for (int j = 0; j < NX; ++j) l[u][j] = col[j * NX];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int rho = base + u * BT;
      if (rho < R) {
        const float* wt = dt + (rho / NX) * NX;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < NX; ++j) acc = fma(l[u][j], (double)wt[j], acc);
        out[rho] = (float)acc;
      }
    }
  }
  __syncthreads();
}

template <int NX>
__device__ __forceinline__ ResNorms fwd_residual64_body(const ProbRec* rec, const float* data,
                                                        float* ws, float kkt_tol) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = blockDim.x;
  const Prob P = make_prob<NX>(*rec, data, ws);
  const Carve C = carve_of<NX>(P);
  const int T = P.T, m = P.m, R = P.R, TM = P.TM;
  const float* w0 = smem + C.w0 + NX;   // lambda, high part (unpadded view)
  const float* w2 = smem + C.w2 + NX;   // low part
  float* w1 = smem + C.w1;
  double* xz = (double*)(bulk_base(smem, P) + C.ls);  // primal point of lambda: x [R], u [TM]
  double* uz = xz + R;
  const int nwv = (BT + 63) >> 6;
  const float* q = P.Wq + P.L.q;
  const float* rr = P.Wq + P.L.r;
  const double* iQd = (const double*)(P.Wq + P.L.iQd);
  const double* iRd = (const double*)(P.Wq + P.L.iRd);
  if (P.Ad == nullptr) {
    constexpr int U = gather_rows<NX>();
    for (int base = tid; base < R; base += U * BT) {
      float a[U][NX], qv[U];
      double iq[U];
      gather_A<NX, U, true>(P.A, base, BT, 0, T * NX, a);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = base + u * BT < R ? base + u * BT : 0;
        qv[u] = q[r];
        iq[u] = iQd[r];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rho = base + u * BT;
        if (rho < R) {
          const int t = rho / NX;
          double acc = (double)qv[u] + ((double)w0[rho] + (double)w2[rho]);
          if (t < T) {
#pragma unroll
            for (int k = 0; k < NX; ++k)
              acc -= (double)a[u][k] * ((double)w0[(t + 1) * NX + k] + (double)w2[(t + 1) * NX + k]);
          }
          xz[rho] = -acc * iq[u];
        }
      }
    }
  } else {
    for (int rho = tid; rho < R; rho += BT) {
      const int t = rho / NX, i = rho - t * NX;
      double acc = (double)q[rho] + ((double)w0[rho] + (double)w2[rho]);
      if (t < T) {
        const int a0 = t * NX * NX;
#pragma unroll
        for (int k = 0; k < NX; ++k)
          acc -= ldA<double>(P, a0 + k * NX + i) *
                 ((double)w0[(t + 1) * NX + k] + (double)w2[(t + 1) * NX + k]);
      }
      xz[rho] = -acc * iQd[rho];
    }
  }
  for (int idx = tid; idx < TM; idx += BT) {
    const int t = idx / m, l = idx - t * m;
    const int b0 = t * NX * m;
    double acc = (double)rr[idx];
#pragma unroll
    for (int k = 0; k < NX; ++k)
      acc -= ldB<double>(P, b0 + k * m + l) *
             ((double)w0[(t + 1) * NX + k] + (double)w2[(t + 1) * NX + k]);
    uz[idx] = -acc * iRd[idx];
  }
  __syncthreads();
  float r2 = 0.f, b2 = 0.f;
  auto defect_row = [&](int rho, auto&& aent) {
    const int t = rho / NX, i = rho - t * NX;
    double res;
    float dv;
    if (t == 0) {
      dv = P.x0[i];
      res = xz[i] - (double)dv;
    } else {
      const int tt = t - 1;
      dv = P.c[tt * NX + i];
      double acc = ldc<double>(P, tt * NX + i);
#pragma unroll
      for (int j = 0; j < NX; ++j) acc += aent(tt, i, j) * xz[tt * NX + j];
      for (int l = 0; l < m; ++l) acc += ldB<double>(P, tt * NX * m + i * m + l) * uz[tt * m + l];
      res = xz[rho] - acc;
    }
    w1[NX + rho] = (float)res;
    r2 += (float)(res * res);
    b2 += q[rho] * q[rho] + dv * dv;
  };
  if (P.Ad == nullptr) {
    constexpr int U = gather_rows<NX>();
    for (int base = tid; base < R; base += U * BT) {
      float a[U][NX];
      gather_A<NX, U, false>(P.A, base, BT, NX, T * NX, a);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rho = base + u * BT;
        if (rho < R) defect_row(rho, [&](int, int, int j) { return (double)a[u][j]; });
      }
    }
  } else {
    for (int rho = tid; rho < R; rho += BT)
      defect_row(rho, [&](int tt, int i, int j) { return ldA<double>(P, tt * NX * NX + i * NX + j); });
  }
  for (int idx = tid; idx < TM; idx += BT) b2 += rr[idx] * rr[idx];
  const ResNorms n = block_sum2(r2, b2, smem + C.red, nwv);
  __syncthreads();   // xz is the line search's region
  if constexpr (NX == 8 || NX == 12 || NX == 16) {
    // (not when the residual meets the KKT target: the caller stops there,
    // by the same test)
    if ((P.flags & kRecScaled) && !(n.r2 <= kkt_tol * kkt_tol * n.rhs2))
      scaled_rhs<NX>(P, smem + C.w1 + NX, smem + C.w2 + NX);
  }
  return n;
}

// Line-search tasks (ai, t) -- stage t at the current point (ai = 0) or at
// candidate alphas[ai-1] -- for one dynamics and cost kind: cost and dynamics
// defect in double to tc/td.  Two tasks per lane per pass, computed side by
// side (branch free: lanes past the end and the last stage evaluate clamped
// stages and discard the result), so that the long double-precision chains
// of the two overlap.
struct LsTaskArgs {
  const float *xbar, *xp, *ubar, *up;
  double *tc, *td;
  double* dn;   // this thread's share of grad c(z)'(z+ - z), from its row-0 tasks
  int ntask, na;
};
template <int NX, int DYN, int COST>
__device__ __forceinline__ void ls_tasks(const Prob& P, const ModelPar& mp, const LsParams& lp,
                                         const LsTaskArgs& a) {
  constexpr int MU = DYN == DMPC_DYN_CARTPOLE ? 1 : 2;   // inputs of the nonlinear models
  const int tid = threadIdx.x, BT = blockDim.x;
  const int N = P.N, T = P.T, m = P.m;
  int ai[2], tt[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int task = tid + h * BT;
    ai[h] = task / N;
    tt[h] = task - ai[h] * N;
  }
  for (int task0 = 0; task0 < a.ntask; task0 += 2 * BT) {
    double cst[2], dfc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bool live = task0 + h * BT + tid < a.ntask;
      const int aic = live ? ai[h] : a.na;
      const int tcl = live ? tt[h] : N - 1;
      const int tn = tcl < T ? tcl : T - 1;    // dynamics stage (clamped)
      const double al = (double)pick_alpha(lp, aic);
      double xa[NX], xa1[NX];
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        const double b0 = a.xbar[tcl * NX + j], q0 = a.xp[tcl * NX + j];
        const double b1 = a.xbar[(tn + 1) * NX + j], q1 = a.xp[(tn + 1) * NX + j];
        xa[j] = b0 + al * (q0 - b0);
        xa1[j] = b1 + al * (q1 - b1);
      }
      const float* ub = a.ubar + tn * m;
      const float* uq = a.up + tn * m;
      double c = cost_x<NX>(P, tcl, xa, COST), cu = 0.0;
      double xn[NX];
      if constexpr (DYN == DMPC_DYN_LTV) {
        const float* At = P.A + tn * NX * NX;
        const float* Bt = P.B + tn * NX * m;
#pragma unroll
        for (int i = 0; i < NX; ++i) {
          double sacc = P.c[tn * NX + i];
#pragma unroll
          for (int j = 0; j < NX; ++j) sacc += (double)At[i * NX + j] * xa[j];
          xn[i] = sacc;
        }
        for (int l = 0; l < m; ++l) {
          const double u = (double)ub[l] + al * ((double)uq[l] - (double)ub[l]);
          cu += cost_u1<NX>(P, tn, l, u, COST);
#pragma unroll
          for (int i = 0; i < NX; ++i) xn[i] += (double)Bt[i * m + l] * u;
        }
      } else {
        double ua[2];
#pragma unroll
        for (int l = 0; l < 2; ++l) {
          ua[l] = l < MU ? (double)ub[l] + al * ((double)uq[l] - (double)ub[l]) : 0.0;
          if (l < MU) cu += cost_u1<NX>(P, tn, l, ua[l], COST);
        }
        dyn_step<NX>(P, mp, tn, xa, ua, xn, DYN);
      }
      double d = 0.0;
#pragma unroll
      for (int j = 0; j < NX; ++j) d += fabs(xa1[j] - xn[j]);
      const bool dyn_stage = tcl < T;
      cst[h] = c + (dyn_stage ? cu : 0.0);
      dfc[h] = dyn_stage ? d : 0.0;
      // row 0 (the current point): the directional derivative of its costs
      double g = dcost_x<NX>(P, tcl, a.xbar + tcl * NX, a.xp + tcl * NX, COST);
      double gu = 0.0;
      for (int l = 0; l < m; ++l) gu += dcost_u1<NX>(P, tn, l, ub[l], uq[l], COST);
      g += dyn_stage ? gu : 0.0;
      *a.dn += (live && aic == 0) ? g : 0.0;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (task0 + h * BT + tid < a.ntask) {
        const int row = ai[h] * N + tt[h];
        a.tc[row] = cst[h];
        a.td[row] = dfc[h];
      }
      tt[h] += 2 * BT;
      while (tt[h] >= N) {
        tt[h] -= N;
        ++ai[h];
      }
    }
  }
}

// Line-search sums for linear dynamics (App. A.3, Alg. linesearch): the
// stage costs and dynamics defects are sums over state rows (t, i) and input
// rows (t, l), so threads take rows instead of stages.  Along a candidate
// step the next state is affine in alpha, (A_t x + B_t u + c_t)(alpha) = a0 +
// alpha a1, with a0 and a1 formed once per row in double.  cs[a], ds[a]: this
// thread's share of the cost and of the l1 defect at candidate a (a = 0: the
// current point); dn: its share of the cost's directional derivative.
template <int NX, int COST>
__device__ __forceinline__ void ls_rows_ltv(const Prob& P, const LsParams& lp, const float* xbar,
                                            const float* xp, const float* ubar, const float* up,
                                            double (&cs)[kMaxAlphas + 1],
                                            double (&ds)[kMaxAlphas + 1], double& dn) {
  const int tid = threadIdx.x, BT = blockDim.x;
  const int T = P.T, m = P.m, R = P.R, TM = P.TM;
  double al[kMaxAlphas + 1];
#pragma unroll
  for (int a = 0; a <= kMaxAlphas; ++a) {
    al[a] = a <= lp.n ? (double)pick_alpha(lp, a) : 0.0;
    cs[a] = ds[a] = 0.0;
  }
  dn = 0.0;
  constexpr int U = gather_rows<NX>();
  if constexpr (COST == DMPC_COST_DIAG) {
    // the diagonal Hessian and linear term of U rows loaded before any is used
    for (int base = tid; base < R; base += U * BT) {
      float qd[U], ql[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = base + u * BT < R ? base + u * BT : 0;
        qd[u] = P.costp[r];
        ql[u] = P.costp[R + r];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rho = base + u * BT;
        if (rho >= R) continue;
        const double xb = xbar[rho], dx = (double)xp[rho] - xb;
        const double h = qd[u], q = ql[u];
#pragma unroll
        for (int a = 0; a <= kMaxAlphas; ++a) {
          const double x = xb + al[a] * dx;
          cs[a] += a <= lp.n ? 0.5 * h * x * x + q * x : 0.0;
        }
        dn += (h * xb + q) * dx;
      }
    }
  } else {
    for (int rho = tid; rho < R; rho += BT) {
      const int t = rho / NX, i = rho - t * NX;
      const double xb = xbar[rho], dx = (double)xp[rho] - xb;
#pragma unroll
      for (int a = 0; a <= kMaxAlphas; ++a)
        cs[a] += a <= lp.n ? cost_x1<NX>(P, t, i, xb + al[a] * dx, COST) : 0.0;
      dn += dcost_x1<NX>(P, t, i, xb, dx, COST);
    }
  }
  // dynamics defects, rows t < T
  for (int base = tid; base < T * NX; base += U * BT) {
    float ag[U][NX], cv[U];
    gather_A<NX, U, false>(P.A, base, BT, 0, T * NX, ag);
#pragma unroll
    for (int u = 0; u < U; ++u) cv[u] = P.c[base + u * BT < T * NX ? base + u * BT : 0];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int rho = base + u * BT;
      if (rho >= T * NX) continue;
      const int t = rho / NX, i = rho - t * NX;
      const float* Bi = P.B + (t * NX + i) * m;
      const float* xs = xbar + t * NX;
      const float* qs = xp + t * NX;
      double a0 = cv[u], a1 = 0.0;
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        const double xj = xs[j];
        a0 += (double)ag[u][j] * xj;
        a1 += (double)ag[u][j] * ((double)qs[j] - xj);
      }
      for (int l = 0; l < m; ++l) {
        const double ul = ubar[t * m + l];
        a0 += (double)Bi[l] * ul;
        a1 += (double)Bi[l] * ((double)up[t * m + l] - ul);
      }
      const double xn = xbar[rho + NX];
      const double e0 = xn - a0, e1 = ((double)xp[rho + NX] - xn) - a1;
#pragma unroll
      for (int a = 0; a <= kMaxAlphas; ++a) ds[a] += a <= lp.n ? fabs(e0 + al[a] * e1) : 0.0;
    }
  }
  for (int idx = tid; idx < TM; idx += BT) {
    const int t = idx / m, l = idx - t * m;
    const double ub = ubar[idx], du = (double)up[idx] - ub;
#pragma unroll
    for (int a = 0; a <= kMaxAlphas; ++a)
      cs[a] += a <= lp.n ? cost_u1<NX>(P, t, l, ub + al[a] * du, COST) : 0.0;
    dn += dcost_u1<NX>(P, t, l, ubar[idx], up[idx], COST);
  }
}

// QP primal solution (Eq. schur:xu, user signs; accumulated in double):
//   x_t = -Q_t^-1 (q_t + lambda_t - A_t' lambda_{t+1}),  u_t = -R_t^-1 (r_t - B_t' lambda_{t+1})
// lambda from the LDS window w0; then the line search (App. A.3, Alg.
// linesearch) and the SQP update of (x, u).  Returns sel | flags << 8.
template <int NX>
__device__ __forceinline__ LsResult fwd_recover_ls_body(const ProbRec* rec, const float* data,
                                                        float* ws, LsParams lp, int last,
                                                        int recovered) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = blockDim.x, nwv = (BT + 63) >> 6;
  const Prob P = make_prob<NX>(*rec, data, ws);
  const Carve C = carve_of<NX>(P);
  const int T = P.T, N = P.N, m = P.m, R = P.R, TM = P.TM;
  float* xbar = bulk_base(smem, P) + C.xbar;
  float* ubar = bulk_base(smem, P) + C.ubar;
  float* xp = bulk_base(smem, P) + C.xp;
  float* up = bulk_base(smem, P) + C.up;
  const float* w0 = smem + C.w0;   // multipliers, high part
  const float* w2 = smem + C.w2;   // low part
  if (!recovered) {   // (the wave-block kernels recover z in registers: wave_recover)
    const double* iQd = (const double*)(P.Wq + P.L.iQd);
    const double* iRd = (const double*)(P.Wq + P.L.iRd);
    const float* q = P.Wq + P.L.q;
    const float* rr = P.Wq + P.L.r;
      if (P.Ad == nullptr) {
      constexpr int U = gather_rows<NX>();
      for (int base = tid; base < R; base += U * BT) {
        float a[U][NX], qv[U];
        double iq[U];
        gather_A<NX, U, true>(P.A, base, BT, 0, T * NX, a);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int r = base + u * BT < R ? base + u * BT : 0;
          qv[u] = q[r];
          iq[u] = iQd[r];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int rho = base + u * BT;
          if (rho < R) {
            const int t = rho / NX;
            double acc = (double)qv[u] + ((double)w0[NX + rho] + (double)w2[NX + rho]);
            if (t < T) {
              const float* lh = w0 + NX + (t + 1) * NX;
              const float* ll = w2 + NX + (t + 1) * NX;
#pragma unroll
              for (int kk = 0; kk < NX; ++kk) acc -= (double)a[u][kk] * ((double)lh[kk] + (double)ll[kk]);
            }
            xp[rho] = (float)(-acc * iq[u]);
          }
        }
      }
    } else {
      for (int rho = tid; rho < R; rho += BT) {
        const int t = rho / NX, i = rho - t * NX;
        double acc = (double)q[rho] + ((double)w0[NX + rho] + (double)w2[NX + rho]);
        if (t < T) {
          const int a0 = t * NX * NX;
          const float* lh = w0 + NX + (t + 1) * NX;
          const float* ll = w2 + NX + (t + 1) * NX;
#pragma unroll
          for (int kk = 0; kk < NX; ++kk)
            acc -= ldA<double>(P, a0 + kk * NX + i) * ((double)lh[kk] + (double)ll[kk]);
        }
        xp[rho] = (float)(-acc * iQd[rho]);
      }
    }
    for (int idx = tid; idx < TM; idx += BT) {
      const int t = idx / m, l = idx - t * m;
      const int b0 = t * NX * m;
      const float* lh = w0 + NX + (t + 1) * NX;
      const float* ll = w2 + NX + (t + 1) * NX;
      double acc = (double)rr[idx];
#pragma unroll
      for (int kk = 0; kk < NX; ++kk)
        acc -= ldB<double>(P, b0 + kk * m + l) * ((double)lh[kk] + (double)ll[kk]);
      up[idx] = (float)(-acc * iRd[idx]);
    }
  }
  __syncthreads();
  // Task (ai, t): stage t at the current point (ai = 0) or at candidate
  // alphas[ai-1], in double; its cost and dynamics defect go to LDS, one wave
  // then reduces each candidate in a fixed order.  Branch free: lanes past
  // the end and the last stage evaluate clamped stages and discard the result.
  const int na = lp.n;
  const int nrow = na + 1;
  const int ntask = nrow * N;
  double* tc = (double*)(bulk_base(smem, P) + C.ls);
  double* td = tc + (kMaxAlphas + 1) * N;
  double* res = td + (kMaxAlphas + 1) * N;
  double dn = 0.0;   // directional derivative of the cost at the current point (row 0 tasks)
  // per-candidate sums in a fixed order, held in registers by every thread
  double csum[kMaxAlphas + 1], dsum[kMaxAlphas + 1];
  if (P.dyn == DMPC_DYN_LTV) {
    // rows in parallel; wave sums, then the waves' partial sums in order
    if (P.cost == DMPC_COST_DIAG)
      ls_rows_ltv<NX, DMPC_COST_DIAG>(P, lp, xbar, xp, ubar, up, csum, dsum, dn);
    else
      ls_rows_ltv<NX, DMPC_COST_SOFTPLUS>(P, lp, xbar, xp, ubar, up, csum, dsum, dn);
    wave_sum_d_multi<kMaxAlphas + 1>(csum);
    wave_sum_d_multi<kMaxAlphas + 1>(dsum);
    constexpr int K = kMaxAlphas + 1;
    if (nwv > 1 && nwv <= N) {   // (the region holds 2 K (N + 1) doubles: the waves' rows, totals)
      if ((tid & 63) == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          tc[(tid >> 6) * 2 * K + k] = csum[k];
          tc[(tid >> 6) * 2 * K + K + k] = dsum[k];
        }
      }
      __syncthreads();
      // 2 K threads total the waves' rows in order; the others read the totals
      double* tot = tc + nwv * 2 * K;
      if (tid < 2 * K) {
        double acc = 0.0;
        for (int w = 0; w < nwv; ++w) acc += tc[w * 2 * K + tid];
        tot[tid] = acc;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < K; ++k) {
        csum[k] = tot[k];
        dsum[k] = tot[K + k];
      }
      __syncthreads();
    } else if (nwv > 1) {
      double* rd = (double*)(smem + C.red);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if ((tid & 63) == 0) rd[tid >> 6] = csum[k];
        if ((tid & 63) == 0) rd[16 + (tid >> 6)] = dsum[k];
        __syncthreads();
        double c0 = 0.0, d0 = 0.0;
        for (int w = 0; w < nwv; ++w) {
          c0 += rd[w];
          d0 += rd[16 + w];
        }
        csum[k] = c0;
        dsum[k] = d0;
        __syncthreads();
      }
    }
  } else {
    const ModelPar mp = load_par(P);
    const LsTaskArgs ta{xbar, xp, ubar, up, tc, td, &dn, ntask, na};
    // (the cart-pole has nx = 4 and the bicycle nx = 8: other pairs are refused
    // when the problem is validated)
    {
      constexpr int D = NX == 4 ? DMPC_DYN_CARTPOLE : DMPC_DYN_BICYCLE;
      if constexpr (NX == 4 || NX == 8) {
        if (P.cost == DMPC_COST_DIAG) ls_tasks<NX, D, DMPC_COST_DIAG>(P, mp, lp, ta);
        else ls_tasks<NX, D, DMPC_COST_SOFTPLUS>(P, mp, lp, ta);
      }
    }
    __syncthreads();
    if (nwv == 1) {
      // one wave: every row's partial sums first (rows past the last read the
      // last row and count zero), then all the wave sums in one branch-free
      // block, side by side
#pragma unroll
      for (int r = 0; r <= kMaxAlphas; ++r) csum[r] = dsum[r] = 0.0;
      for (int tt = tid; tt < N; tt += 64) {
#pragma unroll
        for (int r = 0; r <= kMaxAlphas; ++r) {
          const int rr = r < nrow ? r : nrow - 1;
          const double cv = tc[rr * N + tt], dv = td[rr * N + tt];
          csum[r] += r < nrow ? cv : 0.0;
          dsum[r] += r < nrow ? dv : 0.0;
        }
      }
      wave_sum_d_multi<kMaxAlphas + 1>(csum);
      wave_sum_d_multi<kMaxAlphas + 1>(dsum);
    } else {
      const int lane = tid & 63;
      for (int r = tid >> 6; r < nrow; r += nwv) {
        double c0 = 0.0, d0 = 0.0;
        for (int tt = lane; tt < N; tt += 64) {
          c0 += tc[r * N + tt];
          d0 += td[r * N + tt];
        }
        c0 = wave_sum_d(c0);
        d0 = wave_sum_d(d0);
        if (lane == 0) {
          res[r] = c0;
          res[kMaxAlphas + 1 + r] = d0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r <= kMaxAlphas; ++r) {
        csum[r] = r < nrow ? res[r] : 0.0;
        dsum[r] = r < nrow ? res[kMaxAlphas + 1 + r] : 0.0;
      }
    }
  }
  const double num = block_sum_d(dn, (double*)(smem + C.red), nwv);
  const double c_cur = csum[0];
  const double fl1 = dsum[0];
  const double mu = fmax(num, 0.0) / fmax(0.5 * fl1, 1e-30);      // Eq. linesearch:penalty
  const double Dmu = num - mu * fl1;                               // Eq. linesearch:descent
  const double phi0 = c_cur + mu * fl1;                            // Eq. linesearch:merit
  int sel = na - 1;                                                // min of the candidates
  bool passed = false;
#pragma unroll
  for (int a = 1; a <= kMaxAlphas; ++a) {
    if (a <= na && !passed) {
      const double al = pick_alpha(lp, a);
      const double dphi = (csum[a] + mu * dsum[a]) - phi0 - (double)lp.eta * al * Dmu;
      if (dphi < 0.f) {   // Eq. linesearch:decrease
        sel = a - 1;
        passed = true;
      }
    }
  }
  int flags = 0;
  if (last && !passed && na > 1) flags |= DMPC_PROB_LS_FALLBACK;
  const float al = pick_alpha(lp, sel + 1);
  if (last) {   // the last linearisation point and QP solution, for the backward pass
    float* xl = P.W + P.L.xlin;
    float* ul = P.W + P.L.ulin;
    float* wx = P.W + P.L.xp;
    float* wu = P.W + P.L.up;
    for (int i = tid; i < R; i += BT) {
      xl[i] = xbar[i];
      wx[i] = xp[i];
    }
    for (int i = tid; i < TM; i += BT) {
      ul[i] = ubar[i];
      wu[i] = up[i];
    }
  }
  __syncthreads();
  for (int i = tid; i < R; i += BT) xbar[i] = fmaf(al, xp[i] - xbar[i], xbar[i]);
  for (int i = tid; i < TM; i += BT) ubar[i] = fmaf(al, up[i] - ubar[i], ubar[i]);
  __syncthreads();
  return LsResult{sel, flags};
}

// Solution output (x, u after the last line search).  Returns NONFINITE bits.
template <int NX>
__device__ __noinline__ int fwd_finish(const ProbRec* rec, const float* data, float* sol,
                                       float* ws) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = blockDim.x;
  const Prob P = make_prob<NX>(*rec, data, ws);
  const Carve C = carve_of<NX>(P);
  const float* xbar = bulk_base(smem, P) + C.xbar;
  const float* ubar = bulk_base(smem, P) + C.ubar;
  float* solx = sol + rec->sol_off;
  float* solu = solx + P.R;
  if (P.flags & kRecLinLds) {
    // the last QP data to the workspace, where the backward pass reads it
    copy_block<true>(P.W, P.Wq, (int)a4h(lin_span(P.T, NX, P.m, P.dyn)));
  }
  int bad = 0;
  for (int i = tid; i < P.R; i += BT) {
    solx[i] = xbar[i];
    if (!isfinite(xbar[i])) bad = 1;
  }
  for (int i = tid; i < P.TM; i += BT) {
    solu[i] = ubar[i];
    if (!isfinite(ubar[i])) bad = 1;
  }
  return __syncthreads_or(bad) ? DMPC_PROB_NONFINITE : 0;
}

// ===========================================================================
// Backward phases
// ===========================================================================
// Loads the last QP's solution and multipliers and writes the adjoint
// right-hand side g~ (float) to the workspace vector.
template <int NX>
__device__ __noinline__ void bwd_begin(const ProbRec* rec, const float* data, float* ws,
                                       const float* dl) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = blockDim.x;
  const Prob P = make_prob<NX>(*rec, data, ws);
  const Carve C = carve_of<NX>(P);
  const int R = P.R, TM = P.TM;
  zero_pads<NX>(smem, C, P);
  for (int i = tid; i < R; i += BT) {
    bulk_base(smem, P)[C.xp + i] = P.W[P.L.xp + i];
    bulk_base(smem, P)[C.lam + i] = P.W[P.L.lam + i];
  }
  for (int i = tid; i < TM; i += BT) bulk_base(smem, P)[C.up + i] = P.W[P.L.up + i];
  if (P.flags & kRecLinLds) {
    stage_lin<NX>(P, *rec, data, true);
    __syncthreads();
  }
  const float* dlx = dl + rec->sol_off;
  const float* dlu = dlx + R;
  const float* dll = dlu + TM;
  float* gv = P.W + P.L.g;
  if (P.Ad == nullptr) {
    constexpr int U = gather_rows<NX>();
    for (int base = tid; base < R; base += U * BT) {
      float ag[U][NX];   // row i of A_{t-1}
      gather_A<NX, U, false>(P.A, base, BT, NX, P.T * NX, ag);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rho = base + u * BT;
        if (rho < R)
          gv[rho] = (float)adjoint_rhs_row<NX, double>(P, rho / NX, rho % NX, dlx, dlu, dll, ag[u]);
      }
    }
  } else {
    for (int rho = tid; rho < R; rho += BT) {
      const int t = rho / NX, i = rho - t * NX;
      gv[rho] = (float)adjoint_rhs_row<NX, double>(P, t, i, dlx, dlu, dll);
    }
  }
  __syncthreads();
}

// Residual of the adjoint Schur system in double, g~ - S^ lambda~ with
// lambda~ = w0 + w2, in factored form as for the forward residual: with the
// adjoint primal point of Alg. backward
//   x~_t = Q_t^-1 (dl/dx_t - lambda~_t + A_t' lambda~_{t+1}),  u~_t = R_t^-1 (dl/du_t + B_t' lambda~_{t+1})
// the rows are  r_0 = x~_0 - dl/dlambda_0,
//   r_{t+1} = x~_{t+1} - A_t x~_t - B_t u~_t - dl/dlambda_{t+1}.
// Result to w1; norms of r and of the adjoint right-hand side (dl/dz, dl/dlambda).
template <int NX>
__device__ __forceinline__ ResNorms bwd_residual64_body(const ProbRec* rec, const float* data,
                                                        float* ws, const float* dl, float kkt_tol) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = blockDim.x;
  const Prob P = make_prob<NX>(*rec, data, ws);
  const Carve C = carve_of<NX>(P);
  const int T = P.T, m = P.m, R = P.R, TM = P.TM;
  const float* w0 = smem + C.w0 + NX;
  const float* w2 = smem + C.w2 + NX;
  float* w1 = smem + C.w1;
  double* xz = (double*)(bulk_base(smem, P) + C.ls);
  double* uz = xz + R;
  const float* dlx = dl + rec->sol_off;
  const float* dlu = dlx + R;
  const float* dll = dlu + TM;
  const double* iQd = (const double*)(P.Wq + P.L.iQd);
  const double* iRd = (const double*)(P.Wq + P.L.iRd);
  const int nwv = (BT + 63) >> 6;
  if (P.Ad == nullptr) {
    constexpr int U = gather_rows<NX>();
    for (int base = tid; base < R; base += U * BT) {
      float a[U][NX], dv[U];
      double iq[U];
      gather_A<NX, U, true>(P.A, base, BT, 0, T * NX, a);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = base + u * BT < R ? base + u * BT : 0;
        dv[u] = dlx[r];
        iq[u] = iQd[r];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rho = base + u * BT;
        if (rho < R) {
          const int t = rho / NX;
          double acc = (double)dv[u] - ((double)w0[rho] + (double)w2[rho]);
          if (t < T) {
#pragma unroll
            for (int k = 0; k < NX; ++k)
              acc += (double)a[u][k] * ((double)w0[(t + 1) * NX + k] + (double)w2[(t + 1) * NX + k]);
          }
          xz[rho] = acc * iq[u];
        }
      }
    }
  } else {
    for (int rho = tid; rho < R; rho += BT) {
      const int t = rho / NX, i = rho - t * NX;
      double acc = (double)dlx[rho] - ((double)w0[rho] + (double)w2[rho]);
      if (t < T) {
        const int a0 = t * NX * NX;
#pragma unroll
        for (int k = 0; k < NX; ++k)
          acc += ldA<double>(P, a0 + k * NX + i) *
                 ((double)w0[(t + 1) * NX + k] + (double)w2[(t + 1) * NX + k]);
      }
      xz[rho] = acc * iQd[rho];
    }
  }
  for (int idx = tid; idx < TM; idx += BT) {
    const int t = idx / m, l = idx - t * m;
    const int b0 = t * NX * m;
    double acc = (double)dlu[idx];
#pragma unroll
    for (int k = 0; k < NX; ++k)
      acc += ldB<double>(P, b0 + k * m + l) *
             ((double)w0[(t + 1) * NX + k] + (double)w2[(t + 1) * NX + k]);
    uz[idx] = acc * iRd[idx];
  }
  __syncthreads();
  float r2 = 0.f, b2 = 0.f;
  auto defect_row = [&](int rho, auto&& aent) {
    const int t = rho / NX, i = rho - t * NX;
    double acc = (double)dll[rho];
    if (t > 0) {
      const int tt = t - 1;
#pragma unroll
      for (int j = 0; j < NX; ++j) acc += aent(tt, i, j) * xz[tt * NX + j];
      for (int l = 0; l < m; ++l) acc += ldB<double>(P, tt * NX * m + i * m + l) * uz[tt * m + l];
    }
    const double res = xz[rho] - acc;
    w1[NX + rho] = (float)res;
    r2 += (float)(res * res);
    b2 += dlx[rho] * dlx[rho] + dll[rho] * dll[rho];
  };
  if (P.Ad == nullptr) {
    constexpr int U = gather_rows<NX>();
    for (int base = tid; base < R; base += U * BT) {
      float a[U][NX];
      gather_A<NX, U, false>(P.A, base, BT, NX, T * NX, a);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rho = base + u * BT;
        if (rho < R) defect_row(rho, [&](int, int, int j) { return (double)a[u][j]; });
      }
    }
  } else {
    for (int rho = tid; rho < R; rho += BT)
      defect_row(rho, [&](int tt, int i, int j) { return ldA<double>(P, tt * NX * NX + i * NX + j); });
  }
  for (int idx = tid; idx < TM; idx += BT) b2 += dlu[idx] * dlu[idx];
  const ResNorms n = block_sum2(r2, b2, smem + C.red, nwv);
  __syncthreads();
  if constexpr (NX == 8 || NX == 12 || NX == 16) {
    // (not when the residual meets the KKT target: the caller stops there,
    // by the same test)
    if ((P.flags & kRecScaled) && !(n.r2 <= kkt_tol * kkt_tol * n.rhs2))
      scaled_rhs<NX>(P, smem + C.w1 + NX, smem + C.w2 + NX);
  }
  return n;
}

// Wave-block refinement residual: the factored residuals above with a lane
// per stage block (block t = lane + 64 b of value slots b NX .. b NX + NX-1)
// and everything in registers.  Lane t forms the primal point of stage t from
// lambda_t and lambda_{t+1} (the next lane's values), then the prediction of
// stage t+1 -- forward c_t + A_t x_t + B_t u_t, backward dl/dlambda_{t+1} +
// A_t x~_t + B_t u~_t -- which the next lane subtracts from its own point; the
// same operations in the same order as the workgroup versions.  rr gets the
// residual rows; returns the norms as they do.
__device__ __forceinline__ double wave_prev_d(double x) {   // lane l <- lane l - 1, lane 0 <- 0
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)u, 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), 0x138, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int NX, int SLOTS, bool BWD>
__device__ __forceinline__ ResNorms wave_residual(const Prob& P, const float (&hi)[SLOTS],
                                                  const float (&lo)[SLOTS], float (&rr)[SLOTS],
                                                  const float* dlx, const float* dlu,
                                                  const float* dll) {
  constexpr int BPL = SLOTS / NX;
  const int lane = threadIdx.x & 63;
  const int T = P.T, N = P.N, m = P.m;
  const float* q = P.Wq + P.L.q;
  const float* rv = P.Wq + P.L.r;
  const double* iQd = (const double*)(P.Wq + P.L.iQd);
  const double* iRd = (const double*)(P.Wq + P.L.iRd);
  float nh[SLOTS], nl[SLOTS], unused[SLOTS];
  wave_neighbours<NX, SLOTS>(hi, unused, nh);
  wave_neighbours<NX, SLOTS>(lo, unused, nl);
  double x[BPL][NX], v[BPL][NX];
  float r2 = 0.f, b2 = 0.f;
#pragma unroll
  for (int b = 0; b < BPL; ++b) {
    const int t = lane + 64 * b;
    const int tc = t < N ? t : N - 1;   // lanes past the horizon load in bounds, count nothing
    double ln[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) ln[k] = (double)nh[b * NX + k] + (double)nl[b * NX + k];
    // (at the last stage lambda_{t+1} = 0: the clamped A_{T-1} adds exact zeros)
    const int tp = tc < T ? tc : T - 1;
    const int a0 = tp * NX * NX;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int rho = tc * NX + i;
      const double lt = (double)hi[b * NX + i] + (double)lo[b * NX + i];
      double acc = BWD ? (double)dlx[rho] - lt : (double)q[rho] + lt;
#pragma unroll
      for (int k = 0; k < NX; ++k) {
        if constexpr (BWD) acc += ldA<double>(P, a0 + k * NX + i) * ln[k];
        else acc -= ldA<double>(P, a0 + k * NX + i) * ln[k];
      }
      x[b][i] = BWD ? acc * iQd[rho] : -acc * iQd[rho];
    }
    // prediction of stage t + 1 (unused at the last stage)
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      double acc = BWD ? (double)dll[(tp + 1) * NX + i] : ldc<double>(P, tp * NX + i);
#pragma unroll
      for (int j = 0; j < NX; ++j) acc += ldA<double>(P, tp * NX * NX + i * NX + j) * x[b][j];
      v[b][i] = acc;
    }
    for (int l = 0; l < m; ++l) {
      const int idx = tp * m + l;
      double acc = BWD ? (double)dlu[idx] : (double)rv[idx];
#pragma unroll
      for (int k = 0; k < NX; ++k) {
        if constexpr (BWD) acc += ldB<double>(P, tp * NX * m + k * m + l) * ln[k];
        else acc -= ldB<double>(P, tp * NX * m + k * m + l) * ln[k];
      }
      const double uz = BWD ? acc * iRd[idx] : -acc * iRd[idx];
#pragma unroll
      for (int i = 0; i < NX; ++i) v[b][i] += ldB<double>(P, tp * NX * m + i * m + l) * uz;
      if (t < T) {
        const float bu = BWD ? dlu[idx] : rv[idx];
        b2 += bu * bu;
      }
    }
  }
#pragma unroll
  for (int b = 0; b < BPL; ++b) {
    const int t = lane + 64 * b;
    const bool live = t < N;
    const int tc = live ? t : N - 1;
    const int tt = tc >= 1 ? tc - 1 : 0;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int rho = tc * NX + i;
      const float d0 = BWD ? dll[i] : P.x0[i];
      const float dc = BWD ? 0.f : P.c[tt * NX + i];
      const float nb = BWD ? dlx[rho] * dlx[rho] + dll[rho] * dll[rho] : q[rho] * q[rho];
      double vp = wave_prev_d(v[b][i]);
      if (b > 0) vp = lane == 0 ? readlane_d(v[b - 1][i], 63) : vp;
      const float dv = t == 0 ? d0 : dc;
      vp = t == 0 ? (double)d0 : vp;
      const double res = x[b][i] - vp;
      rr[b * NX + i] = live ? (float)res : 0.f;
      r2 += live ? (float)(res * res) : 0.f;
      b2 += live ? (BWD ? nb : nb + dv * dv) : 0.f;
    }
  }
  return ResNorms{wave_sum(r2), wave_sum(b2)};
}

// Wave-block recovery of the QP solution (Eq. schur:xu, user signs, in
// double, rounded to float) from the multipliers in registers, a lane per
// stage block: the operations of the recovery in fwd_recover_ls, with the
// next stage's multipliers from the next lane and every load before the
// arithmetic (clamped stages; at the last stage lambda_{t+1} = 0 and the
// clamped A_{T-1} adds exact zeros).  Writes x and u to xp, up.
template <int NX, int SLOTS>
__device__ __forceinline__ void wave_recover(const Prob& P, const float (&hi)[SLOTS],
                                             const float (&lo)[SLOTS], float* xp, float* up) {
  constexpr int BPL = SLOTS / NX;
  const int lane = threadIdx.x & 63;
  const int T = P.T, N = P.N, m = P.m;
  const float* q = P.Wq + P.L.q;
  const float* rv = P.Wq + P.L.r;
  const double* iQd = (const double*)(P.Wq + P.L.iQd);
  const double* iRd = (const double*)(P.Wq + P.L.iRd);
  float nh[SLOTS], nl[SLOTS], unused[SLOTS];
  wave_neighbours<NX, SLOTS>(hi, unused, nh);
  wave_neighbours<NX, SLOTS>(lo, unused, nl);
#pragma unroll
  for (int b = 0; b < BPL; ++b) {
    const int t = lane + 64 * b;
    const bool live = t < N;
    const int tc = live ? t : N - 1;
    const int tp = tc < T ? tc : T - 1;
    double ln[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) ln[k] = (double)nh[b * NX + k] + (double)nl[b * NX + k];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int rho = tc * NX + i;
      double acc = (double)q[rho] + ((double)hi[b * NX + i] + (double)lo[b * NX + i]);
#pragma unroll
      for (int k = 0; k < NX; ++k) acc -= ldA<double>(P, tp * NX * NX + k * NX + i) * ln[k];
      const float x = (float)(-acc * iQd[rho]);
      if (live) xp[rho] = x;
    }
    for (int l = 0; l < m; ++l) {
      const int idx = tp * m + l;
      double acc = (double)rv[idx];
#pragma unroll
      for (int k = 0; k < NX; ++k) acc -= ldB<double>(P, tp * NX * m + k * m + l) * ln[k];
      const float u = (float)(-acc * iRd[idx]);
      if (live && tc < T) up[idx] = u;
    }
  }
}

// Wave-block assembly (Eq. shurcomplement) and stair preconditioner (Eq.
// S_Phiinv) in registers, a lane per stage block: the lane's Schur rows and
// right-hand side from the QP data, D_t^-1 by Gauss-Jordan, and the
// off-diagonal preconditioner blocks with the neighbouring lanes' inverses
// (DPP wave shifts) -- the operations of schur_row and precond_rows in the
// same order.  Branch free: every lane loads the data of stages t-1 and t
// (indices clamped into the horizon) before any arithmetic, and the first
// stage, the last stage and lanes past the horizon select their entries
// (zero rows past the horizon).  With `save` the rows also go to the
// workspace (the backward pass loads them).  Returns true (in every lane) on
// a non-positive pivot.
template <int NX, int SLOTS>
__device__ __forceinline__ bool wave_blocks(const Prob& P, RowRegs<NX, SLOTS, true>& S,
                                            RowRegs<NX, SLOTS, true>& Ph, float (&g)[SLOTS],
                                            bool save) {
  constexpr int BPL = SLOTS / NX;
  const int lane = threadIdx.x & 63;
  const int N = P.N, T = P.T, m = P.m;
  const float* iQ = P.Wq + P.L.iQ;
  const float* qv = P.Wq + P.L.q;
  const float* iR = P.Wq + P.L.iR;
  const float* rv = P.Wq + P.L.r;
  bool nonpd = false;
  float Dv[BPL][NX][NX];
  float Ap[BPL][NX][NX], At[BPL][NX][NX], iQp[BPL][NX], iQt[BPL][NX];
#pragma unroll
  for (int b = 0; b < BPL; ++b) {
    const int t = lane + 64 * b;
    const bool live = t < N;
    const int tc = live ? t : N - 1;
    const int tt = tc >= 1 ? tc - 1 : 0;     // stage t - 1 (clamped)
    const int tn = tc < T ? tc : T - 1;      // stage t as a dynamics stage (clamped)
    float qp[NX], qt[NX], ct[NX], x0[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        Ap[b][i][j] = ldA<float>(P, tt * NX * NX + i * NX + j);
        At[b][i][j] = ldA<float>(P, tn * NX * NX + i * NX + j);
      }
      iQp[b][i] = iQ[tt * NX + i];
      iQt[b][i] = iQ[tc * NX + i];
      qp[i] = qv[tt * NX + i];
      qt[i] = qv[tc * NX + i];
      ct[i] = ldc<float>(P, tt * NX + i);
      x0[i] = P.x0[i];
    }
    // rows of block t (schur_row): general stage, first stage, E_{t,t+1}
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      float* Si = S[b * NX + i];
      float ai[NX], gs = 0.f;
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        ai[j] = Ap[b][i][j] * iQp[b][j];
        gs += ai[j] * qp[j];
      }
      float Dr[NX];
#pragma unroll
      for (int k = 0; k < NX; ++k) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < NX; ++j) acc += ai[j] * Ap[b][k][j];
        Dr[k] = acc;
      }
      for (int l = 0; l < m; ++l) {
        const float bi = ldB<float>(P, tt * NX * m + i * m + l) * iR[tt * m + l];
        gs += bi * rv[tt * m + l];
#pragma unroll
        for (int k = 0; k < NX; ++k) Dr[k] += bi * ldB<float>(P, tt * NX * m + k * m + l);
      }
      const float dq = iQt[b][i];
#pragma unroll
      for (int k = 0; k < NX; ++k) Dr[k] += (k == i) ? dq : 0.f;
      const float gg = -(ct[i] - gs + qt[i] * dq);
      const float g0 = -(x0[i] + qt[i] * dq);
      const bool first = tc == 0;
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        Si[j] = (live && !first) ? -ai[j] : 0.f;
        Si[NX + j] = live ? (first ? ((j == i) ? dq : 0.f) : Dr[j]) : 0.f;
        Si[2 * NX + j] = (live && tc < T) ? -At[b][j][i] * dq : 0.f;
      }
      g[b * NX + i] = live ? (first ? g0 : gg) : 0.f;
    }
    float a[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
      for (int j = 0; j < NX; ++j) a[i][j] = live ? S[b * NX + i][NX + j] : (i == j ? 1.f : 0.f);
    if (gj_invert<NX>(a, Dv[b])) nonpd = true;
  }
#pragma unroll
  for (int b = 0; b < BPL; ++b) {
    const int t = lane + 64 * b;
    const bool live = t < N;
    const int tc = live ? t : N - 1;
    // preconditioner rows of block t (precond_rows): lo = D_t^-1 E_{t,t-1}
    // D_{t-1}^-1, up = D_t^-1 E_{t,t+1} D_{t+1}^-1 (both negated), from row k
    // of the neighbouring inverses
    float lo[NX][NX], up[NX][NX], bq[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        lo[i][j] = 0.f;
        up[i][j] = 0.f;
        bq[i][j] = Dv[b][i][j] * iQt[b][j];
      }
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      float dp[NX], dn[NX];
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        float x = wave_prev(Dv[b][k][j]);
        float y = wave_next(Dv[b][k][j]);
        if (b > 0) {
          const float e = __int_as_float(
              __builtin_amdgcn_readlane(__float_as_int(Dv[b > 0 ? b - 1 : 0][k][j]), 63));
          x = lane == 0 ? e : x;
        }
        if (b < BPL - 1) {
          const float e = __int_as_float(
              __builtin_amdgcn_readlane(__float_as_int(Dv[b < BPL - 1 ? b + 1 : 0][k][j]), 0));
          y = lane == 63 ? e : y;
        }
        dp[j] = x;
        dn[j] = y;
      }
#pragma unroll
      for (int i = 0; i < NX; ++i) {
        float w = 0.f;
#pragma unroll
        for (int j = 0; j < NX; ++j) w = fmaf(Dv[b][i][j], Ap[b][j][k], w);
        w *= iQp[b][k];
        float v = 0.f;
#pragma unroll
        for (int j = 0; j < NX; ++j) v = fmaf(bq[i][j], At[b][k][j], v);
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          lo[i][j] = fmaf(w, dp[j], lo[i][j]);
          up[i][j] = fmaf(v, dn[j], up[i][j]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        Ph[b * NX + i][j] = (live && tc >= 1) ? lo[i][j] : 0.f;
        Ph[b * NX + i][NX + j] = live ? Dv[b][i][j] : 0.f;
        Ph[b * NX + i][2 * NX + j] = (live && tc < T) ? up[i][j] : 0.f;
      }
    if (save && live) {
      float* blk = P.W + P.L.blk;
      float* gv = P.W + P.L.g;
#pragma unroll
      for (int i = 0; i < NX; ++i) {
        const int rho = t * NX + i;
#pragma unroll
        for (int j = 0; j < 3 * NX; ++j) {
          blk[blk_at<NX>(rho, j)] = S[b * NX + i][j];
          blk[blk_at<NX>(rho, 3 * NX + j)] = Ph[b * NX + i][j];
        }
        gv[rho] = g[b * NX + i];
      }
    }
  }
  return __ballot(nonpd ? 1 : 0) != 0;
}

// z~ = G^-1 (dl/dz - H' lambda~) (the recovery step of Alg. backward, in double), then the
// VJP of Eq. loss_gradient, -dF/dtheta' [z~; lambda~], laid out like the data
// arena.  lambda~ from the window w0.
template <int NX>
__device__ __noinline__ void bwd_finish(const ProbRec* rec, const float* data, float* ws,
                                        const float* dl, float* adj, float* grad) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = blockDim.x;
  const Prob P = make_prob<NX>(*rec, data, ws);
  const Carve C = carve_of<NX>(P);
  const int T = P.T, m = P.m, R = P.R, TM = P.TM;
  float* xt = bulk_base(smem, P) + C.xbar;
  float* ut = bulk_base(smem, P) + C.ubar;
  const float* xpl = bulk_base(smem, P) + C.xp;
  const float* upl = bulk_base(smem, P) + C.up;
  const float* laml = bulk_base(smem, P) + C.lam;
  const float* w0 = smem + C.w0;
  const float* lw = w0 + NX;                // lambda~, high part (unpadded view)
  const float* lwl = smem + C.w2 + NX;      // low part
  const double* iQd = (const double*)(P.Wq + P.L.iQd);
  const double* iRd = (const double*)(P.Wq + P.L.iRd);
  const float* dlx = dl + rec->sol_off;
  const float* dlu = dlx + R;
  float* ax = adj + rec->sol_off;
  float* au = ax + R;
  float* al = au + TM;
  auto primal_row = [&](int rho, auto&& aent) {
    const int t = rho / NX;
    double acc = (double)dlx[rho] - ((double)lw[rho] + (double)lwl[rho]);
    if (t < T) {
      const float* lh = lw + (t + 1) * NX;
      const float* ll = lwl + (t + 1) * NX;
#pragma unroll
      for (int kk = 0; kk < NX; ++kk) acc += aent(t, kk) * ((double)lh[kk] + (double)ll[kk]);
    }
    const float v = (float)(acc * iQd[rho]);
    xt[rho] = v;
    ax[rho] = v;
    al[rho] = lw[rho];
  };
  if (P.Ad == nullptr) {
    constexpr int U = gather_rows<NX>();
    for (int base = tid; base < R; base += U * BT) {
      float a[U][NX];
      gather_A<NX, U, true>(P.A, base, BT, 0, T * NX, a);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rho = base + u * BT;
        if (rho < R) primal_row(rho, [&](int, int kk) { return (double)a[u][kk]; });
      }
    }
  } else {
    for (int rho = tid; rho < R; rho += BT) {
      const int i = rho % NX;
      primal_row(rho, [&](int t, int kk) { return ldA<double>(P, t * NX * NX + kk * NX + i); });
    }
  }
  for (int idx = tid; idx < TM; idx += BT) {
    const int t = idx / m, l = idx - t * m;
    const int b0 = t * NX * m;
    const float* lh = lw + (t + 1) * NX;
    const float* ll = lwl + (t + 1) * NX;
    double acc = (double)dlu[idx];
#pragma unroll
    for (int kk = 0; kk < NX; ++kk)
      acc += ldB<double>(P, b0 + kk * m + l) * ((double)lh[kk] + (double)ll[kk]);
    const float v = (float)(acc * iRd[idx]);
    ut[idx] = v;
    au[idx] = v;
  }
  __syncthreads();
  // ---- VJP: -dF/dtheta' [z~; lambda~]
  float* gx0 = grad + rec->x0_off;
  for (int i = tid; i < NX; i += BT) gx0[i] = lw[i];   // d x_s = lambda~_0
  const float* xl = P.W + P.L.xlin;
  const float* ul = P.W + P.L.ulin;
  if (P.cost == DMPC_COST_DIAG) {
    // dq = -x~, dQd = -x~ x (through the PD projection: a clamped entry moves q)
    float* gQ = grad + rec->cost_off;
    float* gq = gQ + R;
    float* gR = gq + R;
    float* gr = gR + TM;
    for (int idx = tid; idx < R; idx += BT) {
      const float h = P.costp[idx];
      const float dq = -xt[idx];
      gq[idx] = dq;
      gQ[idx] = (h >= kPdEps) ? -xt[idx] * xpl[idx] : dq * xl[idx];
    }
    for (int idx = tid; idx < TM; idx += BT) {
      const float h = P.costp[2 * R + idx];
      const float dr = -ut[idx];
      gr[idx] = dr;
      gR[idx] = (h >= kPdEps) ? -ut[idx] * upl[idx] : dr * ul[idx];
    }
  } else {
    // softplus weights: theta (one thread per entry, stages of its phase in
    // order), wscale and wfix get 0, xref
    const int K = P.nw + m;
    const float* th = P.costp;
    const float* xr = sp_xref<NX>(P);
    float* gth = grad + rec->cost_off;
    float* gws = gth + P.phases * K;
    float* gwf = gws + K;
    float* gxr = gwf + (NX - P.nw);
    for (int e = tid; e < P.phases * K; e += BT) {
      const int ph = e / K, j = e - ph * K;
      float dw = 0.f;
      for (int t = 0; t <= T; ++t) {
        if (sp_phase(P, t) != ph) continue;
        if (j < P.nw) {
          const int idx = t * NX + j;
          const bool act = sp_weight(P, t, j) >= kPdEps;
          const float dq = -xt[idx];
          dw += (act ? -xt[idx] * xpl[idx] : 0.f) + dq * (-xr[j] + (act ? 0.f : xl[idx]));
        } else if (t < T) {
          const int idx = t * m + (j - P.nw);
          const bool act = sp_weight(P, t, j) >= kPdEps;
          const float dr = -ut[idx];
          dw += (act ? -ut[idx] * upl[idx] : 0.f) + dr * (act ? 0.f : ul[idx]);
        }
      }
      const float* wsc = th + P.phases * K;
      gth[e] = dw * wsc[j] * sigmoidf(th[e]);
    }
    for (int e = tid; e < K + (NX - P.nw); e += BT) gws[e] = 0.f;   // wscale, wfix
    for (int i = tid; i < NX; i += BT) {
      float d = 0.f;
      for (int t = 0; t <= T; ++t) d += xt[t * NX + i] * sp_wx<NX>(P, t, i);
      gxr[i] = d;   // dq/dxref = -w, dq = -x~
    }
  }
  float* gd = grad + rec->dyn_off;
  if (P.dyn == DMPC_DYN_LTV) {
    // dA_t = lambda_{t+1} x~_t' + lambda~_{t+1} x_t',  dB_t likewise,  dc_t = lambda~_{t+1}
    float* gA = gd;
    float* gB = gA + T * NX * NX;
    float* gc = gB + T * NX * m;
    for (int e = tid; e < T * NX * NX; e += BT) {
      const int t = e / (NX * NX), ij = e - t * NX * NX, i = ij / NX, j = ij - i * NX;
      gA[e] = laml[(t + 1) * NX + i] * xt[t * NX + j] + lw[(t + 1) * NX + i] * xpl[t * NX + j];
    }
    for (int e = tid; e < T * NX * m; e += BT) {
      const int t = e / (NX * m), il = e - t * NX * m, i = il / m, l = il - i * m;
      gB[e] = laml[(t + 1) * NX + i] * ut[t * m + l] + lw[(t + 1) * NX + i] * upl[t * m + l];
    }
    for (int e = tid; e < T * NX; e += BT) gc[e] = lw[NX + e];
  } else {
    const int np = P.dyn == DMPC_DYN_CARTPOLE ? kCartpoleParams : kBicycleParams;
    for (int e = tid; e < np; e += BT) gd[e] = 0.f;
  }
  __syncthreads();
}

// ===========================================================================
// Kernels
// ===========================================================================
typedef void (*KernelFn)(KArgs);
struct KEntry {
  int nx, slots, maxbt, reg;
  KernelFn fwd, bwd;
};

// Loads this thread's register rows (Schur and, without the factored
// preconditioner, preconditioner) from the workspace copy of the assembly.
template <int NX, int SLOTS, bool REG, bool WAVE, bool DINV, bool TAIL, bool SC = false>
__device__ __forceinline__ void load_reg_rows(const Prob& P, RowRegs<NX, SLOTS - TAIL, REG>& S,
                                              RowRegs<NX, SLOTS - TAIL, REG && !DINV>& Ph) {
  if constexpr (SC) {
    // the scaled off-diagonal blocks (coefficients 3 nx .. 5 nx of the row)
    const int tid = threadIdx.x, BT = blockDim.x;
    const float* blk = P.W + P.L.blk;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int rho = row_of<NX, false>(s, tid, BT);
      const bool ok = rho < P.R;
#pragma unroll
      for (int j = 0; j < 2 * NX; ++j) S[s][j] = ok ? blk[blk_at<NX>(rho, 3 * NX + j)] : 0.f;
    }
  } else if constexpr (REG) {
    const int tid = threadIdx.x, BT = block_threads<TAIL>();
    const float* blk = P.W + P.L.blk;
#pragma unroll
    for (int s = 0; s < SLOTS - TAIL; ++s) {
      const int rho = row_of<NX, WAVE>(s, tid, BT);
      const bool ok = rho < P.R;
#pragma unroll
      for (int j = 0; j < 3 * NX; ++j) {
        S[s][j] = ok ? blk[blk_at<NX>(rho, j)] : 0.f;
        if constexpr (!DINV) Ph[s][j] = ok ? blk[blk_at<NX>(rho, 3 * NX + j)] : 0.f;
      }
    }
  }
}

// Loads this thread's rows (Schur, preconditioner, right-hand side); TAIL:
// the Schur rows past the register slots into LDS.
// (lds_kept: the LDS copies of an earlier SQP iteration still hold, as for
// linear dynamics with diagonal costs, whose blocks do not change)
template <int NX, int SLOTS, bool REG, bool WAVE, bool DINV, bool TAIL, bool SC = false>
__device__ __forceinline__ void load_rows(const Prob& P, const Lds& sh,
                                          RowRegs<NX, SLOTS - TAIL, REG>& S,
                                          RowRegs<NX, SLOTS - TAIL, REG && !DINV>& Ph,
                                          float (&g)[SLOTS], bool lds_kept = false) {
  const int tid = threadIdx.x, BT = block_threads<TAIL>();
  const float* gv = P.W + P.L.g;
  if (!lds_kept) {   // (uniform over the workgroup)
    if constexpr (TAIL) {
      const float* blk = P.W + P.L.blk;
      const int base = (SLOTS - 1) * BT, nt = P.R - base;
      for (int e = tid; e < nt * 3 * NX; e += BT) {
        const int k = e / (3 * NX), j = e - k * (3 * NX);
        sh.tail[k * tail_stride(NX) + j] = blk[blk_at<NX>(base + k, j)];
      }
    }
    if constexpr (DINV) {
      // the inverted diagonal blocks (row-major per stage: row rho at rho NX,
      // chunks permuted as dinv_swz says), four 16-byte loads in flight
      static_assert(NX % 4 == 0, "factored preconditioner: nx a multiple of 4");
      constexpr int CH = NX / 4;
      const float4* s4 = reinterpret_cast<const float4*>(P.W + P.L.Dinv);
      float4* d4 = reinterpret_cast<float4*>(sh.dinv);
      const int n4 = P.R * CH;
      int e = tid;
      for (; e + 3 * BT < n4; e += 4 * BT) {
        float4 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = s4[e + q * BT];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = e + q * BT, rho = f / CH, j = f - rho * CH;
          d4[rho * CH + (j ^ dinv_swz<NX>(rho))] = v[q];
        }
      }
      for (; e < n4; e += BT) {
        const int rho = e / CH, j = e - rho * CH;
        d4[rho * CH + (j ^ dinv_swz<NX>(rho))] = s4[e];
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int rho = row_of<NX, WAVE>(s, tid, BT);
    g[s] = rho < P.R ? gv[rho] : 0.f;
  }
  load_reg_rows<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, S, Ph);
}

// Scaled system (kRecScaled): out = L^-1 v, stage by stage, through the
// window w, accumulated in double with the double L_t^-1 (zero above its
// diagonal): for ill-conditioned diagonal blocks a float copy of L^-1 would
// limit what the refinement passes can reach.  (Used for the preconditioned
// norm of the right-hand side; the refinement passes map their residuals in
// the residual call, scaled_rhs.)
template <int NX, int SLOTS>
__device__ __forceinline__ void scale_vec(const Prob& P, float* w, const float (&v)[SLOTS],
                                          float (&out)[SLOTS]) {
  const int tid = threadIdx.x, BT = blockDim.x, R = P.R;
  publish<NX, SLOTS, false, false>(w, v, R);
  __syncthreads();
  const double* Li = (const double*)(P.W + P.L.Lid);
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int rho = row_of<NX, false>(s, tid, BT);
    out[s] = 0.f;
    if (rho < R) {
      const float* wt = w + NX + (rho / NX) * NX;
      const double* row = Li + (int64_t)rho * NX;
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < NX; ++j) acc = fma(row[j], (double)wt[j], acc);
      out[s] = (float)acc;
    }
  }
  __syncthreads();
}

// One QP solve of the Schur system, mixed precision.  lambda = hi + lo is a
// double-float pair carried across SQP iterations (the warm start of Alg.
// pcg).  Each pass computes the residual g - S^ lambda with rows re-assembled
// in double, solves for the correction with the float PCG (Alg. pcg) and adds
// it to (hi, lo).  Pass 0 stops at ||r||_{Phi^-1} <= tol ||g||_{Phi^-1} (the
// paper's relative tolerance); then up to `steps` refinement passes, each to
// relative tolerance ref_tol.  Passes stop once the residual meets the KKT
// target (||r||_2 <= kkt_tol ||rhs||_2) -- before pass 0 too, when the warm
// start already meets it (converged SQP iterates).  SC: the PCG runs on the
// scaled system (scaled_blocks); the residual call returns its right-hand
// side L^-1 r, and the solution is mapped back by L^-T.
template <int NX, int SLOTS, bool REG, bool WAVE, bool DINV, bool TAIL, bool SC,
          typename ResidualFn, typename UnscaleFn>
__device__ __forceinline__ int qp_solve(const Prob& P, const Lds& sh,
                                        RowRegs<NX, SLOTS - TAIL, REG>& S,
                                        RowRegs<NX, SLOTS - TAIL, REG && !DINV>& Ph,
                                        const float (&g)[SLOTS],
                                        float (&hi)[SLOTS], float (&lo)[SLOTS], int steps,
                                        int maxit, float tol, float abs_tol, float ref_tol,
                                        float kkt_tol, int& flags, int& redi, int maxit_flag,
                                        int unmet_flag, ResidualFn residual,
                                        UnscaleFn unscale) {
  float etab = 0.f;   // g'Phi^-1 g, formed when pass 0 runs
  int its = 0;
  float prev_r2 = 0.f;
  bool met = false;
  for (int k = 0; k <= steps; ++k) {
    float rr[SLOTS], d[SLOTS];
    const ResNorms nr = residual(hi, lo, rr);
    if (nr.r2 <= kkt_tol * kkt_tol * nr.rhs2) {   // (k = 0: the warm start already meets it)
      met = true;
      break;
    }
    // a pass that did not halve the residual has reached the float32 floor
    // of this system: further passes would not gain either
    if (k > 0 && nr.r2 > 0.25f * prev_r2) break;
    prev_r2 = nr.r2;
    // register rows are read again after the residual, which is a call at
    // nx > 4: held across it they would be saved through scratch and
    // reloaded from there at every use inside the PCG loop
    if constexpr (REG && !WAVE) load_reg_rows<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, S, Ph);
    if (k == 0) {
      if constexpr (SC) {
        float gt[SLOTS];
        scale_vec<NX, SLOTS>(P, sh.w2, g, gt);
        etab = precond_norm<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, sh, S, Ph, gt, redi);
      } else {
        etab = precond_norm<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, sh, S, Ph, g, redi);
      }
    }
    if constexpr (TAIL) {
      // the multipliers wait in the workspace while the PCG runs: in
      // registers they would crowd out the rows (the PCG loop's fences keep
      // the compiler from carrying them across it)
      const int tid = threadIdx.x, BT = block_threads<TAIL>();
      float* st = P.W + P.L.stash;
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        const int rho = row_of<NX, false>(s, tid, BT);
        if (rho < P.R) {
          st[rho] = hi[s];
          st[P.R + rho] = lo[s];
        }
      }
    }
    if (k == 0)
      its += pcg<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, sh, S, Ph, rr, d, maxit, 0.f,
                                       fmaxf(tol * tol * etab, abs_tol), flags, redi, maxit_flag);
    else
      its += pcg<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, sh, S, Ph, rr, d, maxit, ref_tol, 0.f,
                                       flags, redi, maxit_flag);
    if constexpr (SC) unscale(d);
    if constexpr (TAIL) {
      const int tid = threadIdx.x, BT = block_threads<TAIL>();
      const float* st = P.W + P.L.stash;
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        const int rho = row_of<NX, false>(s, tid, BT);
        hi[s] = rho < P.R ? st[rho] : 0.f;
        lo[s] = rho < P.R ? st[P.R + rho] : 0.f;
      }
    }
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const double v = ((double)hi[s] + (double)lo[s]) + (double)d[s];
      hi[s] = (float)v;
      lo[s] = (float)(v - (double)hi[s]);
    }
    if (k == steps) {
      // the passes ran out: one more residual tells whether the last met it
      float rr2[SLOTS];
      const ResNorms nl = residual(hi, lo, rr2);
      met = nl.r2 <= kkt_tol * kkt_tol * nl.rhs2;
    }
  }
  if (!met) flags |= unmet_flag;
  return its;
}

// The phases that run every SQP iteration (and the refinement residuals) as
// calls, so that their registers are not live across the PCG, or, for the
// smallest state sizes, inlined: the call frames save and restore some sixty
// callee-saved registers per call through scratch, and at nx <= 4 the inlined
// kernels still fit their registers without spills.
template <int NX>
__device__ __noinline__ int fwd_blocks_call(const ProbRec* rec, const float* data, float* ws,
                                            int first) {
  return fwd_blocks_body<NX>(rec, data, ws, first);
}
template <int NX>
__device__ __noinline__ void fwd_form_call(const ProbRec* rec, const float* data, float* ws,
                                           int first) {
  fwd_form_body<NX>(rec, data, ws, first);
}
template <int NX>
__device__ __noinline__ LsResult fwd_recover_ls_call(const ProbRec* rec, const float* data, float* ws,
                                                LsParams lp, int last, int recovered) {
  return fwd_recover_ls_body<NX>(rec, data, ws, lp, last, recovered);
}
template <int NX>
__device__ __noinline__ ResNorms fwd_residual64_call(const ProbRec* rec, const float* data,
                                                     float* ws, float kkt_tol) {
  return fwd_residual64_body<NX>(rec, data, ws, kkt_tol);
}
template <int NX>
__device__ __noinline__ ResNorms bwd_residual64_call(const ProbRec* rec, const float* data,
                                                     float* ws, const float* dl, float kkt_tol) {
  return bwd_residual64_body<NX>(rec, data, ws, dl, kkt_tol);
}
template <int NX>
__device__ __forceinline__ ResNorms fwd_residual64(const ProbRec* rec, const float* data,
                                                   float* ws, float kkt_tol) {
  if constexpr (NX <= 4) return fwd_residual64_body<NX>(rec, data, ws, kkt_tol);
  return fwd_residual64_call<NX>(rec, data, ws, kkt_tol);
}
template <int NX>
__device__ __forceinline__ ResNorms bwd_residual64(const ProbRec* rec, const float* data,
                                                   float* ws, const float* dl, float kkt_tol) {
  if constexpr (NX <= 4) return bwd_residual64_body<NX>(rec, data, ws, dl, kkt_tol);
  return bwd_residual64_call<NX>(rec, data, ws, dl, kkt_tol);
}
template <int NX>
__device__ __forceinline__ int fwd_blocks(const ProbRec* rec, const float* data, float* ws,
                                          int first) {
  if constexpr (NX <= 4) return fwd_blocks_body<NX>(rec, data, ws, first);
  return fwd_blocks_call<NX>(rec, data, ws, first);
}
template <int NX>
__device__ __forceinline__ void fwd_form(const ProbRec* rec, const float* data, float* ws,
                                         int first) {
  if constexpr (NX <= 4) fwd_form_body<NX>(rec, data, ws, first);
  else fwd_form_call<NX>(rec, data, ws, first);
}
template <int NX>
__device__ __forceinline__ LsResult fwd_recover_ls(const ProbRec* rec, const float* data, float* ws,
                                              LsParams lp, int last, int recovered) {
  if constexpr (NX <= 4) return fwd_recover_ls_body<NX>(rec, data, ws, lp, last, recovered);
  return fwd_recover_ls_call<NX>(rec, data, ws, lp, last, recovered);
}

// Refinement residual of the current multipliers (hi + lo) into rr, in the
// thread's row layout: the wave-block version in registers, else through the
// LDS windows and the workgroup residual.
template <int NX, int SLOTS, bool WAVE, bool BWD>
__device__ __forceinline__ ResNorms residual_rows(const ProbRec* rec, const KArgs& a,
                                                  const Prob& P, const Lds& sh,
                                                  const float (&hi)[SLOTS],
                                                  const float (&lo)[SLOTS], float (&rr)[SLOTS]) {
  const float* dlx = BWD ? a.dl + rec->sol_off : nullptr;
  if constexpr (WAVE) {
    return wave_residual<NX, SLOTS, BWD>(P, hi, lo, rr, dlx, BWD ? dlx + P.R : nullptr,
                                         BWD ? dlx + P.R + P.TM : nullptr);
  } else {
    const int tid = threadIdx.x, BT = blockDim.x;
    publish<NX, SLOTS, false, false>(sh.w0, hi, P.R);
    publish<NX, SLOTS, false, false>(sh.w2, lo, P.R);
    __syncthreads();
    ResNorms nr;
    if constexpr (BWD) nr = bwd_residual64<NX>(rec, a.data, a.ws, a.dl, a.kkt_tol);
    else nr = fwd_residual64<NX>(rec, a.data, a.ws, a.kkt_tol);
    // (scaled system: the call left r~ = L^-1 r in w2 unless r met the KKT
    // target, when the caller does not use rr)
    const float* rw = (P.flags & kRecScaled) ? sh.w2 : sh.w1;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int rho = row_of<NX, false>(s, tid, BT);
      rr[s] = rho < P.R ? rw[NX + rho] : 0.f;
    }
    __syncthreads();
    return nr;
  }
}

// Scaled system: the PCG's solution d~ (thread's rows) mapped back to
// d = L^-T d~ through the LDS window w1 and the call above.
template <int NX, int SLOTS>
__device__ __forceinline__ void scaled_solution_rows(const ProbRec* rec, const KArgs& a,
                                                     const Prob& P, const Lds& sh,
                                                     float (&d)[SLOTS]) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = blockDim.x;
  publish<NX, SLOTS, false, false>(sh.w1, d, P.R);
  __syncthreads();
  scaled_solution_call<NX>(rec, a.data, a.ws);
  const float* out = bulk_base(smem, P) + carve_of<NX>(P).ls;
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int rho = row_of<NX, false>(s, tid, BT);
    d[s] = rho < P.R ? out[rho] : 0.f;
  }
  __syncthreads();
}

// MODE: 0 = rows of S^ and Phi^-1 read from the workspace, 1 = rows in
// registers, 2 = rows in registers in the wave-block layout (one wave per
// problem, a lane per stage block, neighbour values by DPP wave shifts),
// 3 = rows of S^ in registers and the preconditioner in factored form with
// the inverted diagonal blocks in LDS (half the registers of mode 1), 4 = as
// 3 with the rows of the last value slot in LDS (for problems a few rows
// past what the register slots of the largest register-resident launch hold),
// 5 = the scaled system (scaled_blocks): rows of the two scaled off-diagonal
// blocks in registers, no preconditioner blocks.
template <int NX, int SLOTS, int MAXBT, int MODE>
__global__ __launch_bounds__(MAXBT) void forward_kernel(KArgs a) {
  constexpr bool REG = MODE != 0, WAVE = MODE == 2, DINV = MODE == 3 || MODE == 4,
                 TAIL = MODE == 4, SC = MODE == 5;
  static_assert(!WAVE || (MAXBT == 64 && SLOTS % NX == 0), "wave-block kernels are one wave");
  static_assert(!TAIL || MAXBT == kTailThreads, "LDS-row kernels: kTailThreads threads");
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = block_threads<TAIL>();
  LsParams lp;
#pragma unroll
  for (int i = 0; i < kMaxAlphas; ++i) lp.alphas[i] = a.alphas[i];
  lp.n = a.n_alphas;
  lp.eta = a.ls_eta;
  for (int pi = a.first + blockIdx.x; pi < a.first + a.count; pi += gridDim.x) {
    const ProbRec* rec = a.recs + pi;
    const Prob P = make_prob<NX>(*rec, a.data, a.ws);
    const Lds sh = lds_of<NX>(smem, P);
    const Carve lds_carve = carve_of<NX>(P);
    float* soll = a.sol + rec->sol_off + P.R + P.TM;
    fwd_begin<NX>(rec, a.data, a.sol, a.ws, a.init);
    float lam[SLOTS], lo[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int rho = row_of<NX, WAVE>(s, tid, BT);
      lam[s] = (rho < P.R && a.init == DMPC_INIT_GIVEN) ? soll[rho] : 0.f;
      lo[s] = 0.f;
    }
    int flags = 0, pcg_total = 0, sel = 0, redi = 0;
    const int maxit = a.pcg_max_iter > 0 ? a.pcg_max_iter : P.R + 10;
    const float rtol = a.refine_tol > 0.f ? a.refine_tol : a.pcg_tol;
    for (int k = 0; k < a.sqp_iters; ++k) {
      RowRegs<NX, SLOTS - TAIL, REG> S;
      RowRegs<NX, SLOTS - TAIL, REG && !DINV> Ph;
      float g[SLOTS];
      if constexpr (WAVE) {
        fwd_form<NX>(rec, a.data, a.ws, k == 0);
        if (wave_blocks<NX, SLOTS>(P, S, Ph, g, k == a.sqp_iters - 1)) flags |= DMPC_PROB_NONPD;
      } else {
        if (fwd_blocks<NX>(rec, a.data, a.ws, k == 0)) flags |= DMPC_PROB_NONPD;
        // linear dynamics, diagonal costs: the assembly of the first
        // iteration stays (see fwd_blocks_body), and so do its LDS copies
        const bool kept = k > 0 && P.dyn == DMPC_DYN_LTV && P.cost == DMPC_COST_DIAG;
        load_rows<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, sh, S, Ph, g, kept);
      }
      pcg_total += qp_solve<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(
          P, sh, S, Ph, g, lam, lo, a.refine_steps, maxit, a.pcg_tol, a.pcg_abs_tol, rtol,
          a.kkt_tol, flags, redi, DMPC_PROB_PCG_MAXITER,
          k == a.sqp_iters - 1 ? DMPC_PROB_KKT_UNMET : 0,
          [&](const float (&h)[SLOTS], const float (&l)[SLOTS], float (&rr)[SLOTS]) {
            return residual_rows<NX, SLOTS, WAVE, false>(rec, a, P, sh, h, l, rr);
          },
          [&](float (&dv)[SLOTS]) {
            if constexpr (SC) scaled_solution_rows<NX, SLOTS>(rec, a, P, sh, dv);
          });
      if constexpr (WAVE) {
        wave_recover<NX, SLOTS>(P, lam, lo, bulk_base(smem, P) + lds_carve.xp,
                                bulk_base(smem, P) + lds_carve.up);
      } else {
        publish<NX, SLOTS, false, WAVE>(sh.w0, lam, P.R);
        publish<NX, SLOTS, false, WAVE>(sh.w2, lo, P.R);
      }
      __syncthreads();
      const LsResult r = fwd_recover_ls<NX>(rec, a.data, a.ws, lp, k == a.sqp_iters - 1, WAVE);
      sel = r.sel;
      flags |= r.flags;
    }
    float* wlam = P.W + P.L.lam;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int rho = row_of<NX, WAVE>(s, tid, BT);
      if (rho < P.R) {
        soll[rho] = lam[s];
        wlam[rho] = lam[s];
      }
    }
    flags |= fwd_finish<NX>(rec, a.data, a.sol, a.ws);
    // every flag source is uniform over the workgroup (block reductions)
    if (tid == 0) {
      a.status[rec->index] = flags;
      a.info[4 * rec->index + 0] = pcg_total;
      a.info[4 * rec->index + 2] = sel;
      a.info[4 * rec->index + 3] = a.sqp_iters;
    }
    __syncthreads();
  }
}

template <int NX, int SLOTS, int MAXBT, int MODE>
__global__ __launch_bounds__(MAXBT) void backward_kernel(KArgs a) {
  constexpr bool REG = MODE != 0, WAVE = MODE == 2, DINV = MODE == 3 || MODE == 4,
                 TAIL = MODE == 4, SC = MODE == 5;
  static_assert(!WAVE || (MAXBT == 64 && SLOTS % NX == 0), "wave-block kernels are one wave");
  static_assert(!TAIL || MAXBT == kTailThreads, "LDS-row kernels: kTailThreads threads");
  extern __shared__ float smem[];
  const int tid = threadIdx.x, BT = block_threads<TAIL>();
  for (int pi = a.first + blockIdx.x; pi < a.first + a.count; pi += gridDim.x) {
    const ProbRec* rec = a.recs + pi;
    const Prob P = make_prob<NX>(*rec, a.data, a.ws);
    const Lds sh = lds_of<NX>(smem, P);
    bwd_begin<NX>(rec, a.data, a.ws, a.dl);
    RowRegs<NX, SLOTS - TAIL, REG> S;
    RowRegs<NX, SLOTS - TAIL, REG && !DINV> Ph;
    float g[SLOTS], lt[SLOTS], lo[SLOTS];
    load_rows<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(P, sh, S, Ph, g);
    const float* alv = a.adj + rec->sol_off + P.R + P.TM;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int rho = row_of<NX, WAVE>(s, tid, BT);
      lt[s] = (rho < P.R && a.bwd_warm) ? alv[rho] : 0.f;
      lo[s] = 0.f;
    }
    __syncthreads();
    int flags = 0, redi = 0;
    const int maxit = a.bwd_max_iter > 0 ? a.bwd_max_iter : P.R + 10;
    const float rtol = a.refine_tol > 0.f ? a.refine_tol : a.bwd_tol;
    const int its = qp_solve<NX, SLOTS, REG, WAVE, DINV, TAIL, SC>(
        P, sh, S, Ph, g, lt, lo, a.refine_steps, maxit, a.bwd_tol, 0.f, rtol, a.kkt_tol, flags,
        redi, DMPC_PROB_BWD_PCG_MAXITER, DMPC_PROB_BWD_KKT_UNMET,
        [&](const float (&h)[SLOTS], const float (&l)[SLOTS], float (&rr)[SLOTS]) {
          return residual_rows<NX, SLOTS, WAVE, true>(rec, a, P, sh, h, l, rr);
        },
        [&](float (&dv)[SLOTS]) {
          if constexpr (SC) scaled_solution_rows<NX, SLOTS>(rec, a, P, sh, dv);
        });
    publish<NX, SLOTS, false, WAVE>(sh.w0, lt, P.R);
    publish<NX, SLOTS, false, WAVE>(sh.w2, lo, P.R);
    __syncthreads();
    bwd_finish<NX>(rec, a.data, a.ws, a.dl, a.adj, a.grad);
    if (tid == 0) {
      a.status[rec->index] |= flags;
      a.info[4 * rec->index + 1] = its;
    }
    __syncthreads();
  }
}

}  // namespace dmpc
