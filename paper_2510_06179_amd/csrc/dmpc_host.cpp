// Host runtime of the C ABI declared in include/dmpc.h: validation, plan
// construction (grouping problems by kernel instantiation, workspace layout,
// descriptor upload) and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <mutex>
#include <string>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <new>
#include <vector>

#include "dmpc.h"
#include "dmpc_internal.h"

using namespace dmpc;

struct dmpc_handle {
  int device;
  void* static_ws;   // device address of this device's copy of `scratch`
};

// Workspace of dmpc_solve_static, for callers that cannot allocate: a
// file-scope device array, one copy per device, held until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host it is a
// stand-in, not a device address); it uses the address hipGetSymbolAddress
// gives for the current device, kept per device below.
constexpr size_t kStaticWsBytes = (size_t)64 << 20;
static __device__ __align__(256) float scratch[kStaticWsBytes / sizeof(float)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ws[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up once per device with
// that device current.  nullptr on failure.
void* static_ws_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static_ws[device]) return g_static_ws[device];
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return nullptr;
  if (prev != device && hipSetDevice(device) != hipSuccess) return nullptr;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (prev != device) hipSetDevice(prev);
  if (e != hipSuccess) return nullptr;
  g_static_ws[device] = ptr;
  return ptr;
}
}  // namespace

struct Group {
  LaunchCfg cfg;
  int first, count;
  double work;     // estimated duration (see group_estimate)
  int lane;        // side stream it runs on in a batched call
};

// Groups of one batched call run concurrently on up to kLanes side streams
// (fork/join through events on the caller's stream), heaviest first onto the
// least-loaded stream.  Four matches the hardware queues a process gets by
// default; DMPC_LANES (1..kLanes) in the environment at plan creation sets
// the number for processes given more queues.
constexpr int kLanes = 16;
constexpr int kDefaultLanes = 4;

// Estimated duration of one problem, for ordering and balancing the groups:
// a workgroup per problem, so a group lasts about as long as its slowest
// problem (once per wave of workgroups over the chip).  Per PCG iteration a
// thread does slots rows of 6 nx coefficients, rows read from the workspace
// cost about four times as much as rows in registers, and the iteration
// count grows with the state size and slowly with the horizon.
static double problem_estimate(const dmpc_problem& p, const LaunchCfg& c) {
  const double row_work = (double)c.slots * 6.0 * p.nx + 40.0;
  const double mode = c.reg == 0 ? 4.0 : 1.0;
  const double iters = 10.0 * p.nx * std::cbrt((double)(p.T + 1));
  return row_work * mode * iters;
}

// A HIP graph of one pass (forward or backward) over every launch group of a
// plan: one kernel node per group, chained per side-stream lane as the
// fork/join launches run them (so at most kLanes groups run at once), built
// at the plan's first batched call of that pass.  Replays reuse it; when the
// caller's buffers differ from the last call's, the nodes' kernel arguments
// are updated in the instantiated graph.
struct PassGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipGraphNode_t> nodes;   // one per group
  KArgs key;                           // the arguments of the last call
  bool failed = false;                 // building failed: launch directly
};

struct dmpc_plan {
  dmpc_handle* h;
  int count;
  std::vector<ProbRec> recs;  // grouped; within a group heaviest first
  std::vector<int> pos;       // pos[problem index] = record index
  std::vector<int> grp;       // grp[record index] = group index
  std::vector<Group> groups;
  ProbRec* d_recs;
  size_t ws_bytes;
  dmpc_opts opts;
  int lanes = 0;                       // side streams (0: launch on the caller's stream)
  hipStream_t side[kLanes] = {};
  hipEvent_t joined[kLanes] = {};
  hipEvent_t fork = nullptr;
  PassGraph pass_graph[2];             // [0] backward, [1] forward
};

namespace dmpc {

const int kStateSizes[] = {2, 3, 4, 8, 12, 16, 32};

bool nx_supported(int nx) {
  for (int v : kStateSizes)
    if (v == nx) return true;
  return false;
}

bool finite_nonneg(float v) { return std::isfinite(v) && v >= 0.f; }

dmpc_status check_opts(const dmpc_opts* o) {
  if (!o) return DMPC_ERR_INVALID_ARG;
  if (o->sqp_iters < 1 || o->sqp_iters > 1000) return DMPC_ERR_INVALID_ARG;
  if (o->pcg_max_iter < 0 || o->bwd_pcg_max_iter < 0) return DMPC_ERR_INVALID_ARG;
  if (!finite_nonneg(o->pcg_tol) || !finite_nonneg(o->pcg_abs_tol) || !finite_nonneg(o->bwd_pcg_tol))
    return DMPC_ERR_INVALID_ARG;
  if (o->n_alphas < 1 || o->n_alphas > kMaxAlphas) return DMPC_ERR_INVALID_ARG;
  for (int i = 0; i < o->n_alphas; ++i) {
    const float a = o->alphas[i];
    if (!(a > 0.f && a <= 1.f)) return DMPC_ERR_INVALID_ARG;
    if (i > 0 && !(a < o->alphas[i - 1])) return DMPC_ERR_INVALID_ARG;
  }
  if (!(o->ls_eta > 0.f && o->ls_eta < 1.f)) return DMPC_ERR_INVALID_ARG;
  if (o->init != DMPC_INIT_GIVEN && o->init != DMPC_INIT_ROLLOUT) return DMPC_ERR_INVALID_ARG;
  if (o->bwd_warm_start != 0 && o->bwd_warm_start != 1) return DMPC_ERR_INVALID_ARG;
  if (o->block_threads != 0 &&
      (o->block_threads < 64 || o->block_threads > 1024 || o->block_threads % 64 != 0))
    return DMPC_ERR_INVALID_ARG;
  if (o->refine_steps < 0 || o->refine_steps > 8 || !finite_nonneg(o->refine_tol) ||
      !finite_nonneg(o->kkt_tol))
    return DMPC_ERR_INVALID_ARG;
  if (o->graph != 0 && o->graph != 1) return DMPC_ERR_INVALID_ARG;
  return DMPC_OK;
}

bool in_arena(int64_t off, int64_t len, int64_t arena) {
  return off >= 0 && len >= 0 && off <= arena && len <= arena - off;
}

dmpc_status check_problem(const dmpc_problem& p, int64_t data_len, int64_t sol_len) {
  if (p.T < 1 || p.T > 1000000) return DMPC_ERR_INVALID_ARG;
  if (p.nx < 1 || p.nx > kMaxNx || p.nu < 1 || p.nu > kMaxNu) return DMPC_ERR_INVALID_ARG;
  if (p.reserved != 0) return DMPC_ERR_INVALID_ARG;
  switch (p.dyn) {
    case DMPC_DYN_LTV:
      break;
    case DMPC_DYN_CARTPOLE:
      if (p.nx != 4 || p.nu != 1) return DMPC_ERR_INVALID_ARG;
      break;
    case DMPC_DYN_BICYCLE:
      if (p.nx != 8 || p.nu != 2) return DMPC_ERR_INVALID_ARG;
      break;
    default:
      return DMPC_ERR_INVALID_ARG;
  }
  switch (p.cost) {
    case DMPC_COST_DIAG:
      if (p.cost_phases != 0 || p.cost_nw != 0) return DMPC_ERR_INVALID_ARG;
      break;
    case DMPC_COST_SOFTPLUS:
      if (p.cost_phases < 1 || p.cost_phases > p.T + 1 || p.cost_nw < 0 || p.cost_nw > p.nx)
        return DMPC_ERR_INVALID_ARG;
      break;
    default:
      return DMPC_ERR_INVALID_ARG;
  }
  if (!in_arena(p.dyn_off, dyn_block_len(p.T, p.nx, p.nu, p.dyn), data_len))
    return DMPC_ERR_INVALID_ARG;
  if (!in_arena(p.cost_off, cost_block_len(p.T, p.nx, p.nu, p.cost, p.cost_phases, p.cost_nw),
                data_len))
    return DMPC_ERR_INVALID_ARG;
  if (!in_arena(p.x0_off, p.nx, data_len)) return DMPC_ERR_INVALID_ARG;
  if (!in_arena(p.sol_off, sol_block_len(p.T, p.nx, p.nu), sol_len)) return DMPC_ERR_INVALID_ARG;
  return DMPC_OK;
}

// Kernel mapping of one problem: its R = (T+1)*nx rows are spread over the
// threads of a workgroup, `slots` rows per thread (wave-block variants: one
// wave, `slots` = rows of the stage blocks a lane holds).  Among the instantiated
// variants that hold the rows, the one with the fewest estimated instructions
// per PCG iteration is taken: every wave repeats the per-iteration overhead
// (reductions, divide, barriers), every row costs its two row products;
// workspace-resident rows cost three times a register-resident one.
struct Variant {
  int slots, maxbt, reg;
};
const Variant kVariants[] = {
    {1, 64, 1},  {2, 64, 1},  {4, 64, 1},  {8, 64, 1},  {1, 128, 1}, {2, 128, 1}, {4, 128, 1},
    {8, 128, 1}, {1, 256, 1}, {2, 256, 1}, {4, 256, 1}, {1, 512, 1}, {2, 512, 1}, {1, 1024, 1},
    {3, 512, 1}, {2, 1024, 1}, {2, 640, 3}, {2, 1024, 3}, {5, 512, 4}, {4, 512, 4},
    {3, 512, 4}, {2, 512, 4}, {5, 512, 5}, {4, 512, 5}, {3, 512, 5}, {2, 512, 5},
    {2, 320, 5}, {1, 320, 5}, {3, 384, 5}, {2, 128, 5}, {3, 192, 5}, {5, 256, 5}, {9, 256, 5},
    {2, 192, 5}, {3, 128, 5}, {3, 576, 5}, {5, 384, 5}, {5, 192, 5}, {3, 384, 5}, {3, 192, 5},
    {4, 256, 0}, {8, 256, 0}, {8, 512, 0}, {2, 1024, 0}, {4, 1024, 0}, {8, 1024, 0}, {12, 1024, 0},
    {2, 64, 2},  {4, 64, 2},  {8, 64, 2},
};

// Whether a problem's LDS regions fit a workgroup under a mapping (the bulk
// regions move to the workspace when they do not fit; the inverted diagonal
// blocks and LDS rows of modes 3 and 4 cannot).
bool lds_fits(const dmpc_problem& p, int slots, int bt, int reg) {
  const int f = rec_flags(p.T, p.nx, p.nu, bt, slots, reg, lin_floats_of(p), 0);
  return lds_floats(p.T, p.nx, p.nu, bt, slots, f, 0) * (int64_t)sizeof(float) <= kLdsBytes;
}

// Process-wide tuning table (rows of 7 int32, see dmpc_set_tuning).
std::mutex g_tune_mu;
std::vector<std::array<int32_t, 7>> g_tune;

bool tuned_cfg(const dmpc_problem& p, LaunchCfg* c) {
  const int64_t R = (int64_t)(p.T + 1) * p.nx;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& r : g_tune) {
    if (r[0] != p.nx || p.T < r[1] || p.T > r[2]) continue;
    const int slots = r[3], maxbt = r[4], reg = r[5], bt = r[6];
    if (!kernel_available(p.nx, slots, maxbt, reg)) continue;
    if ((int64_t)slots * bt < R || !lds_fits(p, slots, bt, reg)) continue;
    if (reg == 4 && bt != kTailThreads) continue;
    if (reg == 5 && bt % p.nx != 0) continue;   // (whole stages per group of bt rows)
    *c = LaunchCfg{p.nx, slots, maxbt, reg, bt, 0, 0};
    return true;
  }
  return false;
}

bool choose_cfg(const dmpc_problem& p, int force_bt, LaunchCfg* c) {
  if (force_bt == 0 && tuned_cfg(p, c)) return true;
  const int64_t R = (int64_t)(p.T + 1) * p.nx;
  const double per_row = 6.0 * p.nx + 10.0, per_wave = 100.0;
  double best = 1e300;
  bool found = false;
  for (const Variant& v : kVariants) {
    if (!kernel_available(p.nx, v.slots, v.maxbt, v.reg)) continue;
    int bt;
    if (force_bt > 0) {
      bt = force_bt;
      if (bt > v.maxbt || R > (int64_t)v.slots * bt) continue;
    } else {
      bt = (int)((R + 64LL * v.slots - 1) / (64LL * v.slots) * 64);
      if (bt > v.maxbt) continue;
    }
    if (v.reg == 5 && bt % p.nx != 0) continue;   // scaled system: whole stages per group
    // LDS-row kernels run with exactly kTailThreads threads
    if (v.reg == 4) {
      if (force_bt > 0 && force_bt != kTailThreads) continue;
      bt = kTailThreads;
      if (R > (int64_t)v.slots * bt) continue;
    }
    if (!lds_fits(p, v.slots, bt, v.reg)) continue;
    const int waves = bt / 64;
    // wave-block variants (reg = 2) need no LDS round trip per row product
    const double row_w = v.reg == 2 ? 0.7 : ((v.reg == 3 || v.reg == 4) ? 1.4 : (v.reg ? 1.0 : 3.0));
    const double cost = waves * (per_wave + v.slots * per_row * row_w) + 1e-3 * v.maxbt;
    if (cost < best) {
      best = cost;
      *c = LaunchCfg{p.nx, v.slots, v.maxbt, v.reg, bt, 0, 0};
      found = true;
    }
  }
  return found;
}

int problem_flags(const dmpc_problem& p, int force_bt) {
  LaunchCfg c;
  if (!nx_supported(p.nx) || !choose_cfg(p, force_bt, &c)) return 0;
  return rec_flags(p.T, p.nx, p.nu, c.bt, c.slots, c.reg, lin_floats_of(p), 0);
}

}  // namespace dmpc

namespace {

KArgs make_args(const dmpc_plan* pl, const float* data, float* sol, void* ws, const float* dl,
                float* adj, float* grad, int32_t* status, int32_t* info) {
  return dmpc::make_kargs(pl->opts, pl->d_recs, data, sol, ws, dl, adj, grad, status, info);
}

}  // namespace

namespace dmpc {

KArgs make_kargs(const dmpc_opts& o, const ProbRec* recs, const float* data, float* sol, void* ws,
                 const float* dl, float* adj, float* grad, int32_t* status, int32_t* info) {
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.recs = recs;
  a.data = data;
  a.sol = sol;
  a.ws = (float*)ws;
  a.dl = dl;
  a.adj = adj;
  a.grad = grad;
  a.status = status;
  a.info = info;
  a.sqp_iters = o.sqp_iters;
  a.pcg_max_iter = o.pcg_max_iter;
  a.n_alphas = o.n_alphas;
  a.init = o.init;
  a.bwd_warm = o.bwd_warm_start;
  a.bwd_max_iter = o.bwd_pcg_max_iter;
  a.pcg_tol = o.pcg_tol;
  a.pcg_abs_tol = o.pcg_abs_tol;
  a.ls_eta = o.ls_eta;
  a.bwd_tol = o.bwd_pcg_tol;
  a.refine_steps = o.refine_steps;
  a.refine_tol = o.refine_tol;
  a.kkt_tol = o.kkt_tol;
  for (int i = 0; i < kMaxAlphas; ++i) a.alphas[i] = i < o.n_alphas ? o.alphas[i] : 0.f;
  return a;
}

}  // namespace

extern "C" {

void dmpc_default_opts(dmpc_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->sqp_iters = 1;
  o->pcg_tol = 1e-6f;
  o->n_alphas = 5;
  const float al[5] = {1.0f, 0.7f, 0.3f, 0.1f, 0.01f};
  for (int i = 0; i < 5; ++i) o->alphas[i] = al[i];
  o->ls_eta = 0.4f;
  o->init = DMPC_INIT_GIVEN;
  o->bwd_pcg_tol = 1e-6f;
  o->refine_steps = 3;
  o->refine_tol = 1e-1f;
  o->kkt_tol = 1e-6f;
  o->graph = 1;
}

const char* dmpc_status_string(dmpc_status s) {
  switch (s) {
    case DMPC_OK: return "ok";
    case DMPC_ERR_INVALID_ARG: return "invalid argument";
    case DMPC_ERR_UNSUPPORTED: return "unsupported problem shape";
    case DMPC_ERR_HIP: return "HIP runtime error";
    case DMPC_ERR_NOMEM: return "out of memory or buffer too small";
  }
  return "unknown status";
}

int32_t dmpc_version(void) { return 100; }

int32_t dmpc_list_variants(int32_t* out, int32_t max_rows) {
  int32_t n = 0;
  for (int nx : kStateSizes)
    for (const Variant& v : kVariants) {
      if (!kernel_available(nx, v.slots, v.maxbt, v.reg)) continue;
      if (out && n < max_rows) {
        out[4 * n] = nx;
        out[4 * n + 1] = v.slots;
        out[4 * n + 2] = v.maxbt;
        out[4 * n + 3] = v.reg;
      }
      ++n;
    }
  return n;
}

dmpc_status dmpc_set_tuning(const int32_t* rows, int32_t n_rows) {
  if (n_rows < 0 || (n_rows > 0 && !rows)) return DMPC_ERR_INVALID_ARG;
  std::vector<std::array<int32_t, 7>> t(n_rows);
  for (int i = 0; i < n_rows; ++i) {
    for (int j = 0; j < 7; ++j) t[i][j] = rows[7 * i + j];
    const auto& r = t[i];
    if (!nx_supported(r[0]) || r[1] < 1 || r[2] < r[1] || r[3] < 1 || r[4] < 64 ||
        r[4] > 1024 || r[5] < 0 || r[5] > 5 || r[6] < 64 || r[6] > r[4] || r[6] % 64 != 0)
      return DMPC_ERR_INVALID_ARG;
    // a wave-block row is one wave holding whole stage blocks per lane
    if (r[5] == 2 && (r[4] != 64 || r[3] % r[0] != 0)) return DMPC_ERR_INVALID_ARG;
    // an LDS-row row runs kTailThreads threads and has a register slot
    if (r[5] == 4 && (r[4] != kTailThreads || r[6] != kTailThreads || r[3] < 2))
      return DMPC_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.swap(t);
  return DMPC_OK;
}

dmpc_status dmpc_choose_mapping(const dmpc_problem* problem, const dmpc_opts* opts, int32_t* out) {
  if (!problem || !out) return DMPC_ERR_INVALID_ARG;
  dmpc_status st = check_opts(opts);
  if (st != DMPC_OK) return st;
  if (problem->T < 1 || problem->nx < 1 || problem->nu < 1) return DMPC_ERR_INVALID_ARG;
  LaunchCfg c;
  if (!nx_supported(problem->nx) || !choose_cfg(*problem, opts->block_threads, &c))
    return DMPC_ERR_UNSUPPORTED;
  out[0] = c.slots;
  out[1] = c.maxbt;
  out[2] = c.reg;
  out[3] = c.bt;
  return DMPC_OK;
}

int32_t dmpc_get_tuning(int32_t* rows, int32_t max_rows) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const int32_t n = (int32_t)g_tune.size();
  for (int i = 0; i < n && i < max_rows && rows; ++i)
    for (int j = 0; j < 7; ++j) rows[7 * i + j] = g_tune[i][j];
  return n;
}

dmpc_status dmpc_validate(const dmpc_problem* problems, int32_t count, int64_t data_len,
                          int64_t sol_len, const dmpc_opts* opts, int32_t* bad_index) {
  if (bad_index) *bad_index = -1;
  if (count < 0 || (count > 0 && !problems) || data_len < 0 || sol_len < 0)
    return DMPC_ERR_INVALID_ARG;
  dmpc_status st = check_opts(opts);
  if (st != DMPC_OK) return st;
  for (int i = 0; i < count; ++i) {
    st = check_problem(problems[i], data_len, sol_len);
    if (st != DMPC_OK) {
      if (bad_index) *bad_index = i;
      return st;
    }
  }
  // solution blocks must not overlap (each workgroup writes its own block)
  std::vector<std::pair<int64_t, int>> sb;
  sb.reserve(count);
  for (int i = 0; i < count; ++i) sb.push_back({problems[i].sol_off, i});
  std::sort(sb.begin(), sb.end());
  for (size_t k = 1; k < sb.size(); ++k) {
    const dmpc_problem& p = problems[sb[k - 1].second];
    if (sb[k - 1].first + sol_block_len(p.T, p.nx, p.nu) > sb[k].first) {
      if (bad_index) *bad_index = sb[k].second;
      return DMPC_ERR_INVALID_ARG;
    }
  }
  for (int i = 0; i < count; ++i) {
    LaunchCfg c;
    if (!nx_supported(problems[i].nx) ||
        !choose_cfg(problems[i], opts->block_threads, &c)) {
      if (bad_index) *bad_index = i;
      return DMPC_ERR_UNSUPPORTED;
    }
  }
  return DMPC_OK;
}

dmpc_status dmpc_workspace_size(const dmpc_problem* problems, int32_t count,
                                const dmpc_opts* opts, size_t* bytes) {
  if (!bytes || count < 0 || (count > 0 && !problems)) return DMPC_ERR_INVALID_ARG;
  int64_t total = 0;
  for (int i = 0; i < count; ++i) {
    const dmpc_problem& p = problems[i];
    if (p.T < 1 || p.nx < 1 || p.nu < 1) return DMPC_ERR_INVALID_ARG;
    total += ws_layout(p.T, p.nx, p.nu, p.dyn, problem_flags(p, opts ? opts->block_threads : 0)).total;
  }
  *bytes = (size_t)total * sizeof(float);
  return DMPC_OK;
}

dmpc_status dmpc_create(dmpc_handle** h, int device) {
  if (!h) return DMPC_ERR_INVALID_ARG;
  *h = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return DMPC_ERR_HIP;
  if (device < 0 || device >= n) return DMPC_ERR_INVALID_ARG;
  void* sws = static_ws_address(device);
  if (!sws) return DMPC_ERR_HIP;
  dmpc_handle* p = new (std::nothrow) dmpc_handle;
  if (!p) return DMPC_ERR_NOMEM;
  p->device = device;
  p->static_ws = sws;
  *h = p;
  return DMPC_OK;
}

dmpc_status dmpc_destroy(dmpc_handle* h) {
  delete h;
  return DMPC_OK;
}

dmpc_status dmpc_plan_create(dmpc_handle* h, const dmpc_problem* problems, int32_t count,
                             int64_t data_len, int64_t sol_len, const dmpc_opts* opts,
                             dmpc_plan** plan) {
  if (!h || !plan) return DMPC_ERR_INVALID_ARG;
  *plan = nullptr;
  dmpc_status st = dmpc_validate(problems, count, data_len, sol_len, opts, nullptr);
  if (st != DMPC_OK) return st;
  dmpc_plan* pl = new (std::nothrow) dmpc_plan;
  if (!pl) return DMPC_ERR_NOMEM;
  pl->h = h;
  pl->count = count;
  pl->opts = *opts;
  pl->d_recs = nullptr;

  // kernel configuration per problem, then group (stable: heaviest first)
  std::vector<LaunchCfg> cfg(count);
  std::vector<int64_t> work(count);
  for (int i = 0; i < count; ++i) {
    choose_cfg(problems[i], opts->block_threads, &cfg[i]);
    const dmpc_problem& p = problems[i];
    work[i] = (int64_t)(p.T + 1) * p.nx * p.nx;
  }
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto key = [&](int i) {
    const LaunchCfg& c = cfg[i];
    return std::make_tuple(c.nx, c.slots, c.maxbt, c.reg, c.bt);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (key(a) != key(b)) return key(a) < key(b);
    return work[a] > work[b];
  });
  pl->recs.resize(count);
  pl->pos.resize(count);
  pl->grp.resize(count);
  int64_t ws_off = 0;
  for (int k = 0; k < count; ++k) {
    const int i = order[k];
    const dmpc_problem& p = problems[i];
    ProbRec r;
    std::memset(&r, 0, sizeof(r));
    r.T = p.T;
    r.nx = p.nx;
    r.nu = p.nu;
    r.dyn = p.dyn;
    r.cost = p.cost;
    r.phases = p.cost_phases;
    r.nw = p.cost_nw;
    r.index = i;
    r.dyn_off = p.dyn_off;
    r.cost_off = p.cost_off;
    r.x0_off = p.x0_off;
    r.sol_off = p.sol_off;
    r.ws_off = ws_off;
    r.slots = cfg[i].slots;
    r.flags = rec_flags(p.T, p.nx, p.nu, cfg[i].bt, cfg[i].slots, cfg[i].reg, lin_floats_of(p),
                        lin_budget(count));
    ws_off += ws_layout(p.T, p.nx, p.nu, p.dyn, r.flags).total;
    pl->recs[k] = r;
    pl->pos[i] = k;
    if (k == 0 || key(order[k - 1]) != key(i)) {
      Group g;
      g.cfg = cfg[i];
      g.first = k;
      g.count = 0;
      g.work = 0.0;
      g.lane = 0;
      g.cfg.lds_bytes = 0;
      pl->groups.push_back(g);
    }
    Group& g = pl->groups.back();
    g.count += 1;
    g.cfg.lds_bytes = std::max(
        g.cfg.lds_bytes,
        (size_t)lds_floats(p.T, p.nx, p.nu, g.cfg.bt, g.cfg.slots, r.flags, lin_floats_of(p)) *
            sizeof(float));
    g.work = std::max(g.work, problem_estimate(p, cfg[i]));
    pl->grp[k] = (int)pl->groups.size() - 1;
  }
  pl->ws_bytes = (size_t)ws_off * sizeof(float);
  for (Group& g : pl->groups) {
    // one more slowest-problem duration per extra wave of workgroups
    g.work *= (double)((g.count + kComputeUnits - 1) / kComputeUnits);
    g.cfg.grid = g.count;
    if (g.cfg.lds_bytes > (size_t)kLdsBytes ||
        !kernel_available(g.cfg.nx, g.cfg.slots, g.cfg.maxbt, g.cfg.reg)) {
      delete pl;
      return DMPC_ERR_UNSUPPORTED;
    }
  }
  if (count > 0) {
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(h->device) != hipSuccess) {
      delete pl;
      return DMPC_ERR_HIP;
    }
    const size_t bytes = sizeof(ProbRec) * (size_t)count;
    if (hipMalloc((void**)&pl->d_recs, bytes) != hipSuccess) {
      hipSetDevice(prev);
      delete pl;
      return DMPC_ERR_NOMEM;
    }
    if (hipMemcpy(pl->d_recs, pl->recs.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(pl->d_recs);
      hipSetDevice(prev);
      delete pl;
      return DMPC_ERR_HIP;
    }
    if (pl->groups.size() > 1) {
      // longest-processing-time assignment of groups to side streams; the
      // groups are kept heaviest first, which is also their launch order
      int want = kDefaultLanes;
      if (const char* e = std::getenv("DMPC_LANES")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= kLanes) want = v;
      }
      const int lanes = std::min<int>(want, (int)pl->groups.size());
      std::stable_sort(pl->groups.begin(), pl->groups.end(),
                       [](const Group& a, const Group& b) { return a.work > b.work; });
      for (size_t g = 0; g < pl->groups.size(); ++g)
        for (int k = pl->groups[g].first; k < pl->groups[g].first + pl->groups[g].count; ++k)
          pl->grp[k] = (int)g;
      std::vector<int> gi(pl->groups.size());
      for (size_t g = 0; g < gi.size(); ++g) gi[g] = (int)g;
      double load[kLanes] = {};
      for (int g : gi) {
        int best = 0;
        for (int l = 1; l < lanes; ++l)
          if (load[l] < load[best]) best = l;
        pl->groups[g].lane = best;
        load[best] += pl->groups[g].work;
      }
      bool ok = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming) == hipSuccess;
      for (int l = 0; l < lanes && ok; ++l)
        ok = hipStreamCreateWithFlags(&pl->side[l], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&pl->joined[l], hipEventDisableTiming) == hipSuccess;
      pl->lanes = lanes;
      if (!ok) {
        dmpc_plan_destroy(pl);
        hipSetDevice(prev);
        return DMPC_ERR_HIP;
      }
    }
    hipSetDevice(prev);
  }
  *plan = pl;
  return DMPC_OK;
}

dmpc_status dmpc_plan_workspace_size(const dmpc_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return DMPC_ERR_INVALID_ARG;
  *bytes = plan->ws_bytes;
  return DMPC_OK;
}

dmpc_status dmpc_workspace_offsets(const dmpc_plan* plan, int32_t index, int64_t* out) {
  if (!plan || !out || index < 0 || index >= plan->count) return DMPC_ERR_INVALID_ARG;
  const ProbRec& r = plan->recs[plan->pos[index]];
  const WsLayout L = ws_layout(r.T, r.nx, r.nu, r.dyn, r.flags);
  const int64_t v[7] = {L.xlin, L.ulin, L.xp, L.up, L.lam, L.Qd, L.Rd};
  for (int i = 0; i < 7; ++i) out[i] = r.ws_off + v[i];
  return DMPC_OK;
}

dmpc_status dmpc_plan_describe(const dmpc_plan* plan, char* buf, size_t len) {
  if (!plan || !buf || len == 0) return DMPC_ERR_INVALID_ARG;
  std::string s = "[";
  for (size_t g = 0; g < plan->groups.size(); ++g) {
    const LaunchCfg& c = plan->groups[g].cfg;
    char tmp[256];
    std::snprintf(tmp, sizeof(tmp),
                  "%s{\"nx\": %d, \"slots\": %d, \"block_threads\": %d, \"launch_bound\": %d, "
                  "\"register_rows\": %d, \"problems\": %d, \"lds_bytes\": %zu, \"stream\": %d}",
                  g ? ", " : "", c.nx, c.slots, c.bt, c.maxbt, c.reg, plan->groups[g].count,
                  c.lds_bytes, plan->lanes ? plan->groups[g].lane : -1);
    s += tmp;
  }
  s += "]";
  std::snprintf(buf, len, "%s", s.c_str());
  return DMPC_OK;
}

dmpc_status dmpc_plan_destroy(dmpc_plan* plan) {
  if (!plan) return DMPC_OK;
  for (PassGraph& g : plan->pass_graph) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    if (g.graph) hipGraphDestroy(g.graph);
  }
  for (int l = 0; l < kLanes; ++l) {
    if (plan->side[l]) hipStreamDestroy(plan->side[l]);
    if (plan->joined[l]) hipEventDestroy(plan->joined[l]);
  }
  if (plan->fork) hipEventDestroy(plan->fork);
  if (plan->d_recs) hipFree(plan->d_recs);
  delete plan;
  return DMPC_OK;
}

static bool same_buffers(const KArgs& a, const KArgs& b) {
  return a.data == b.data && a.sol == b.sol && a.ws == b.ws && a.dl == b.dl && a.adj == b.adj &&
         a.grad == b.grad && a.status == b.status && a.info == b.info;
}

static hipKernelNodeParams node_params(const Group& g, const void* fn, KArgs* a) {
  hipKernelNodeParams p;
  std::memset(&p, 0, sizeof(p));
  p.func = const_cast<void*>(fn);
  p.gridDim = dim3(g.cfg.grid);
  p.blockDim = dim3(g.cfg.bt);
  p.sharedMemBytes = (unsigned)g.cfg.lds_bytes;
  static thread_local void* args[1];
  args[0] = a;
  p.kernelParams = args;
  p.extra = nullptr;
  return p;
}

// Replays the pass's graph on `stream` (building or updating it first).
// Returns 0, or -2 when a HIP call failed; -3 when the graph cannot be built
// (the caller then launches the groups directly).
static int run_graph(dmpc_plan* pl, bool fwd, const KArgs& a, hipStream_t stream) {
  PassGraph& pg = pl->pass_graph[fwd ? 1 : 0];
  if (pg.failed) return -3;
  const size_t ng = pl->groups.size();
  if (!pg.exec) {
    if (hipGraphCreate(&pg.graph, 0) != hipSuccess) {
      pg.failed = true;
      return -3;
    }
    pg.nodes.assign(ng, nullptr);
    std::vector<hipGraphNode_t> last(kLanes, nullptr);
    for (size_t i = 0; i < ng; ++i) {
      const Group& g = pl->groups[i];
      const void* fn = kernel_function(g.cfg, fwd);
      KArgs ai = a;
      ai.first = g.first;
      ai.count = g.count;
      const int lane = pl->lanes ? g.lane : 0;
      hipKernelNodeParams p = node_params(g, fn, &ai);
      hipGraphNode_t dep = last[lane];
      if (!fn || hipGraphAddKernelNode(&pg.nodes[i], pg.graph, dep ? &dep : nullptr, dep ? 1 : 0,
                                       &p) != hipSuccess) {
        pg.failed = true;
        return -3;
      }
      last[lane] = pg.nodes[i];
    }
    if (hipGraphInstantiate(&pg.exec, pg.graph, nullptr, nullptr, 0) != hipSuccess) {
      pg.exec = nullptr;
      pg.failed = true;
      return -3;
    }
    pg.key = a;
  } else if (!same_buffers(a, pg.key)) {
    for (size_t i = 0; i < ng; ++i) {
      const Group& g = pl->groups[i];
      KArgs ai = a;
      ai.first = g.first;
      ai.count = g.count;
      hipKernelNodeParams p = node_params(g, kernel_function(g.cfg, fwd), &ai);
      if (hipGraphExecKernelNodeSetParams(pg.exec, pg.nodes[i], &p) != hipSuccess) return -2;
    }
    pg.key = a;
  }
  return hipGraphLaunch(pg.exec, stream) == hipSuccess ? 0 : -2;
}

static dmpc_status run(dmpc_plan* pl, int index, bool fwd, const float* data, float* sol,
                       const float* dl, float* adj, float* grad, void* ws, int32_t* status,
                       int32_t* info, void* stream) {
  if (!pl) return DMPC_ERR_INVALID_ARG;
  if (pl->count == 0) return DMPC_OK;
  if (!data || !ws || !status || !info) return DMPC_ERR_INVALID_ARG;
  if (fwd && !sol) return DMPC_ERR_INVALID_ARG;
  if (!fwd && (!dl || !adj || !grad)) return DMPC_ERR_INVALID_ARG;
  if (index >= pl->count) return DMPC_ERR_INVALID_ARG;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return DMPC_ERR_HIP;
  if (prev != pl->h->device && hipSetDevice(pl->h->device) != hipSuccess) return DMPC_ERR_HIP;
  KArgs a = make_args(pl, data, sol, ws, dl, adj, grad, status, info);
  int rc = 0;
  if (index < 0 && pl->opts.graph) {
    rc = run_graph(pl, fwd, a, (hipStream_t)stream);
    if (rc != -3) {
      if (prev != pl->h->device) hipSetDevice(prev);
      return rc == 0 ? DMPC_OK : DMPC_ERR_HIP;
    }
    rc = 0;   // the graph could not be built: launch the groups directly
  }
  if (index >= 0) {
    const int k = pl->pos[index];
    LaunchCfg c = pl->groups[pl->grp[k]].cfg;
    c.grid = 1;
    a.first = k;
    a.count = 1;
    rc = fwd ? launch_forward(c, a, stream) : launch_backward(c, a, stream);
  } else if (pl->lanes == 0) {
    for (const Group& g : pl->groups) {
      a.first = g.first;
      a.count = g.count;
      rc = fwd ? launch_forward(g.cfg, a, stream) : launch_backward(g.cfg, a, stream);
      if (rc != 0) break;
    }
  } else {
    // fork: every side stream waits for the caller's stream; join: the
    // caller's stream waits for every side stream
    hipStream_t st = (hipStream_t)stream;
    if (hipEventRecord(pl->fork, st) != hipSuccess) rc = -2;
    for (int l = 0; l < pl->lanes && rc == 0; ++l)
      if (hipStreamWaitEvent(pl->side[l], pl->fork, 0) != hipSuccess) rc = -2;
    for (const Group& g : pl->groups) {
      if (rc != 0) break;
      a.first = g.first;
      a.count = g.count;
      hipStream_t ls = pl->side[g.lane];
      rc = fwd ? launch_forward(g.cfg, a, ls) : launch_backward(g.cfg, a, ls);
    }
    for (int l = 0; l < pl->lanes; ++l) {
      if (hipEventRecord(pl->joined[l], pl->side[l]) != hipSuccess ||
          hipStreamWaitEvent(st, pl->joined[l], 0) != hipSuccess)
        rc = rc ? rc : -2;
    }
  }
  if (prev != pl->h->device) hipSetDevice(prev);
  if (rc == -1) return DMPC_ERR_UNSUPPORTED;
  return rc == 0 ? DMPC_OK : DMPC_ERR_HIP;
}

dmpc_status dmpc_solve(dmpc_plan* plan, const float* data, float* sol, void* workspace,
                       int32_t* status, int32_t* info, void* stream) {
  return run(plan, -1, true, data, sol, nullptr, nullptr, nullptr, workspace, status, info, stream);
}

dmpc_status dmpc_solve_static(dmpc_plan* plan, const float* data, float* sol, int32_t* status,
                              int32_t* info, void* stream) {
  if (!plan) return DMPC_ERR_INVALID_ARG;
  if (plan->ws_bytes > kStaticWsBytes) return DMPC_ERR_NOMEM;
  return run(plan, -1, true, data, sol, nullptr, nullptr, nullptr, plan->h->static_ws, status,
             info, stream);
}

dmpc_status dmpc_solve_backward(dmpc_plan* plan, const float* data, const float* dl_dsol,
                                float* adj, float* grad, void* workspace, int32_t* status,
                                int32_t* info, void* stream) {
  return run(plan, -1, false, data, nullptr, dl_dsol, adj, grad, workspace, status, info, stream);
}

dmpc_status dmpc_solve_jvp(dmpc_plan* plan, const float* data, const float* tangent, float* rhs,
                           float* out, float* grad, void* workspace, int32_t* status,
                           int32_t* info, void* stream) {
  if (!plan) return DMPC_ERR_INVALID_ARG;
  if (plan->count == 0) return DMPC_OK;
  if (!data || !tangent || !rhs || !out || !grad || !workspace || !status || !info)
    return DMPC_ERR_INVALID_ARG;
  for (const ProbRec& r : plan->recs)
    if (r.cost != DMPC_COST_DIAG) return DMPC_ERR_UNSUPPORTED;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return DMPC_ERR_HIP;
  if (prev != plan->h->device && hipSetDevice(plan->h->device) != hipSuccess) return DMPC_ERR_HIP;
  const int rc = launch_jvp_rhs(plan->d_recs, plan->count, data, tangent, (const float*)workspace,
                                rhs, stream);
  if (prev != plan->h->device) hipSetDevice(prev);
  if (rc != 0) return DMPC_ERR_HIP;
  // K is symmetric: the adjoint solve with the JVP right-hand side returns dw
  return run(plan, -1, false, data, nullptr, rhs, out, grad, workspace, status, info, stream);
}

dmpc_status dmpc_solve_one(dmpc_plan* plan, int32_t index, const float* data, float* sol,
                           void* workspace, int32_t* status, int32_t* info, void* stream) {
  if (index < 0) return DMPC_ERR_INVALID_ARG;
  return run(plan, index, true, data, sol, nullptr, nullptr, nullptr, workspace, status, info,
             stream);
}

dmpc_status dmpc_solve_backward_one(dmpc_plan* plan, int32_t index, const float* data,
                                    const float* dl_dsol, float* adj, float* grad,
                                    void* workspace, int32_t* status, int32_t* info,
                                    void* stream) {
  if (index < 0) return DMPC_ERR_INVALID_ARG;
  return run(plan, index, false, data, nullptr, dl_dsol, adj, grad, workspace, status, info,
             stream);
}

}  // extern "C"
