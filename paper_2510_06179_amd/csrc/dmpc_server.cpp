// Continuous-batching server of the C ABI (dmpc_server_* in include/dmpc.h).
//
// Threads: callers submit into a FIFO; one dispatcher thread forms launch
// groups whenever an in-flight share (stream + workspace + staging) is free;
// one completion thread per share waits for its group's event, copies the
// results out of pinned staging into per-ticket host results and frees the
// share and the group's sessions.
//
// Device work of a group, all on the share's stream:
//   1. one host-to-device copy of [records | segments | x_s and cotangent payload]
//   2. scatter kernel: payload -> session stores (x_s into the data block,
//      cotangent into the cotangent store)
//   3. forward launches, one per kernel instantiation present in the group
//   4. backward launches over the backward requests (ordered first in each
//      instantiation's record range)
//   5. gather kernel: solution and gradient blocks -> result staging
//   6. one device-to-host copy of [status | info | results], event record
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "dmpc.h"
#include "dmpc_internal.h"

using namespace dmpc;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int64_t kDefaultStaging = 64ll << 20;
constexpr int kTraceKeep = 1024;

int64_t a256(int64_t v) { return (v + 255) / 256 * 256; }
int64_t a4(int64_t v) { return (v + 3) / 4 * 4; }

struct Session {
  bool used = false;
  dmpc_problem p{};      // offsets rebased into the server stores
  LaunchCfg cfg{};
  int flags = 0;         // ProbRec::flags
  bool heavy = false;    // too large for LDS: runs in groups of its own (see form_group)
  int64_t data_len = 0, sol_len = 0, ws_floats = 0;
  int queued = 0;        // requests pending or in flight
  bool busy = false;     // a request in flight
};

struct Request {
  int64_t ticket = 0;
  int32_t session = 0, backward = 0;
  bool has_x0 = false, has_dl = false;
  float x0[kMaxNx];
  std::vector<float> dl;
  double t_submit = 0;
};

struct Result {
  int state = DMPC_REQ_PENDING;
  int32_t status = 0;
  int32_t info[4] = {0, 0, 0, 0};
  std::vector<float> sol, grad;
  double t_submit = 0, t_done = 0;
};

struct GroupTrace {
  int64_t id = 0;
  int slot = 0;
  std::vector<int64_t> tickets;
  int64_t ws_bytes = 0;
  double t_launch = 0, t_done = 0;
};

// Per-request staging footprint (bytes), conservative: the group layout adds
// at most 2 x 255 bytes of alignment per region, reserved once per group.
int64_t est_in(const Session& s, const Request& r) {
  return (int64_t)sizeof(ProbRec) + 4 * (int64_t)sizeof(Seg) + 4 * a4(s.p.nx) +
         (r.has_dl ? 4 * a4(s.sol_len) : 0);
}
int64_t est_out(const Session& s, const Request& r) {
  return 4 + 16 + 4 * a4(s.sol_len) + (r.backward ? 4 * a4(s.data_len) : 0);
}

struct Slot {
  int id = 0;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  float* d_ws = nullptr;
  char* h_in = nullptr;
  char* d_in = nullptr;
  char* h_out = nullptr;
  char* d_out = nullptr;
  // group in flight
  std::vector<Request> reqs;          // record order
  std::vector<int64_t> out_sol, out_grad;   // byte offsets of each request's results
  int64_t status_off = 0, info_off = 0, out_used = 0;
  int64_t ws_bytes = 0;
  int64_t group_id = -1;
  bool busy = false, launched = false, failed = false;
  bool heavy = false;   // the group holds heavy requests
  double t_launch = 0;
  std::thread th;
  std::condition_variable cv;
};

}  // namespace

struct dmpc_server {
  dmpc_server_config cfg{};
  Clock::time_point t0;
  int64_t data_stride = 0, sol_stride = 0;
  int64_t ws_share = 0, staging = 0;

  // device stores [max_sessions] blocks
  float* d_data = nullptr;
  float* d_grad = nullptr;
  float* d_sol = nullptr;
  float* d_adj = nullptr;
  float* d_dl = nullptr;

  std::mutex mu;
  std::condition_variable cv_disp, cv_res;
  bool stop = false;
  std::vector<Session> sessions;
  std::list<Request> pending;
  std::unordered_map<int64_t, Result> results;
  std::vector<std::unique_ptr<Slot>> slots;
  std::thread dispatcher;
  int64_t next_ticket = 1, next_group = 0;

  // statistics
  int64_t accepted_total = 0, finished_total = 0;
  int64_t st_submitted = 0, st_rejected = 0, st_completed = 0, st_bwd = 0, st_failed = 0;
  int64_t st_groups = 0, st_group_reqs = 0, st_max_group = 0, st_max_pending = 0;
  double st_first_submit = -1, st_last_done = 0;
  std::vector<double> latencies, lat_light, lat_heavy;
  int heavy_inflight = 0;
  int max_heavy = 1;    // heavy groups in flight at once
  std::deque<GroupTrace> trace;

  double now() const {
    return std::chrono::duration<double>(Clock::now() - t0).count();
  }
  bool dry() const { return cfg.dry_run != 0; }

  void run_dispatcher();
  void run_slot(Slot* s);
  bool ready_request() const;
  Slot* free_slot();
  void form_group(Slot* s);
  bool launch_group(Slot* s);
  void finish_group(Slot* s);
  void release();
};

namespace {

int64_t max_data_len(int T, int nx, int nu) {
  const int64_t dyn = std::max<int64_t>(dyn_block_len(T, nx, nu, DMPC_DYN_LTV), kBicycleParams);
  const int64_t diag = cost_block_len(T, nx, nu, DMPC_COST_DIAG, 0, 0);
  const int64_t soft = cost_block_len(T, nx, nu, DMPC_COST_SOFTPLUS, T + 1, nx);
  return dyn + std::max(diag, soft) + nx + 64;
}

dmpc_status check_config(const dmpc_server_config* c) {
  if (!c) return DMPC_ERR_INVALID_ARG;
  if (c->max_sessions < 1 || c->max_batch < 1 || c->max_batch > 65536) return DMPC_ERR_INVALID_ARG;
  if (c->max_inflight < 1 || c->max_inflight > 8) return DMPC_ERR_INVALID_ARG;
  if (c->max_T < 1 || c->max_nx < 1 || c->max_nx > kMaxNx || c->max_nu < 1 || c->max_nu > kMaxNu)
    return DMPC_ERR_INVALID_ARG;
  if (c->max_pending < 0 || c->batch_window_us < 0 || c->batch_window_us > 1000000)
    return DMPC_ERR_INVALID_ARG;
  if ((c->dry_run != 0 && c->dry_run != 1) || c->dry_run_us < 0) return DMPC_ERR_INVALID_ARG;
  if (c->reserved != 0 || c->hbm_budget <= 0 || c->staging_bytes < 0) return DMPC_ERR_INVALID_ARG;
  dmpc_status st = check_opts(&c->opts);
  if (st != DMPC_OK) return st;
  if (c->opts.init != DMPC_INIT_GIVEN) return DMPC_ERR_INVALID_ARG;
  return DMPC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// dispatcher
// ---------------------------------------------------------------------------
bool dmpc_server::ready_request() const {
  for (const Request& r : pending) {
    const Session& ss = sessions[r.session];
    if (!ss.busy && (!ss.heavy || heavy_inflight < max_heavy)) return true;
  }
  return false;
}

Slot* dmpc_server::free_slot() {
  for (auto& s : slots)
    if (!s->busy) return s.get();
  return nullptr;
}

// Takes pending requests in arrival order into slot s (lock held).  Requests
// of a session already in flight (or already taken) are skipped and keep their
// place; admission stops at the first request that would overflow the
// group's workspace share or staging, so a large request is never overtaken.
void dmpc_server::form_group(Slot* s) {
  s->reqs.clear();
  // A group holds light or heavy requests, never both, and at most max_heavy
  // heavy groups run at once: a heavy request (one whose bulk regions live in
  // the workspace, far slower than the rest) never holds up light ones that
  // share its group, and light requests always have a share to run in.  The
  // class is that of the oldest request that can run now.
  bool heavy = false;
  for (const Request& r : pending) {
    const Session& ss = sessions[r.session];
    if (ss.busy || (ss.heavy && heavy_inflight >= max_heavy)) continue;
    heavy = ss.heavy;
    break;
  }
  s->heavy = heavy;
  int64_t ws = 0, in = 512, out = 512;
  for (auto it = pending.begin(); it != pending.end() && (int)s->reqs.size() < cfg.max_batch;) {
    Session& ss = sessions[it->session];
    if (ss.busy || ss.heavy != heavy) {
      ++it;
      continue;
    }
    const int64_t w = ss.ws_floats * 4, ei = est_in(ss, *it), eo = est_out(ss, *it);
    if (ws + w > ws_share || in + ei > staging || out + eo > staging) break;
    ws += w;
    in += ei;
    out += eo;
    ss.busy = true;
    results[it->ticket].state = DMPC_REQ_RUNNING;
    s->reqs.push_back(std::move(*it));
    it = pending.erase(it);
  }
  s->ws_bytes = ws;
}

void dmpc_server::run_dispatcher() {
  if (!dry()) hipSetDevice(cfg.device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_disp.wait(lk, [&] { return stop || (free_slot() && ready_request()); });
    if (stop) break;
    if (cfg.batch_window_us > 0 && (int)pending.size() < cfg.max_batch) {
      cv_disp.wait_for(lk, std::chrono::microseconds(cfg.batch_window_us),
                       [&] { return stop || (int)pending.size() >= cfg.max_batch; });
      if (stop) break;
    }
    Slot* s = free_slot();
    if (!s) continue;
    form_group(s);
    if (s->reqs.empty()) continue;
    if (s->heavy) heavy_inflight += 1;
    s->busy = true;
    s->group_id = next_group++;
    s->t_launch = now();
    lk.unlock();
    const bool ok = launch_group(s);
    // a partly enqueued group must drain before its share is reused
    if (!ok && !dry()) hipStreamSynchronize(s->stream);
    lk.lock();
    s->failed = !ok;
    s->launched = true;
    s->cv.notify_one();
  }
}

// Builds the group's records, segments and staging layout and enqueues its
// device work (no lock held; the group's sessions are busy, so nothing else
// touches their stores or descriptors).
bool dmpc_server::launch_group(Slot* s) {
  const int n = (int)s->reqs.size();
  // record order: by kernel instantiation, backward requests first within one
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto key = [&](int i) {
    const LaunchCfg& c = sessions[s->reqs[i].session].cfg;
    return std::make_tuple(c.nx, c.slots, c.maxbt, c.reg, c.bt);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (key(a) != key(b)) return key(a) < key(b);
    return s->reqs[a].backward > s->reqs[b].backward;
  });
  std::vector<Request> reqs(n);
  for (int k = 0; k < n; ++k) reqs[k] = std::move(s->reqs[order[k]]);
  s->reqs.swap(reqs);

  // input staging: [records | segments | payload]
  int n_in = 0;
  for (const Request& r : s->reqs) n_in += (r.has_x0 ? 1 : 0) + (r.has_dl ? 1 : 0);
  int n_bwd = 0;
  for (const Request& r : s->reqs) n_bwd += r.backward ? 1 : 0;
  const int n_out = n + n_bwd;
  const int64_t rec_off = 0, seg_off = a256((int64_t)n * sizeof(ProbRec));
  int64_t pay = seg_off + a256((int64_t)(n_in + n_out) * sizeof(Seg));
  // result staging: [status | info | sol blocks | grad blocks]
  s->status_off = 0;
  s->info_off = a256(4LL * n);
  int64_t oo = s->info_off + a256(16LL * n);
  s->out_sol.assign(n, 0);
  s->out_grad.assign(n, -1);

  std::vector<ProbRec> recs(n);
  std::vector<Seg> segs;
  segs.reserve(n_in + n_out);
  std::vector<std::pair<int64_t, const float*>> payload;   // (byte offset, source), sizes below
  std::vector<int64_t> payload_len;
  int64_t ws_off = 0;
  for (int k = 0; k < n; ++k) {
    const Request& r = s->reqs[k];
    const Session& ss = sessions[r.session];
    ProbRec& rec = recs[k];
    std::memset(&rec, 0, sizeof(rec));
    rec.T = ss.p.T;
    rec.nx = ss.p.nx;
    rec.nu = ss.p.nu;
    rec.dyn = ss.p.dyn;
    rec.cost = ss.p.cost;
    rec.phases = ss.p.cost_phases;
    rec.nw = ss.p.cost_nw;
    rec.index = k;
    rec.dyn_off = ss.p.dyn_off;
    rec.cost_off = ss.p.cost_off;
    rec.x0_off = ss.p.x0_off;
    rec.sol_off = ss.p.sol_off;
    rec.ws_off = ws_off;
    rec.slots = ss.cfg.slots;
    rec.flags = ss.flags;
    ws_off += ss.ws_floats;
    if (r.has_x0) {
      segs.push_back(Seg{(const uint32_t*)(s->d_in + pay), (uint32_t*)(d_data + ss.p.x0_off), ss.p.nx});
      payload.push_back({pay, r.x0});
      payload_len.push_back(ss.p.nx);
      pay += 4 * a4(ss.p.nx);
    }
    if (r.has_dl) {
      segs.push_back(Seg{(const uint32_t*)(s->d_in + pay), (uint32_t*)(d_dl + ss.p.sol_off), ss.sol_len});
      payload.push_back({pay, r.dl.data()});
      payload_len.push_back(ss.sol_len);
      pay += 4 * a4(ss.sol_len);
    }
  }
  for (int k = 0; k < n; ++k) {
    const Session& ss = sessions[s->reqs[k].session];
    s->out_sol[k] = oo;
    segs.push_back(Seg{(const uint32_t*)(d_sol + ss.p.sol_off), (uint32_t*)(s->d_out + oo), ss.sol_len});
    oo += 4 * a4(ss.sol_len);
  }
  for (int k = 0; k < n; ++k) {
    const Session& ss = sessions[s->reqs[k].session];
    if (!s->reqs[k].backward) continue;
    s->out_grad[k] = oo;
    const int64_t base = (int64_t)s->reqs[k].session * data_stride;
    segs.push_back(Seg{(const uint32_t*)(d_grad + base), (uint32_t*)(s->d_out + oo), ss.data_len});
    oo += 4 * a4(ss.data_len);
  }
  s->out_used = oo;
  if (pay > staging || oo > staging || (int64_t)ws_off * 4 > ws_share) return false;
  if (dry()) return true;

  // fill pinned input staging and enqueue
  std::memcpy(s->h_in + rec_off, recs.data(), sizeof(ProbRec) * n);
  std::memcpy(s->h_in + seg_off, segs.data(), sizeof(Seg) * segs.size());
  for (size_t i = 0; i < payload.size(); ++i)
    std::memcpy(s->h_in + payload[i].first, payload[i].second, 4 * payload_len[i]);
  hipStream_t st = s->stream;
  if (hipMemcpyAsync(s->d_in, s->h_in, pay, hipMemcpyHostToDevice, st) != hipSuccess) return false;
  const Seg* d_segs = (const Seg*)(s->d_in + seg_off);
  if (launch_seg_copy(d_segs, n_in, st) != 0) return false;

  KArgs a = make_kargs(cfg.opts, (const ProbRec*)(s->d_in + rec_off), d_data, d_sol, s->d_ws, d_dl,
                       d_adj, d_grad, (int32_t*)(s->d_out + s->status_off),
                       (int32_t*)(s->d_out + s->info_off));
  // instantiation ranges
  struct Range {
    LaunchCfg cfg;
    int first, count, nbwd;
  };
  std::vector<Range> ranges;   // s->reqs is in record order now
  for (int k = 0; k < n; ++k) {
    const Session& ss = sessions[s->reqs[k].session];
    if (k == 0 || key(k) != key(k - 1)) {
      Range g;
      g.cfg = ss.cfg;
      g.cfg.lds_bytes = 0;
      g.first = k;
      g.count = 0;
      g.nbwd = 0;
      ranges.push_back(g);
    }
    Range& g = ranges.back();
    g.count += 1;
    g.nbwd += s->reqs[k].backward ? 1 : 0;
    g.cfg.lds_bytes = std::max(g.cfg.lds_bytes,
                               (size_t)lds_floats(ss.p.T, ss.p.nx, ss.p.nu, g.cfg.bt, g.cfg.slots,
                                                  ss.flags, lin_floats_of(ss.p)) *
                                   sizeof(float));
  }
  for (const Range& g : ranges) {
    LaunchCfg c = g.cfg;
    c.grid = g.count;
    a.first = g.first;
    a.count = g.count;
    if (launch_forward(c, a, st) != 0) return false;
  }
  for (const Range& g : ranges) {
    if (g.nbwd == 0) continue;
    LaunchCfg c = g.cfg;
    c.grid = g.nbwd;
    a.first = g.first;
    a.count = g.nbwd;
    if (launch_backward(c, a, st) != 0) return false;
  }
  if (launch_seg_copy(d_segs + n_in, n_out, st) != 0) return false;
  if (hipMemcpyAsync(s->h_out, s->d_out, s->out_used, hipMemcpyDeviceToHost, st) != hipSuccess)
    return false;
  return hipEventRecord(s->done, st) == hipSuccess;
}

// ---------------------------------------------------------------------------
// completion
// ---------------------------------------------------------------------------
void dmpc_server::run_slot(Slot* s) {
  if (!dry()) hipSetDevice(cfg.device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      s->cv.wait(lk, [&] { return s->launched || (stop && !s->busy); });
      if (!s->launched) return;
    }
    bool ok = !s->failed;
    if (ok) {
      if (dry())
        std::this_thread::sleep_for(std::chrono::microseconds(cfg.dry_run_us));
      else
        ok = hipEventSynchronize(s->done) == hipSuccess;
    }
    s->failed = !ok;
    finish_group(s);
  }
}

void dmpc_server::finish_group(Slot* s) {
  const int n = (int)s->reqs.size();
  std::vector<Result> out(n);
  for (int k = 0; k < n; ++k) {
    const Request& r = s->reqs[k];
    const Session& ss = sessions[r.session];
    Result& res = out[k];
    res.t_submit = r.t_submit;
    if (s->failed) {
      res.state = DMPC_REQ_FAILED;
      continue;
    }
    res.state = DMPC_REQ_DONE;
    res.sol.assign(ss.sol_len, 0.f);
    if (r.backward) res.grad.assign(ss.data_len, 0.f);
    if (!dry()) {
      res.status = ((const int32_t*)(s->h_out + s->status_off))[k];
      std::memcpy(res.info, s->h_out + s->info_off + 16LL * k, 16);
      if (!r.backward) res.info[1] = 0;   // written by the backward kernel only
      std::memcpy(res.sol.data(), s->h_out + s->out_sol[k], 4 * ss.sol_len);
      if (r.backward) std::memcpy(res.grad.data(), s->h_out + s->out_grad[k], 4 * ss.data_len);
    }
  }
  std::lock_guard<std::mutex> lk(mu);
  const double t = now();
  GroupTrace tr;
  tr.id = s->group_id;
  tr.slot = s->id;
  tr.ws_bytes = s->ws_bytes;
  tr.t_launch = s->t_launch;
  tr.t_done = t;
  for (int k = 0; k < n; ++k) {
    const Request& r = s->reqs[k];
    Session& ss = sessions[r.session];
    ss.busy = false;
    ss.queued -= 1;
    tr.tickets.push_back(r.ticket);
    out[k].t_done = t;
    if (out[k].state == DMPC_REQ_DONE) {
      st_completed += 1;
      st_bwd += r.backward ? 1 : 0;
      latencies.push_back(t - r.t_submit);
      (ss.heavy ? lat_heavy : lat_light).push_back(t - r.t_submit);
      st_last_done = t;
    } else {
      st_failed += 1;
    }
    finished_total += 1;
    auto it = results.find(r.ticket);
    if (it != results.end()) it->second = std::move(out[k]);
  }
  if (!s->failed) {
    st_groups += 1;
    st_group_reqs += n;
    st_max_group = std::max<int64_t>(st_max_group, n);
  }
  trace.push_back(std::move(tr));
  if ((int)trace.size() > kTraceKeep) trace.pop_front();
  s->reqs.clear();
  s->launched = false;
  if (s->heavy) heavy_inflight -= 1;
  s->heavy = false;
  s->busy = false;
  cv_disp.notify_one();
  cv_res.notify_all();
}

// ---------------------------------------------------------------------------
// set-up and teardown
// ---------------------------------------------------------------------------
void dmpc_server::release() {
  for (auto& s : slots) {
    if (s->stream) hipStreamDestroy(s->stream);
    if (s->done) hipEventDestroy(s->done);
    if (s->d_ws) hipFree(s->d_ws);
    if (s->d_in) hipFree(s->d_in);
    if (s->d_out) hipFree(s->d_out);
    if (s->h_in) hipHostFree(s->h_in);
    if (s->h_out) hipHostFree(s->h_out);
  }
  slots.clear();
  float* bufs[] = {d_data, d_grad, d_sol, d_adj, d_dl};
  for (float* b : bufs)
    if (b) hipFree(b);
  d_data = d_grad = d_sol = d_adj = d_dl = nullptr;
}

extern "C" {

dmpc_status dmpc_server_create(const dmpc_server_config* cfg, dmpc_server** out) {
  if (!out) return DMPC_ERR_INVALID_ARG;
  *out = nullptr;
  dmpc_status st = check_config(cfg);
  if (st != DMPC_OK) return st;
  dmpc_server* sv = new (std::nothrow) dmpc_server;
  if (!sv) return DMPC_ERR_NOMEM;
  sv->cfg = *cfg;
  sv->t0 = Clock::now();
  sv->data_stride = align_up(max_data_len(cfg->max_T, cfg->max_nx, cfg->max_nu), kAlignFloats);
  sv->sol_stride = align_up(sol_block_len(cfg->max_T, cfg->max_nx, cfg->max_nu), kAlignFloats);
  sv->ws_share = cfg->hbm_budget / cfg->max_inflight / 256 * 256;
  sv->staging = cfg->staging_bytes > 0 ? cfg->staging_bytes : kDefaultStaging;
  // one request of the largest shape must fit a share and the staging
  const int64_t ws_max =
      4 * std::max(ws_layout(cfg->max_T, cfg->max_nx, cfg->max_nu, DMPC_DYN_LTV, kRecBulkWs).total,
                   ws_layout(cfg->max_T, cfg->max_nx, cfg->max_nu, DMPC_DYN_CARTPOLE, kRecBulkWs).total);
  const int64_t one_in = 1024 + (int64_t)sizeof(ProbRec) + 4 * sizeof(Seg) +
                         4 * (a4(cfg->max_nx) + sv->sol_stride);
  const int64_t one_out = 1024 + 20 + 4 * (sv->sol_stride + sv->data_stride);
  if (ws_max > sv->ws_share || one_in > sv->staging || one_out > sv->staging) {
    delete sv;
    return DMPC_ERR_NOMEM;
  }
  sv->max_heavy = std::max(1, cfg->max_inflight / 2);
  sv->sessions.resize(cfg->max_sessions);
  sv->slots.resize(cfg->max_inflight);
  for (int i = 0; i < cfg->max_inflight; ++i) {
    sv->slots[i].reset(new Slot);
    sv->slots[i]->id = i;
  }
  if (!sv->dry()) {
    int n = 0, prev = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || cfg->device < 0 || cfg->device >= n) {
      delete sv;
      return DMPC_ERR_INVALID_ARG;
    }
    hipGetDevice(&prev);
    if (hipSetDevice(cfg->device) != hipSuccess) {
      delete sv;
      return DMPC_ERR_HIP;
    }
    const size_t S = (size_t)cfg->max_sessions;
    bool ok = hipMalloc((void**)&sv->d_data, 4 * S * sv->data_stride) == hipSuccess &&
              hipMalloc((void**)&sv->d_grad, 4 * S * sv->data_stride) == hipSuccess &&
              hipMalloc((void**)&sv->d_sol, 4 * S * sv->sol_stride) == hipSuccess &&
              hipMalloc((void**)&sv->d_adj, 4 * S * sv->sol_stride) == hipSuccess &&
              hipMalloc((void**)&sv->d_dl, 4 * S * sv->sol_stride) == hipSuccess;
    for (auto& s : sv->slots) {
      if (!ok) break;
      ok = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&s->done, hipEventDisableTiming) == hipSuccess &&
           hipMalloc((void**)&s->d_ws, sv->ws_share) == hipSuccess &&
           hipMalloc((void**)&s->d_in, sv->staging) == hipSuccess &&
           hipMalloc((void**)&s->d_out, sv->staging) == hipSuccess &&
           hipHostMalloc((void**)&s->h_in, sv->staging, hipHostMallocDefault) == hipSuccess &&
           hipHostMalloc((void**)&s->h_out, sv->staging, hipHostMallocDefault) == hipSuccess;
    }
    if (ok) {
      ok = hipMemset(sv->d_data, 0, 4 * S * sv->data_stride) == hipSuccess &&
           hipMemset(sv->d_grad, 0, 4 * S * sv->data_stride) == hipSuccess &&
           hipMemset(sv->d_sol, 0, 4 * S * sv->sol_stride) == hipSuccess &&
           hipMemset(sv->d_adj, 0, 4 * S * sv->sol_stride) == hipSuccess &&
           hipMemset(sv->d_dl, 0, 4 * S * sv->sol_stride) == hipSuccess &&
           hipDeviceSynchronize() == hipSuccess;
    }
    hipSetDevice(prev);
    if (!ok) {
      sv->release();
      delete sv;
      return DMPC_ERR_NOMEM;
    }
  }
  for (auto& s : sv->slots) {
    Slot* p = s.get();
    p->th = std::thread([sv, p] { sv->run_slot(p); });
  }
  sv->dispatcher = std::thread([sv] { sv->run_dispatcher(); });
  *out = sv;
  return DMPC_OK;
}

dmpc_status dmpc_server_destroy(dmpc_server* sv) {
  if (!sv) return DMPC_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv_disp.notify_all();
  }
  sv->dispatcher.join();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (Request& r : sv->pending) {
      sv->results[r.ticket].state = DMPC_REQ_FAILED;
      sv->sessions[r.session].queued -= 1;
    }
    sv->pending.clear();
    for (auto& s : sv->slots) s->cv.notify_all();
    sv->cv_res.notify_all();
  }
  for (auto& s : sv->slots) s->th.join();
  if (!sv->dry()) {
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(sv->cfg.device);
    sv->release();
    hipSetDevice(prev);
  }
  delete sv;
  return DMPC_OK;
}

dmpc_status dmpc_server_add_session(dmpc_server* sv, int32_t session, const dmpc_problem* problem,
                                    const float* data, int64_t data_len, const float* sol0,
                                    const float* dl) {
  if (!sv || !problem || !data || session < 0 || session >= sv->cfg.max_sessions || data_len <= 0 ||
      data_len > sv->data_stride)
    return DMPC_ERR_INVALID_ARG;
  const dmpc_problem& p = *problem;
  if (p.T > sv->cfg.max_T || p.nx > sv->cfg.max_nx || p.nu > sv->cfg.max_nu)
    return DMPC_ERR_INVALID_ARG;
  const int64_t sol_len = sol_block_len(p.T, p.nx, p.nu);
  dmpc_problem q = p;
  q.sol_off = 0;
  dmpc_status st = check_problem(q, data_len, sol_len);
  if (st != DMPC_OK) return st;
  LaunchCfg c;
  if (!nx_supported(p.nx) || !choose_cfg(p, sv->cfg.opts.block_threads, &c)) return DMPC_ERR_UNSUPPORTED;
  // batches of sessions fill the chip: the QP-data copy gets a quarter of a CU's LDS
  const int flags = rec_flags(p.T, p.nx, p.nu, c.bt, c.slots, c.reg, lin_floats_of(p),
                              lin_budget(4 * kComputeUnits));
  if ((size_t)lds_floats(p.T, p.nx, p.nu, c.bt, c.slots, flags, lin_floats_of(p)) * sizeof(float) >
      (size_t)kLdsBytes)
    return DMPC_ERR_UNSUPPORTED;
  const int64_t ws = ws_layout(p.T, p.nx, p.nu, p.dyn, flags).total;
  if (4 * ws > sv->ws_share) return DMPC_ERR_NOMEM;
  std::lock_guard<std::mutex> lk(sv->mu);
  Session& ss = sv->sessions[session];
  if (ss.queued > 0) return DMPC_ERR_INVALID_ARG;
  const int64_t dbase = (int64_t)session * sv->data_stride, sbase = (int64_t)session * sv->sol_stride;
  if (!sv->dry()) {
    int prev = 0;
    hipGetDevice(&prev);
    if (hipSetDevice(sv->cfg.device) != hipSuccess) return DMPC_ERR_HIP;
    std::vector<float> zeros(sol_len, 0.f);
    bool ok = hipMemcpy(sv->d_data + dbase, data, 4 * data_len, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(sv->d_sol + sbase, sol0 ? sol0 : zeros.data(), 4 * sol_len,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(sv->d_dl + sbase, dl ? dl : zeros.data(), 4 * sol_len,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(sv->d_adj + sbase, zeros.data(), 4 * sol_len, hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemset(sv->d_grad + dbase, 0, 4 * sv->data_stride) == hipSuccess &&
              hipDeviceSynchronize() == hipSuccess;
    hipSetDevice(prev);
    if (!ok) return DMPC_ERR_HIP;
  }
  ss.used = true;
  ss.p = p;
  ss.p.dyn_off += dbase;
  ss.p.cost_off += dbase;
  ss.p.x0_off += dbase;
  ss.p.sol_off = sbase;
  ss.cfg = c;
  ss.flags = flags;
  ss.heavy = (flags & kRecBulkWs) != 0;
  ss.data_len = data_len;
  ss.sol_len = sol_len;
  ss.ws_floats = ws;
  return DMPC_OK;
}

dmpc_status dmpc_server_submit(dmpc_server* sv, int32_t session, int32_t backward, const float* x0,
                               const float* dl, int64_t* ticket) {
  if (!sv || !ticket || session < 0 || session >= sv->cfg.max_sessions ||
      (backward != 0 && backward != 1))
    return DMPC_ERR_INVALID_ARG;
  Request r;
  r.session = session;
  r.backward = backward;
  std::unique_lock<std::mutex> lk(sv->mu);
  Session& ss = sv->sessions[session];
  if (!ss.used) return DMPC_ERR_INVALID_ARG;
  if (sv->cfg.max_pending > 0 && (int64_t)sv->pending.size() >= sv->cfg.max_pending) {
    sv->st_rejected += 1;
    return DMPC_ERR_NOMEM;
  }
  if (x0) {
    r.has_x0 = true;
    std::memcpy(r.x0, x0, 4 * ss.p.nx);
  }
  if (dl) {
    r.has_dl = true;
    r.dl.assign(dl, dl + ss.sol_len);
  }
  r.ticket = sv->next_ticket++;
  r.t_submit = sv->now();
  if (sv->st_first_submit < 0) sv->st_first_submit = r.t_submit;
  Result res;
  res.t_submit = r.t_submit;
  sv->results.emplace(r.ticket, std::move(res));
  *ticket = r.ticket;
  ss.queued += 1;
  sv->pending.push_back(std::move(r));
  sv->accepted_total += 1;
  sv->st_submitted += 1;
  sv->st_max_pending = std::max<int64_t>(sv->st_max_pending, (int64_t)sv->pending.size());
  lk.unlock();
  sv->cv_disp.notify_one();
  return DMPC_OK;
}

dmpc_status dmpc_server_wait(dmpc_server* sv, int64_t ticket, double timeout_s, float* sol,
                             float* grad, int32_t* info, int32_t* state, int32_t* prob_status) {
  if (!sv) return DMPC_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->results.find(ticket) == sv->results.end()) return DMPC_ERR_INVALID_ARG;
  auto finished = [&] {
    auto f = sv->results.find(ticket);
    if (f == sv->results.end()) return true;   // taken by another waiter
    return f->second.state == DMPC_REQ_DONE || f->second.state == DMPC_REQ_FAILED;
  };
  if (timeout_s < 0)
    sv->cv_res.wait(lk, finished);
  else
    sv->cv_res.wait_for(lk, std::chrono::duration<double>(timeout_s), finished);
  auto it = sv->results.find(ticket);
  if (it == sv->results.end()) return DMPC_ERR_INVALID_ARG;
  const int s = it->second.state;
  if (state) *state = s;
  if (s != DMPC_REQ_DONE && s != DMPC_REQ_FAILED) {
    if (prob_status) *prob_status = 0;
    return DMPC_OK;
  }
  Result res = std::move(it->second);
  sv->results.erase(it);
  lk.unlock();
  if (prob_status) *prob_status = res.status;
  if (info) std::memcpy(info, res.info, sizeof(res.info));
  if (sol && !res.sol.empty()) std::memcpy(sol, res.sol.data(), 4 * res.sol.size());
  if (grad && !res.grad.empty()) std::memcpy(grad, res.grad.data(), 4 * res.grad.size());
  return DMPC_OK;
}

dmpc_status dmpc_server_drain(dmpc_server* sv, double timeout_s) {
  if (!sv) return DMPC_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto done = [&] { return sv->finished_total == sv->accepted_total; };
  if (timeout_s < 0) {
    sv->cv_res.wait(lk, done);
    return DMPC_OK;
  }
  return sv->cv_res.wait_for(lk, std::chrono::duration<double>(timeout_s), done)
             ? DMPC_OK
             : DMPC_ERR_INVALID_ARG;
}

dmpc_status dmpc_server_get_stats(dmpc_server* sv, dmpc_server_stats* out) {
  if (!sv || !out) return DMPC_ERR_INVALID_ARG;
  std::vector<double> lat, lat_l, lat_h;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = sv->st_submitted;
    out->rejected = sv->st_rejected;
    out->completed = sv->st_completed;
    out->backward_completed = sv->st_bwd;
    out->failed = sv->st_failed;
    out->groups = sv->st_groups;
    out->mean_group_size = sv->st_groups ? (double)sv->st_group_reqs / sv->st_groups : 0.0;
    out->max_group_size = sv->st_max_group;
    out->max_pending_seen = sv->st_max_pending;
    const double span = sv->st_last_done - sv->st_first_submit;
    out->throughput = (sv->st_completed > 0 && sv->st_first_submit >= 0 && span > 0)
                          ? sv->st_completed / span
                          : 0.0;
    lat = sv->latencies;
    lat_l = sv->lat_light;
    lat_h = sv->lat_heavy;
    out->heavy_completed = (int64_t)lat_h.size();
  }
  auto q = [](std::vector<double>& v, double f) {
    if (v.empty()) return 0.0;
    const size_t i = (size_t)std::min<double>(v.size() - 1, std::ceil(f * v.size()) - 1);
    return v[i];
  };
  std::sort(lat.begin(), lat.end());
  std::sort(lat_l.begin(), lat_l.end());
  std::sort(lat_h.begin(), lat_h.end());
  out->p50_latency_s = q(lat, 0.50);
  out->p99_latency_s = q(lat, 0.99);
  out->max_latency_s = lat.empty() ? 0.0 : lat.back();
  out->light_p50_latency_s = q(lat_l, 0.50);
  out->light_p99_latency_s = q(lat_l, 0.99);
  out->heavy_p50_latency_s = q(lat_h, 0.50);
  out->heavy_p99_latency_s = q(lat_h, 0.99);
  return DMPC_OK;
}

dmpc_status dmpc_server_reset_stats(dmpc_server* sv) {
  if (!sv) return DMPC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->st_submitted = sv->st_rejected = sv->st_completed = sv->st_bwd = sv->st_failed = 0;
  sv->st_groups = sv->st_group_reqs = sv->st_max_group = 0;
  sv->st_max_pending = (int64_t)sv->pending.size();
  sv->st_first_submit = -1;
  sv->st_last_done = 0;
  sv->latencies.clear();
  sv->lat_light.clear();
  sv->lat_heavy.clear();
  sv->trace.clear();
  return DMPC_OK;
}

dmpc_status dmpc_server_trace(dmpc_server* sv, char* buf, size_t len) {
  if (!sv || !buf || len == 0) return DMPC_ERR_INVALID_ARG;
  std::string s = "[";
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    bool first = true;
    for (const GroupTrace& g : sv->trace) {
      char tmp[160];
      std::snprintf(tmp, sizeof(tmp),
                    "%s{\"id\": %lld, \"slot\": %d, \"ws_bytes\": %lld, \"t_launch\": %.6f, "
                    "\"t_done\": %.6f, \"tickets\": [",
                    first ? "" : ", ", (long long)g.id, g.slot, (long long)g.ws_bytes, g.t_launch,
                    g.t_done);
      s += tmp;
      for (size_t i = 0; i < g.tickets.size(); ++i) {
        std::snprintf(tmp, sizeof(tmp), "%s%lld", i ? ", " : "", (long long)g.tickets[i]);
        s += tmp;
      }
      s += "]}";
      first = false;
    }
  }
  s += "]";
  std::snprintf(buf, len, "%s", s.c_str());
  return DMPC_OK;
}

}  // extern "C"
