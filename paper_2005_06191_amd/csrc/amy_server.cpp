// amy_server.cpp -- serving loop with continuous batching.
//
// One worker thread owns a HIP stream and one device arena (allocated once,
// at creation).  Each iteration it
//   1. admits queued requests, in arrival order, while a slot is free and the
//      arena has room for the request's footprint (workspace + FP64 V +
//      optional policy); the mode (stored rows or on the fly) is picked per
//      request by memory and a cost model;
//   2. starts the newly admitted requests (labels / terminal values; the
//      stored rows of Alg. 2 for stored requests);
//   3. advances EVERY active request by one Bellman step: small requests
//      share a single replay of a captured graph (table upload + one
//      batched step kernel reading the slot table from device memory);
//      a request that fills the chip by itself (>= SOLO_STATES states) or
//      whose family the batched kernel lacks gets its own sweep launch for
//      the step, using the single-system kernel chosen for it (the
//      compiled-shape sweep where one matches).  Requests that arrive while
//      others run join at the next step boundary and their work overlaps
//      on the device;
//   4. retires finished requests (result copied to host memory, arena space
//      and slot freed).
// A request's rows are computed by the same per-state code whatever it is
// batched with, so its result equals a lone solve with the sweep variant
// its info reports, bit for bit.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/amytiss.h"
#include "amy_batch.hpp"
#include "amy_host.hpp"
#include "amy_kernels.hpp"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

inline uint64_t al256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// First-fit allocator over [0, size) with coalescing.
struct Arena {
  std::map<uint64_t, uint64_t> free_;  // offset -> length
  uint64_t size = 0, used = 0, peak = 0;
  void init(uint64_t n) {
    size = n;
    free_.clear();
    free_[0] = n;
    used = peak = 0;
  }
  bool alloc(uint64_t n, uint64_t& off) {
    n = al256(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        off = it->first;
        const uint64_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        used += n;
        peak = std::max(peak, used);
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = al256(n);
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

enum { RQ_QUEUED = 0, RQ_ACTIVE = 1, RQ_DONE = 2, RQ_FAILED = 3, RQ_CANCELLED = 4 };

struct Request {
  uint64_t ticket = 0;
  amy_problem prob;
  Plan plan;
  int state = RQ_QUEUED;
  amy_status err = AMY_OK;
  std::string msg;
  double t_submit = 0, t_admit = 0, t_done = 0;
  uint64_t off = 0, bytes = 0, off_v = 0, off_pol = 0;
  int t = 0;  // local step (0 = the step k = T_d)
  bool want_policy = false;
  bool cancel = false;  // cancellation asked for while active (applied at the next step boundary)
  bool solo = false;  // own sweep launch per step instead of the batched one
  std::vector<double> V;
  std::vector<int16_t> pol;
  double max_tail = 0;
};

// Rough device cost of a request (seconds) in each mode, used to choose
// stored rows only where streaming them beats recomputing them.
const double R_ALU = 2.0e13;  // achieved algorithmic flop/s of the OTF sweep
const double R_HBM = 4.0e12;  // achieved byte/s of the stored sweep
// 1024 tiles of 64 states: enough work for one launch to fill the chip
const int64_t SOLO_STATES = 65536;
double cost_otf(const Plan& pl, int T) {
  double edges = 0;
  for (int i = 0; i < pl.dev.n; ++i) edges += pl.dev.L[i] + 1;
  return (double)T * pl.rows * (3.0 * pl.W + 20.0 * edges) / R_ALU;
}
double cost_stored(const Plan& pl, int T) {
  return cost_otf(pl, 1) + (double)T * pl.rows * (pl.W * (pl.f64 ? 8.0 : 4.0) + 4.0) / R_HBM;
}

}  // namespace

struct amy_server {
  amy_server_cfg cfg;
  hipStream_t stream = nullptr;
  char* arena_base = nullptr;
  Arena arena;
  int ncu = 0;
  // per precision (0 FP32, 1 FP64): device and pinned host slot tables
  BatchSys* d_sys[2] = {nullptr, nullptr};
  int32_t* d_meta[2] = {nullptr, nullptr};
  BatchSys* h_sys[2] = {nullptr, nullptr};
  int32_t* h_meta[2] = {nullptr, nullptr};
  std::map<int, hipGraphExec_t> graphs[2];  // family set * 2^20 + LDS tier -> captured step
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> reqs;
  std::vector<Request*> active;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  // statistics
  uint64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, steps = 0;
  int max_active = 0;
  double row_updates = 0, busy_s = 0;
  std::vector<double> lat_ms;

  amy_status step_graph(int prec, int fs, int tier, hipGraphExec_t* out);
  void run();
  void fail_active(const char* what, hipError_t e);
  void retire(Request* r);
  bool admit(Request* r);
};

static const int LDS_TIERS[] = {16 * 1024, 32 * 1024, 48 * 1024, 64 * 1024};

amy_status amy_server::step_graph(int prec, int fs, int tier, hipGraphExec_t* out) {
  const int key = (fs << 20) + tier;
  auto it = graphs[prec].find(key);
  if (it != graphs[prec].end()) {
    *out = it->second;
    return AMY_OK;
  }
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, amy_batch_step_kernel(prec == 1, fs), 64, tier);
  if (e != hipSuccess || occ < 1) return amy_hip_fail(e, "server step occupancy");
  const unsigned grid = (unsigned)(ncu * occ);
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  const int cap = cfg.max_slots;
  if ((e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return amy_hip_fail(e, "server capture");
  hipMemcpyAsync(d_sys[prec], h_sys[prec], sizeof(BatchSys) * cap, hipMemcpyHostToDevice, stream);
  hipMemcpyAsync(d_meta[prec], h_meta[prec], sizeof(int32_t) * (cap + 2), hipMemcpyHostToDevice, stream);
  amy_launch_batch_step(prec == 1, fs, grid, tier, d_sys[prec], d_meta[prec], stream);
  if ((e = hipStreamEndCapture(stream, &g)) != hipSuccess) return amy_hip_fail(e, "server capture end");
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return amy_hip_fail(e, "server graph instantiate");
  graphs[prec][key] = ex;
  *out = ex;
  return AMY_OK;
}

void amy_server::fail_active(const char* what, hipError_t e) {
  (void)hipStreamSynchronize(stream);  // nothing may still use the arena blocks
  std::lock_guard<std::mutex> g(mu);
  for (Request* r : active) {
    r->state = RQ_FAILED;
    r->err = AMY_E_DEVICE;
    r->msg = std::string(what) + ": " + hipGetErrorString(e);
    arena.release(r->off, r->bytes);
    ++failed;
  }
  active.clear();
  cv_done.notify_all();
}

// Footprint and placement of a queued request; false if it does not fit now.
bool amy_server::admit(Request* r) {
  uint64_t off;
  if (!arena.alloc(r->bytes, off)) return false;
  r->off = off;
  return true;
}

void amy_server::retire(Request* r) {
  const int64_t nx = r->plan.dev.n_x;
  r->V.resize(nx);
  hipMemcpy(r->V.data(), arena_base + r->off + r->off_v, nx * 8, hipMemcpyDeviceToHost);
  if (r->want_policy && r->prob.horizon > 0) {
    r->pol.resize((size_t)r->prob.horizon * nx);
    hipMemcpy(r->pol.data(), arena_base + r->off + r->off_pol, r->pol.size() * 2, hipMemcpyDeviceToHost);
  }
  unsigned long long bits = 0;
  hipMemcpy(&bits, arena_base + r->off + r->plan.off_tail, 8, hipMemcpyDeviceToHost);
  memcpy(&r->max_tail, &bits, 8);
  if (r->prob.horizon == 0) r->max_tail = 0;
}

void amy_server::run() {
  hipSetDevice(cfg.device);
  for (;;) {
    std::vector<Request*> started;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
      // cancelled requests leave at this step boundary: the previous
      // iteration ended with a stream synchronisation, so none of their
      // work is still in flight
      bool dropped = false;
      for (size_t i = 0; i < active.size();) {
        Request* r = active[i];
        if (!r->cancel) {
          ++i;
          continue;
        }
        r->state = RQ_CANCELLED;
        r->t_done = now_s();
        arena.release(r->off, r->bytes);
        active.erase(active.begin() + (ptrdiff_t)i);
        ++cancelled;
        dropped = true;
      }
      if (dropped) cv_done.notify_all();
      if (stop && active.empty()) break;
      if (queue.empty() && active.empty()) continue;
      // admission in arrival order while slots and arena space last
      while (!stop && !queue.empty() && (int)active.size() < cfg.max_slots) {
        Request* r = queue.front();
        if (r->bytes > arena.size) {
          r->state = RQ_FAILED;
          r->err = AMY_E_NOMEM;
          r->msg = "request footprint exceeds the server's HBM budget";
          ++failed;
          queue.pop_front();
          cv_done.notify_all();
          continue;
        }
        if (!admit(r)) break;
        queue.pop_front();
        r->state = RQ_ACTIVE;
        r->t_admit = now_s();
        r->t = 0;
        active.push_back(r);
        started.push_back(r);
      }
      max_active = std::max(max_active, (int)active.size());
    }
    const double t0 = now_s();
    // start the newly admitted requests
    for (Request* r : started) {
      const Plan& pl = r->plan;
      char* b = arena_base + r->off;
      double* vout = (double*)(b + r->off_v);
      hipError_t e = amy_launch_init(pl.dev, (uint8_t*)(b + pl.off_label), b + pl.off_v0, pl.f64,
                                     r->prob.horizon == 0 ? vout : nullptr,
                                     (unsigned long long*)(b + pl.off_tail), stream);
      if (e == hipSuccess) e = amy_enqueue_prepare(pl, stream, b, r->prob.horizon);
      // requests on the batched step get their FP64 tail from a pass of its own
      if (e == hipSuccess && !r->solo && pl.mode != AMY_MODE_STORED && r->prob.horizon > 0)
        e = amy_launch_tail(pl.dev, (const uint8_t*)(b + pl.off_label), (unsigned long long*)(b + pl.off_tail),
                            stream);
      if (e == hipSuccess && pl.mode == AMY_MODE_STORED && r->prob.horizon > 0)
        e = amy_launch_build(pl.dev, pl.f64, (const uint8_t*)(b + pl.off_label), b + pl.off_T,
                             (int32_t*)(b + pl.off_org), (unsigned long long*)(b + pl.off_tail), stream);
      if (e != hipSuccess) {
        fail_active("server start", e);
        started.clear();
        break;
      }
    }
    // one Bellman step for every active request, per precision
    std::vector<Request*> act;
    {
      std::lock_guard<std::mutex> g(mu);
      act = active;
    }
    bool ok = true;
    for (int prec = 0; prec < 2 && ok; ++prec) {
      int n = 0, lds = 0, fs = 0;
      int32_t* meta = h_meta[prec];
      meta[1] = 0;
      for (Request* r : act) {
        if (r->solo || (int)r->plan.f64 != prec || r->t >= r->prob.horizon) continue;
        const Plan& pl = r->plan;
        char* b = arena_base + r->off;
        BatchSys& B = h_sys[prec][n];
        memset(&B, 0, sizeof B);
        B.P = pl.dev;
        B.label = (uint8_t*)(b + pl.off_label);
        B.V0 = b + pl.off_v0;
        B.V1 = b + pl.off_v1;
        B.Vout = (double*)(b + r->off_v);
        B.pol = r->want_policy ? (int16_t*)(b + r->off_pol) : nullptr;
        B.tailmax = (unsigned long long*)(b + pl.off_tail);
        B.T = pl.mode == AMY_MODE_STORED ? (void*)(b + pl.off_T) : nullptr;
        B.org = pl.mode == AMY_MODE_STORED ? (int32_t*)(b + pl.off_org) : nullptr;
        B.horizon = r->prob.horizon;
        B.mode = pl.mode;
        B.want_tail = pl.mode == AMY_MODE_STORED ? 0 : 1;
        B.step_base = r->t;
        const int per_tile = 64 / std::max(1, (int)pl.dev.grp_g);
        B.tiles = (int32_t)((pl.dev.n_x + per_tile - 1) / per_tile);
        meta[n + 2] = meta[n + 1] + B.tiles;
        if (pl.mode != AMY_MODE_STORED) {
          // the batched step has no tail path: tables only
          lds = std::max(lds, pl.dev.grp_g > 1 ? pl.dev.lds_bytes_group : pl.dev.lds_bytes);
          fs = std::max(fs, amy_batch_family_set(pl.dev.kind, pl.dev.n));
        }
        ++n;
      }
      if (n == 0) continue;
      meta[0] = n;
      int tier = LDS_TIERS[3];
      for (int t : LDS_TIERS)
        if (lds <= t) {
          tier = t;
          break;
        }
      hipGraphExec_t ex;
      if (step_graph(prec, fs, tier, &ex) != AMY_OK) {
        fail_active("server step graph", hipErrorUnknown);
        ok = false;
        break;
      }
      // the replay reads the pinned tables; they are rewritten only after
      // the stream synchronisation at the end of this iteration
      hipError_t e = hipGraphLaunch(ex, stream);
      if (e != hipSuccess) {
        fail_active("server step launch", e);
        ok = false;
        break;
      }
    }
    for (Request* r : act) {
      if (!ok || !r->solo || r->t >= r->prob.horizon) continue;
      char* b = arena_base + r->off;
      hipError_t e = amy_enqueue_step(r->plan, stream, b, (double*)(b + r->off_v),
                                      r->want_policy ? (int16_t*)(b + r->off_pol) : nullptr, r->prob.horizon,
                                      r->prob.horizon - r->t, r->plan.mode != AMY_MODE_STORED);
      if (e != hipSuccess) {
        fail_active("server solo step", e);
        ok = false;
      }
    }
    if (!ok) continue;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      fail_active("server step", e);
      continue;
    }
    // retire finished requests
    std::vector<Request*> done;
    for (Request* r : act) {
      if (r->t < r->prob.horizon) ++r->t;
      if (r->t >= r->prob.horizon) done.push_back(r);
    }
    for (Request* r : done) retire(r);
    {
      std::lock_guard<std::mutex> g(mu);
      ++steps;
      busy_s += now_s() - t0;
      const double tnow = now_s();
      for (Request* r : done) {
        r->state = RQ_DONE;
        r->t_done = tnow;
        arena.release(r->off, r->bytes);
        active.erase(std::find(active.begin(), active.end(), r));
        ++completed;
        row_updates += (double)r->plan.rows * r->prob.horizon;
        lat_ms.push_back(1e3 * (r->t_done - r->t_submit));
      }
      if (!done.empty()) cv_done.notify_all();
    }
  }
}

extern "C" amy_status amy_server_create(const amy_server_cfg* cfg, amy_server** out) {
  if (!cfg || !out) return amy_fail(AMY_E_INVALID, "cfg or out is NULL");
  if (cfg->max_slots < 1 || cfg->max_slots > 4096) return amy_fail(AMY_E_INVALID, "max_slots not in [1,4096]");
  if (cfg->hbm_budget_bytes < (1u << 20)) return amy_fail(AMY_E_INVALID, "hbm_budget_bytes below 1 MiB");
  amy_server* s = new amy_server();
  s->cfg = *cfg;
  hipError_t e;
  if ((e = hipSetDevice(cfg->device)) != hipSuccess) {
    delete s;
    return amy_hip_fail(e, "server device");
  }
  hipDeviceGetAttribute(&s->ncu, hipDeviceAttributeMultiprocessorCount, cfg->device);
  const uint64_t tbl = al256(sizeof(BatchSys) * cfg->max_slots), mt = al256(4 * (cfg->max_slots + 2));
  bool okm = (e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) == hipSuccess &&
             (e = hipMalloc((void**)&s->arena_base, cfg->hbm_budget_bytes)) == hipSuccess;
  for (int p = 0; okm && p < 2; ++p) {
    okm = (e = hipMalloc((void**)&s->d_sys[p], tbl)) == hipSuccess &&
          (e = hipMalloc((void**)&s->d_meta[p], mt)) == hipSuccess &&
          (e = hipHostMalloc((void**)&s->h_sys[p], tbl, hipHostMallocDefault)) == hipSuccess &&
          (e = hipHostMalloc((void**)&s->h_meta[p], mt, hipHostMallocDefault)) == hipSuccess;
    if (okm) {
      memset(s->h_sys[p], 0, tbl);
      memset(s->h_meta[p], 0, mt);
    }
  }
  if (!okm) {
    amy_status st = amy_hip_fail(e, "server allocation");
    amy_server_destroy(s);
    return st;
  }
  s->arena.init(cfg->hbm_budget_bytes);
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return AMY_OK;
}

extern "C" amy_status amy_server_submit(amy_server* s, const amy_problem* p, int32_t want_policy, uint64_t* ticket) {
  if (!s || !p || !ticket) return amy_fail(AMY_E_INVALID, "NULL argument");
  amy_status st = amy_validate(p);
  if (st != AMY_OK) return st;
  if (p->dyn.kind == AMY_DYN_USER)
    return amy_fail(AMY_E_UNSUPPORTED, "the server takes the built-in dynamics families");
  Request* r = new Request();
  r->prob = *p;
  r->want_policy = want_policy != 0;
  // mode by memory and cost: stored rows only if they fit in half the
  // arena and streaming them is estimated cheaper than recomputing
  amy_problem q = *p;
  int mode = p->mode;
  if (mode == AMY_MODE_AUTO) {
    Plan ps, po;
    amy_problem qs = q, qo = q;
    qs.mode = AMY_MODE_STORED;
    qo.mode = AMY_MODE_OTF;
    const bool stored_ok = amy_resolve(&qs, s->cfg.hbm_budget_bytes / 2, &ps) == AMY_OK;
    st = amy_resolve(&qo, 0, &po);
    if (st != AMY_OK) {
      delete r;
      return st;
    }
    mode = (stored_ok && cost_stored(ps, p->horizon) < cost_otf(po, p->horizon)) ? AMY_MODE_STORED : AMY_MODE_OTF;
  }
  q.mode = mode;
  st = amy_resolve(&q, 0, &r->plan);
  if (st != AMY_OK && mode == AMY_MODE_STORED && p->mode == AMY_MODE_AUTO) {
    q.mode = AMY_MODE_OTF;
    st = amy_resolve(&q, 0, &r->plan);
  }
  if (st != AMY_OK) {
    delete r;
    return st;
  }
  // large requests, and families the batched kernel lacks, take their own
  // launch per step; the rest share the batched step, which runs the
  // run-time-window code (same bits as the compiled-shape sweep)
  // (so do requests with a disturbance or another noise model)
  const DevProblem& Dp = r->plan.dev;
  const bool plain = Dp.pd == 0 && Dp.noise == 0 && Dp.wrule == 0 && !Dp.mult;
  r->solo = Dp.n_x >= SOLO_STATES || !plain || !amy_batch_supports(Dp.kind, Dp.n, r->plan.mode);
  if (!r->solo) {
    q.mode = r->plan.mode;
    st = amy_batch_normalise(&q, &r->plan);
    if (st != AMY_OK) {
      delete r;
      return st;
    }
  }
  r->off_v = al256(r->plan.ws_bytes);
  r->off_pol = al256(r->off_v + (uint64_t)r->plan.dev.n_x * 8);
  r->bytes = r->off_pol + (r->want_policy ? al256((uint64_t)p->horizon * r->plan.dev.n_x * 2) : 0);
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) {
      delete r;
      return amy_fail(AMY_E_INVALID, "server is shutting down");
    }
    r->ticket = s->next_ticket++;
    r->t_submit = now_s();
    s->reqs[r->ticket] = r;
    s->queue.push_back(r);
    ++s->submitted;
  }
  s->cv.notify_one();
  *ticket = r->ticket;
  return AMY_OK;
}

static void fill_req_info(const Request* r, amy_info* info) {
  memset(info, 0, sizeof *info);
  const Plan& pl = r->plan;
  info->mode_used = pl.mode;
  info->kernel = pl.dev.variant;
  for (int i = 0; i < pl.dev.n; ++i) info->window[i] = pl.dev.L[i];
  info->n_x = pl.dev.n_x;
  info->n_u = pl.dev.n_u;
  info->rows = pl.rows;
  info->W = pl.W;
  info->workspace_bytes = r->bytes;
  info->stored_bytes = pl.stored_bytes;
  info->max_row_tail = r->max_tail;
  info->tail_bound_E = r->max_tail * r->prob.horizon;
  info->t_build_ms = 1e3 * (r->t_admit - r->t_submit);  // time in the queue
  info->t_sweeps_ms = 1e3 * (r->t_done - r->t_admit);   // time on the device
  info->t_total_ms = 1e3 * (r->t_done - r->t_submit);   // request latency
}

extern "C" amy_status amy_server_wait(amy_server* s, uint64_t ticket, int32_t timeout_ms, double* V_host,
                                      int16_t* policy_host, amy_info* info) {
  if (!s) return amy_fail(AMY_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return amy_fail(AMY_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  auto ready = [&] { return r->state == RQ_DONE || r->state == RQ_FAILED || r->state == RQ_CANCELLED; };
  if (timeout_ms > 0) s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
  else if (timeout_ms < 0) s->cv_done.wait(lk, ready);
  if (!ready()) return amy_fail(AMY_E_NOTREADY, "request %llu not finished", (unsigned long long)ticket);
  s->reqs.erase(it);
  lk.unlock();
  amy_status st = AMY_OK;
  if (r->state == RQ_FAILED) {
    st = amy_fail(r->err, "%s", r->msg.c_str());
  } else if (r->state == RQ_CANCELLED) {
    st = amy_fail(AMY_E_CANCELLED, "request %llu was cancelled", (unsigned long long)ticket);
  } else {
    if (V_host) memcpy(V_host, r->V.data(), r->V.size() * 8);
    if (policy_host && !r->pol.empty()) memcpy(policy_host, r->pol.data(), r->pol.size() * 2);
    if (info) fill_req_info(r, info);
  }
  delete r;
  return st;
}

extern "C" amy_status amy_server_poll(amy_server* s, uint64_t ticket, double* V_host, int16_t* policy_host,
                                      amy_info* info) {
  return amy_server_wait(s, ticket, 0, V_host, policy_host, info);
}

extern "C" amy_status amy_server_cancel(amy_server* s, uint64_t ticket) {
  if (!s) return amy_fail(AMY_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return amy_fail(AMY_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  if (r->state == RQ_QUEUED) {
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
    r->state = RQ_CANCELLED;
    r->t_done = now_s();
    ++s->cancelled;
    s->cv_done.notify_all();
    return AMY_OK;
  }
  if (r->state == RQ_ACTIVE) {
    r->cancel = true;  // the worker drops it at the next step boundary
    s->cv.notify_one();
    return AMY_OK;
  }
  return amy_fail(AMY_E_INVALID, "request %llu has already finished", (unsigned long long)ticket);
}

extern "C" amy_status amy_server_get_stats(amy_server* s, amy_server_stats* out) {
  if (!s || !out) return amy_fail(AMY_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->cancelled = s->cancelled;
  out->queued = (int32_t)s->queue.size();
  out->active = (int32_t)s->active.size();
  out->max_active = s->max_active;
  out->hbm_in_use = s->arena.used;
  out->hbm_peak = s->arena.peak;
  out->steps = s->steps;
  out->row_updates = s->row_updates;
  out->busy_s = s->busy_s;
  if (!s->lat_ms.empty()) {
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      const double k = (v.size() - 1) * q;
      const size_t f = (size_t)k, c = std::min(v.size() - 1, f + 1);
      return v[f] + (v[c] - v[f]) * (k - f);
    };
    out->p50_ms = pct(0.5);
    out->p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_ms = sum / v.size();
  }
  return AMY_OK;
}

extern "C" amy_status amy_server_reset_stats(amy_server* s) {
  if (!s) return amy_fail(AMY_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  s->completed = s->failed = s->cancelled = s->steps = 0;
  s->submitted = s->reqs.size();
  s->row_updates = s->busy_s = 0;
  s->max_active = (int)s->active.size();
  s->lat_ms.clear();
  s->arena.peak = s->arena.used;
  return AMY_OK;
}

extern "C" amy_status amy_server_destroy(amy_server* s) {
  if (!s) return AMY_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    // queued requests are dropped; active ones finish their steps
    for (Request* r : s->queue) {
      r->state = RQ_FAILED;
      r->err = AMY_E_INVALID;
      r->msg = "server destroyed";
    }
    s->queue.clear();
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->reqs) delete kv.second;
  for (int p = 0; p < 2; ++p) {
    for (auto& kv : s->graphs[p]) hipGraphExecDestroy(kv.second);
    if (s->d_sys[p]) hipFree(s->d_sys[p]);
    if (s->d_meta[p]) hipFree(s->d_meta[p]);
    if (s->h_sys[p]) hipHostFree(s->h_sys[p]);
    if (s->h_meta[p]) hipHostFree(s->h_meta[p]);
  }
  if (s->arena_base) hipFree(s->arena_base);
  if (s->stream) hipStreamDestroy(s->stream);
  delete s;
  return AMY_OK;
}
