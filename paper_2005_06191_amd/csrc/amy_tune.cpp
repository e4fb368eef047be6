// amy_tune.cpp -- autotuner: measures the candidate launch configurations of
// a problem (or a batch) on the device and caches the fastest per shape class.
//
// Single solve: the sweep variant (run-time window LANES vs compiled-shape
// FIXED, where one is compiled).  Batch: tiles per work-queue grab, resident
// workgroups per CU, and the XCD-partitioned queue order.  The cache is an
// in-process map keyed by a shape-class string, saved and loaded as JSON.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/amytiss.h"
#include "amy_host.hpp"
#include "amy_kernels.hpp"
#include "amy_tune.hpp"

namespace {
struct Entry {
  int chunk = 1, blocks_per_cu = 0, xcd_order = 1, variant = 0;
  double ms = 0.0;
};
std::mutex g_mu;
std::map<std::string, Entry> g_cache;

int bucket(double v) { return v > 0 ? (int)lround(log2(v)) : 0; }

std::string key_solve(const Plan& pl, const amy_problem* p) {
  char b[256];
  int o = snprintf(b, sizeof b, "solve:k%d:n%d:%s:%s:L", pl.dev.kind, pl.dev.n, pl.f64 ? "f64" : "f32",
                   pl.mode == AMY_MODE_STORED ? "stored" : "otf");
  for (int i = 0; i < pl.dev.n && o < (int)sizeof b - 8; ++i) o += snprintf(b + o, sizeof b - o, "%d,", pl.dev.L[i]);
  snprintf(b + o, sizeof b - o, ":nu%d:nx%d:s%d", bucket(pl.dev.n_u), bucket(pl.dev.n_x), p->spec);
  return b;
}

std::string key_batch(const amy_problem* probs, int count, const BatchPlan& bp) {
  std::vector<int> fam;
  double rows = 0, wmax = 0;
  for (int i = 0; i < count; ++i) {
    fam.push_back(bp.plans[i].dev.kind * 16 + bp.plans[i].dev.n);
    rows += (double)bp.plans[i].rows * probs[i].horizon;
    wmax = std::max(wmax, (double)bp.plans[i].W);
  }
  std::sort(fam.begin(), fam.end());
  fam.erase(std::unique(fam.begin(), fam.end()), fam.end());
  std::string k = std::string("batch:") + (bp.f64 ? "f64" : "f32") + ":fam";
  for (int f : fam) k += std::to_string(f) + ",";
  k += ":n" + std::to_string(bucket(count)) + ":rows" + std::to_string(bucket(rows)) + ":W" +
       std::to_string(bucket(wmax)) + ":T" + std::to_string(bp.maxT);
  return k;
}

bool lookup(const std::string& k, Entry& e) {
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_cache.find(k);
  if (it == g_cache.end()) return false;
  e = it->second;
  return true;
}

void store(const std::string& k, const Entry& e) {
  std::lock_guard<std::mutex> g(g_mu);
  g_cache[k] = e;
}
}  // namespace

BatchTune amy_tune_lookup_batch(const amy_problem* probs, int32_t count, const BatchPlan& bp) {
  BatchTune t;
  Entry e;
  if (lookup(key_batch(probs, count, bp), e)) {
    t.chunk = e.chunk;
    t.blocks_per_cu = e.blocks_per_cu;
    t.xcd_order = e.xcd_order;
  }
  return t;
}

int amy_tune_lookup_variant(const Plan& pl, const amy_problem* p) {
  Entry e;
  if (lookup(key_solve(pl, p), e)) return e.variant;
  return AMY_VARIANT_AUTO;
}

static void fill_result(amy_tune_result* r, const Entry& best, int n, double worst) {
  if (!r) return;
  memset(r, 0, sizeof *r);
  r->chunk = best.chunk;
  r->blocks_per_cu = best.blocks_per_cu;
  r->xcd_order = best.xcd_order;
  r->variant = best.variant;
  r->best_ms = best.ms;
  r->worst_ms = worst;
  r->candidates = n;
}

extern "C" amy_status amy_tune_solve(const amy_problem* p, void* stream, void* workspace, uint64_t ws_bytes,
                                     double* V_out, amy_tune_result* out) {
  amy_status st = amy_validate(p);
  if (st != AMY_OK) return st;
  std::vector<int> variants;
  for (int v : {AMY_VARIANT_LANES, AMY_VARIANT_FIXED, AMY_VARIANT_GROUP16, AMY_VARIANT_GROUP64,
                AMY_VARIANT_FACTORED, AMY_VARIANT_INPUTS}) {
    amy_problem q = *p;
    q.variant = v;
    Plan pl;
    if (amy_resolve(&q, ws_bytes, &pl) == AMY_OK) variants.push_back(v);
  }
  if (variants.empty()) return amy_fail(AMY_E_UNSUPPORTED, "no sweep variant fits this problem");
  hipStream_t hs = (hipStream_t)stream;
  Entry best;
  best.ms = 1e300;
  double worst = 0.0;
  std::string key;
  for (int v : variants) {
    amy_problem q = *p;
    q.variant = v;
    Plan pl;
    st = amy_resolve(&q, ws_bytes, &pl);
    if (st != AMY_OK) return st;
    if (ws_bytes < pl.ws_bytes) return amy_fail(AMY_E_NOMEM, "workspace too small for tuning");
    key = key_solve(pl, p);
    Timing tm;
    for (int i = 0; i < Timing::N; ++i) hipEventCreate(&tm.ev[i]);
    double ms = 1e300;
    for (int rep = 0; rep < 3; ++rep) {  // first run warms caches and code
      st = amy_enqueue(pl, hs, workspace, V_out, nullptr, p->horizon, false, &tm);
      if (st != AMY_OK) break;
      hipEventSynchronize(tm.ev[4]);
      float t = 0.f;
      hipEventElapsedTime(&t, tm.ev[0], tm.ev[4]);
      if (rep > 0) ms = std::min(ms, (double)t);
    }
    for (int i = 0; i < Timing::N; ++i) hipEventDestroy(tm.ev[i]);
    if (st != AMY_OK) return st;
    worst = std::max(worst, ms);
    if (ms < best.ms) {
      best.ms = ms;
      best.variant = v;
    }
  }
  store(key, best);
  fill_result(out, best, (int)variants.size(), worst);
  return AMY_OK;
}

extern "C" amy_status amy_tune_batch(const amy_problem* probs, int32_t count, void* stream, void* workspace,
                                     uint64_t ws_bytes, double* const* V_out, amy_tune_result* out) {
  BatchPlan bp;
  amy_status st = amy_batch_plan(probs, count, bp);
  if (st != AMY_OK) return st;
  if (!workspace || ws_bytes < bp.ws_bytes) return amy_fail(AMY_E_NOMEM, "batch workspace too small");
  hipStream_t hs = (hipStream_t)stream;
  std::vector<BatchTune> cands;
  for (int chunk : {1, 2, 4, 8})
    for (int xcd : {0, 1})
      for (int bpc : {0, 4, 2}) {
        BatchTune t;
        t.chunk = chunk;
        t.xcd_order = xcd;
        t.blocks_per_cu = bpc;
        cands.push_back(t);
      }
  Entry best;
  best.ms = 1e300;
  double worst = 0.0;
  int valid = 0;
  for (const BatchTune& t : cands) {
    double ms = 1e300;
    bool gave_up = false;
    for (int rep = 0; rep < 2; ++rep) {
      float m = 0.f;
      st = amy_batch_run(probs, bp, hs, (char*)workspace, V_out, nullptr, false, t, &m);
      if (st != AMY_OK) return st;
      // a candidate whose grid-barrier wait gave up produced no valid result
      unsigned ctl[4] = {0u, 0u, 0u, 0u};
      const hipError_t e = hipMemcpy(ctl, (char*)workspace + bp.off_ctl, sizeof ctl, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return amy_hip_fail(e, "batch control readback");
      if (ctl[2] != 0u) gave_up = true;
      if (rep > 0) ms = std::min(ms, (double)m);
    }
    if (gave_up) continue;
    ++valid;
    worst = std::max(worst, ms);
    if (ms < best.ms) {
      best.ms = ms;
      best.chunk = t.chunk;
      best.xcd_order = t.xcd_order;
      best.blocks_per_cu = t.blocks_per_cu;
    }
  }
  if (valid == 0) return amy_fail(AMY_E_DEVICE, "batch tuning: every candidate's grid barrier gave up");
  store(key_batch(probs, count, bp), best);
  fill_result(out, best, valid, worst);
  return AMY_OK;
}

extern "C" amy_status amy_tune_clear(void) {
  std::lock_guard<std::mutex> g(g_mu);
  g_cache.clear();
  return AMY_OK;
}

extern "C" int32_t amy_tune_entries(void) {
  std::lock_guard<std::mutex> g(g_mu);
  return (int32_t)g_cache.size();
}

// JSON: {"<key>": {"chunk": c, "blocks_per_cu": b, "xcd_order": x, "variant": v, "ms": t}, ...}
extern "C" amy_status amy_tune_save(const char* path) {
  if (!path) return amy_fail(AMY_E_INVALID, "path is NULL");
  FILE* f = fopen(path, "w");
  if (!f) return amy_fail(AMY_E_INVALID, "cannot write %s", path);
  std::lock_guard<std::mutex> g(g_mu);
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : g_cache) {
    const Entry& e = kv.second;
    fprintf(f, "  \"%s\": {\"chunk\": %d, \"blocks_per_cu\": %d, \"xcd_order\": %d, \"variant\": %d, \"ms\": %.6f}%s\n",
            kv.first.c_str(), e.chunk, e.blocks_per_cu, e.xcd_order, e.variant, e.ms,
            ++i < g_cache.size() ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
  return AMY_OK;
}

extern "C" amy_status amy_tune_load(const char* path) {
  if (!path) return amy_fail(AMY_E_INVALID, "path is NULL");
  FILE* f = fopen(path, "r");
  if (!f) return amy_fail(AMY_E_INVALID, "cannot read %s", path);
  std::string txt;
  char buf[4096];
  size_t r;
  while ((r = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, r);
  fclose(f);
  std::map<std::string, Entry> loaded;
  size_t pos = 0;
  for (;;) {
    const size_t k0 = txt.find('"', pos);
    if (k0 == std::string::npos) break;
    const size_t k1 = txt.find('"', k0 + 1);
    const size_t b0 = txt.find('{', k1);
    const size_t b1 = txt.find('}', b0);
    if (k1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos)
      return amy_fail(AMY_E_INVALID, "%s: malformed tuning cache", path);
    const std::string key = txt.substr(k0 + 1, k1 - k0 - 1);
    const std::string body = txt.substr(b0, b1 - b0 + 1);
    Entry e;
    if (sscanf(body.c_str(), "{\"chunk\": %d, \"blocks_per_cu\": %d, \"xcd_order\": %d, \"variant\": %d, \"ms\": %lf}",
               &e.chunk, &e.blocks_per_cu, &e.xcd_order, &e.variant, &e.ms) != 5)
      return amy_fail(AMY_E_INVALID, "%s: malformed entry for %s", path, key.c_str());
    if (e.chunk < 1 || e.chunk > 64 || e.blocks_per_cu < 0 || e.variant < 0 || e.variant > AMY_VARIANT_INPUTS)
      return amy_fail(AMY_E_INVALID, "%s: out-of-range entry for %s", path, key.c_str());
    loaded[key] = e;
    pos = b1 + 1;
  }
  std::lock_guard<std::mutex> g(g_mu);
  for (auto& kv : loaded) g_cache[kv.first] = kv.second;
  return AMY_OK;
}
