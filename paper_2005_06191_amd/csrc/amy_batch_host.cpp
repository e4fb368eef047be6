// amy_batch_host.cpp -- C ABI of the batched solve: many systems, one
// cooperative persistent launch.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/amytiss.h"
#include "amy_batch.hpp"
#include "amy_host.hpp"
#include "amy_kernels.hpp"
#include "amy_tune.hpp"

static inline uint64_t al256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Workgroups with `lds` bytes of LDS that one CU holds at once: gfx950
// allocates a workgroup's LDS in granules of 1280 bytes (320 dwords) out of
// the CU's 160 KiB, as a residency probe on MI355X confirms for every size
// from 1 KiB to 40 KiB in 256-byte steps (the occupancy query, which
// divides by the byte count, is above the resident count for 35 of them).
int amy_lds_blocks_per_cu(int dev, size_t lds) {
  const size_t granule = 1280;
  int per_cu = 0;
  if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      per_cu <= 0)
    per_cu = 160 * 1024;
  if (lds == 0) return 1 << 20;
  const size_t alloc = (lds + granule - 1) / granule * granule;
  return (int)((size_t)per_cu / alloc);
}

// A system in a batched launch runs one of the two run-time-window variants
// compiled into the batched kernel, LANES or GROUP64: every variant computes
// the same bits, and leaving the others out keeps the batched kernel's
// register budget (and so its occupancy) at that of those two.  The
// compiled-shape variants become LANES, GROUP16 becomes GROUP64, and stored
// rows are walked 64 states per tile whatever the variant.
static const int BATCH_LANES_LDS = 8 * 1024;  // bytes of per-lane tables a batched LANES system may take

amy_status amy_batch_normalise(const amy_problem* p, Plan* pl, int lanes_lds_cap) {
  DevProblem& D = pl->dev;
  if (pl->mode == AMY_MODE_STORED) {
    D.grp_g = 1;
    return AMY_OK;
  }
  if (D.variant == AMY_VARIANT_FIXED || D.variant == AMY_VARIANT_FACTORED) {
    D.variant = AMY_VARIANT_LANES;
    D.rel_entries = 0;
  }
  if (D.variant == AMY_VARIANT_INPUTS) {
    amy_problem q = *p;
    q.mode = AMY_MODE_OTF;
    q.variant = AMY_VARIANT_LANES;
    const amy_status st = amy_resolve(&q, 0, pl);
    if (st != AMY_OK) return st;
  }
  if (D.variant == AMY_VARIANT_GROUP16) {
    amy_problem q = *p;
    q.mode = AMY_MODE_OTF;
    q.variant = AMY_VARIANT_GROUP64;
    const amy_status st = amy_resolve(&q, 0, pl);
    if (st != AMY_OK) return st;
  }
  // The persistent launch reserves its largest system's LDS for every
  // workgroup: there a LANES system with large per-lane tables would cut
  // the residency of all of them, so it runs one wave per row instead (its
  // state's tables take a few hundred bytes there)
  if (lanes_lds_cap > 0 && D.variant == AMY_VARIANT_LANES && D.lds_bytes > lanes_lds_cap) {
    amy_problem q = *p;
    q.mode = AMY_MODE_OTF;
    q.variant = AMY_VARIANT_GROUP64;
    Plan g;
    if (amy_resolve(&q, 0, &g) == AMY_OK) *pl = g;
  }
  if (D.grp_g != 1 && D.grp_g != 64)
    return amy_fail(AMY_E_UNSUPPORTED, "batched launch: %d lanes per state", (int)D.grp_g);
  return AMY_OK;
}

amy_status amy_batch_plan(const amy_problem* probs, int32_t count, BatchPlan& bp) {
  if (!probs || count < 1 || count > AMY_BATCH_MAX)
    return amy_fail(AMY_E_INVALID, "batch of %d systems (1..%d)", count, AMY_BATCH_MAX);
  bp.plans.assign(count, Plan());
  bp.lds = 0;
  bp.maxT = 0;
  bp.fs = 0;
  for (int i = 0; i < count; ++i) {
    amy_status st = amy_validate(&probs[i]);
    if (st != AMY_OK) return amy_fail(st, "system %d: %s", i, amy_last_error());
    amy_problem q = probs[i];
    if (q.mode == AMY_MODE_STORED)
      return amy_fail(AMY_E_UNSUPPORTED, "system %d: the batched launch recomputes rows (OTF mode only)", i);
    q.mode = AMY_MODE_OTF;
    if (q.variant == AMY_VARIANT_FIXED || q.variant == AMY_VARIANT_FACTORED || q.variant == AMY_VARIANT_INPUTS)
      q.variant = AMY_VARIANT_LANES;
    st = amy_resolve(&q, 0, &bp.plans[i]);
    if (st == AMY_OK) st = amy_batch_normalise(&q, &bp.plans[i], BATCH_LANES_LDS);
    if (st != AMY_OK) return amy_fail(st, "system %d: %s", i, amy_last_error());
    const DevProblem& D = bp.plans[i].dev;
    if (D.pd != 0 || D.noise != 0 || D.wrule != 0 || D.mult)
      return amy_fail(AMY_E_UNSUPPORTED, "system %d: the batched launch takes additive normal noise with the "
                      "centre rule and no disturbance", i);
    if (!amy_batch_supports(D.kind, D.n, AMY_MODE_OTF))
      return amy_fail(AMY_E_UNSUPPORTED, "system %d: dynamics kind %d with n=%d is not compiled into the batched kernel",
                      i, D.kind, D.n);
    if (i == 0) bp.f64 = bp.plans[i].f64;
    else if (bp.plans[i].f64 != bp.f64)
      return amy_fail(AMY_E_UNSUPPORTED, "system %d: a batch runs in one precision", i);
    if (probs[i].horizon > AMY_BATCH_MAX_STEPS)
      return amy_fail(AMY_E_UNSUPPORTED, "system %d: horizon %d > %d", i, probs[i].horizon, AMY_BATCH_MAX_STEPS);
    bp.maxT = std::max(bp.maxT, (int)probs[i].horizon);
    bp.fs = std::max(bp.fs, amy_batch_family_set(D.kind, D.n));
    // the steps' LDS (the FP64 tail has a pass of its own)
    bp.lds = std::max(bp.lds, (size_t)(D.grp_g > 1 ? D.lds_bytes_group : D.lds_bytes));
  }
  // longest horizon first: the systems still running at global step s are a prefix
  bp.order.resize(count);
  for (int i = 0; i < count; ++i) bp.order[i] = i;
  std::stable_sort(bp.order.begin(), bp.order.end(),
                   [&](int a, int b) { return probs[a].horizon > probs[b].horizon; });
  bp.tprefix.assign(count + 1, 0);
  bp.tp64.assign(count + 1, 0);
  for (int r = 0; r < count; ++r) {
    const DevProblem& D = bp.plans[bp.order[r]].dev;
    const int per_tile = 64 / std::max(1, (int)D.grp_g);  // states per 64-lane tile
    bp.tprefix[r + 1] = bp.tprefix[r] + (int32_t)((D.n_x + per_tile - 1) / per_tile);
    bp.tp64[r + 1] = bp.tp64[r] + (int32_t)((D.n_x + 63) / 64);
  }
  bp.active.assign(std::max(bp.maxT, 1), 0);
  for (int s = 0; s < bp.maxT; ++s) {
    int a = 0;
    while (a < count && probs[bp.order[a]].horizon > s) ++a;
    bp.active[s] = a;
  }
  uint64_t o = 0;
  bp.off_sys = o;  o = al256(o + (uint64_t)count * sizeof(BatchSys));
  bp.off_tp = o;   o = al256(o + (uint64_t)(count + 1) * 4);
  bp.off_tp64 = o; o = al256(o + (uint64_t)(count + 1) * 4);
  bp.off_act = o;  o = al256(o + (uint64_t)bp.active.size() * 4);
  bp.off_ctl = o;  o = al256(o + sizeof(BatchCtl));
  bp.base.assign(count, 0);
  for (int i = 0; i < count; ++i) {
    bp.base[i] = o;
    o = al256(o + bp.plans[i].ws_bytes);
  }
  bp.ws_bytes = o;
  return AMY_OK;
}

void amy_batch_fill(const amy_problem* probs, const BatchPlan& bp, char* ws, double* const* V_out,
                    int16_t* const* policy_out, bool want_tail, std::vector<BatchSys>& sys) {
  const int count = (int)bp.plans.size();
  sys.assign(count, BatchSys());
  for (int r = 0; r < count; ++r) {
    const int i = bp.order[r];
    const Plan& pl = bp.plans[i];
    BatchSys& B = sys[r];
    memset(&B, 0, sizeof B);
    B.P = pl.dev;
    char* b = ws + bp.base[i];
    B.label = (uint8_t*)(b + pl.off_label);
    B.V0 = b + pl.off_v0;
    B.V1 = b + pl.off_v1;
    B.tailmax = (unsigned long long*)(b + pl.off_tail);
    B.Vout = V_out[i];
    B.pol = policy_out ? policy_out[i] : nullptr;
    B.horizon = probs[i].horizon;
    B.tiles = (int32_t)((pl.dev.n_x + 64 / pl.dev.grp_g - 1) / (64 / pl.dev.grp_g));
    B.mode = AMY_MODE_OTF;
    B.want_tail = want_tail ? 1 : 0;
  }
}

extern "C" amy_status amy_batch_query(const amy_problem* probs, int32_t count, uint64_t* ws_bytes) {
  BatchPlan bp;
  amy_status st = amy_batch_plan(probs, count, bp);
  if (st != AMY_OK) return st;
  if (ws_bytes) *ws_bytes = bp.ws_bytes;
  return AMY_OK;
}

amy_status amy_batch_run(const amy_problem* probs, const BatchPlan& bp, hipStream_t hs, char* ws,
                         double* const* V_out, int16_t* const* policy_out, bool want_tail, const BatchTune& tune,
                         float* ms_out) {
  const int count = (int)bp.plans.size();
  std::vector<BatchSys> sys;
  amy_batch_fill(probs, bp, ws, V_out, policy_out, want_tail, sys);
  hipError_t e;
  if ((e = hipMemcpyAsync(ws + bp.off_sys, sys.data(), sizeof(BatchSys) * count, hipMemcpyHostToDevice, hs)) ||
      (e = hipMemcpyAsync(ws + bp.off_tp, bp.tprefix.data(), 4 * bp.tprefix.size(), hipMemcpyHostToDevice, hs)) ||
      (e = hipMemcpyAsync(ws + bp.off_tp64, bp.tp64.data(), 4 * bp.tp64.size(), hipMemcpyHostToDevice, hs)) ||
      (e = hipMemcpyAsync(ws + bp.off_act, bp.active.data(), 4 * bp.active.size(), hipMemcpyHostToDevice, hs)))
    return amy_hip_fail(e, "batch tables upload");
  if ((e = amy_launch_fill_u32((unsigned*)(ws + bp.off_ctl), sizeof(BatchCtl) / 4, hs)) != hipSuccess)
    return amy_hip_fail(e, "batch control reset");
  int dev = 0, ncu = 0, occ = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, amy_batch_persistent_kernel(bp.f64, bp.fs), 64, bp.lds);
  if (e != hipSuccess || occ < 1) return amy_hip_fail(e, "batch occupancy query");
  // Every workgroup of the cooperative grid must be resident at once (the
  // grid barrier waits for all of them).  The occupancy query divides the
  // CU's LDS by the block's byte count, but gfx950 allocates LDS in whole
  // granules, so it can promise more blocks than fit; the grid is sized by
  // the granule-rounded reservation as well.
  const int bpc_lds = amy_lds_blocks_per_cu(dev, bp.lds);
  if (bpc_lds < 1) return amy_fail(AMY_E_UNSUPPORTED, "batch needs %zu B of LDS per workgroup", bp.lds);
  const int resident = std::min(occ, bpc_lds);
  const int bpc = tune.blocks_per_cu > 0 ? std::min(tune.blocks_per_cu, resident) : resident;
  const unsigned grid = (unsigned)std::max(1, ncu * bpc);
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (ms_out) {
    hipEventCreate(&ev[0]);
    hipEventCreate(&ev[1]);
    hipEventRecord(ev[0], hs);
  }
  const BatchSys* dsys = (const BatchSys*)(ws + bp.off_sys);
  const int32_t* dtp64 = (const int32_t*)(ws + bp.off_tp64);
  const unsigned g64 = (unsigned)std::min<int64_t>(std::max<int64_t>(bp.tp64[count], 1), (int64_t)ncu * 16);
  e = amy_launch_batch_init(bp.f64, dsys, count, dtp64, g64, hs);
  if (e == hipSuccess && want_tail) e = amy_launch_batch_tail(bp.fs, dsys, count, dtp64, g64, hs);
  if (e == hipSuccess && bp.maxT > 0)
    e = amy_launch_batch_persistent(bp.f64, bp.fs, grid, bp.lds, dsys, count, (const int32_t*)(ws + bp.off_tp),
                                    (const int32_t*)(ws + bp.off_act), bp.maxT, (BatchCtl*)(ws + bp.off_ctl),
                                    std::max(1, tune.chunk), tune.xcd_order, hs);
  if (e == hipSuccess && bp.maxT > 0)
    e = amy_launch_batch_poison(dsys, count, (const BatchCtl*)(ws + bp.off_ctl), hs);
  if (e != hipSuccess) {
    if (ms_out) {
      hipEventDestroy(ev[0]);
      hipEventDestroy(ev[1]);
    }
    return amy_hip_fail(e, "batch launch");
  }
  if (ms_out) {
    hipEventRecord(ev[1], hs);
    hipEventSynchronize(ev[1]);
    hipEventElapsedTime(ms_out, ev[0], ev[1]);
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
  }
  return AMY_OK;
}

extern "C" amy_status amy_batch_solve(const amy_problem* probs, int32_t count, void* stream, void* workspace,
                                      uint64_t ws_bytes, double* const* V_out, int16_t* const* policy_out,
                                      amy_info* infos) {
  BatchPlan bp;
  amy_status st = amy_batch_plan(probs, count, bp);
  if (st != AMY_OK) return st;
  if (!workspace || ((uintptr_t)workspace & 255)) return amy_fail(AMY_E_INVALID, "workspace NULL or not 256-byte aligned");
  if (ws_bytes < bp.ws_bytes)
    return amy_fail(AMY_E_NOMEM, "batch workspace %llu B < %llu B", (unsigned long long)ws_bytes,
                    (unsigned long long)bp.ws_bytes);
  if (!V_out) return amy_fail(AMY_E_INVALID, "V_out is NULL");
  for (int i = 0; i < count; ++i)
    if (!V_out[i]) return amy_fail(AMY_E_INVALID, "V_out[%d] is NULL", i);
  hipStream_t hs = (hipStream_t)stream;
  BatchTune tune = amy_tune_lookup_batch(probs, count, bp);
  float ms = 0.f;
  st = amy_batch_run(probs, bp, hs, (char*)workspace, V_out, policy_out, infos != nullptr, tune,
                     infos ? &ms : nullptr);
  if (st != AMY_OK || !infos) return st;
  BatchCtl ctl;
  hipError_t e = hipMemcpy(&ctl, (char*)workspace + bp.off_ctl, 16, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return amy_hip_fail(e, "batch control readback");
  if (ctl.err) return amy_fail(AMY_E_DEVICE, "batch grid barrier timed out (results invalid)");
  for (int i = 0; i < count; ++i) {
    amy_info& inf = infos[i];
    memset(&inf, 0, sizeof inf);
    const Plan& pl = bp.plans[i];
    inf.mode_used = AMY_MODE_OTF;
    inf.kernel = pl.dev.variant;
    for (int d = 0; d < pl.dev.n; ++d) inf.window[d] = pl.dev.L[d];
    for (int d = 0; d < pl.dev.n; ++d)
      if (pl.dev.ccount[d] > 0) inf.table_cache_mask |= 1 << d;
    inf.lds_bytes = pl.dev.lds_bytes;
    inf.n_x = pl.dev.n_x;
    inf.n_u = pl.dev.n_u;
    inf.rows = pl.rows;
    inf.W = pl.W;
    inf.workspace_bytes = bp.ws_bytes;
    unsigned long long bits = 0;
    e = hipMemcpy(&bits, (char*)workspace + bp.base[i] + pl.off_tail, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return amy_hip_fail(e, "tail readback");
    double t;
    memcpy(&t, &bits, 8);
    inf.max_row_tail = probs[i].horizon > 0 ? t : 0.0;
    inf.tail_bound_E = inf.max_row_tail * probs[i].horizon;
    inf.t_sweeps_ms = inf.t_total_ms = ms;
  }
  return AMY_OK;
}
