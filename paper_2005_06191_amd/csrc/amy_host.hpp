// amy_host.hpp -- host driver internals shared by the solve, batch and server code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/amytiss.h"
#include "amy_plan.hpp"

struct amy_user_dynamics;

struct Plan {
  DevProblem dev;
  const amy_user_dynamics* user = nullptr;  // AMY_DYN_USER: the compiled right-hand side
  int64_t W;        // slots per row (may exceed INT32 for huge windows)
  int64_t rows;     // n_x * n_u
  bool f64;         // FP64 path
  int mode;         // resolved amy_mode
  uint64_t off_label, off_v0, off_v1, off_tail, off_T, off_org;
  uint64_t off_rel;  // factored sweep's shared relative tables (dev.rel_entries > 0)
  uint64_t stored_bytes, ws_bytes;
  // the factored solve's first-step FP64 tails from memoised tables: the
  // problem planned for those tables (its rel_* fields describe them) and
  // their place in the workspace
  bool tail_memo = false;
  DevProblem tail_dev;
  uint64_t off_tailtab = 0;
};

// ev[0] start, ev[1] sweeps begin, ev[5] after the first sweep (k = T_d),
// ev[2] after the first T_d - 1 sweeps, ev[3] after the last sweep, ev[4] end.
struct Timing {
  static const int N = 6;
  hipEvent_t ev[N];
};

amy_status amy_fail(amy_status st, const char* fmt, ...);
// run-time-compiled dynamics (amy_rtc.cpp)
amy_status amy_user_check(const amy_user_dynamics* f, const amy_problem* p);
hipError_t amy_user_launch_sweep(const amy_user_dynamics* f, const DevProblem& P, int sk, const void* Vin,
                                 void* Vout, const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                                 hipStream_t st);
hipError_t amy_user_launch_tail(const amy_user_dynamics* f, const DevProblem& P, const uint8_t* label,
                                unsigned long long* tailmax, hipStream_t st);
amy_status amy_hip_fail(hipError_t e, const char* what);
amy_status amy_validate(const amy_problem* p);
void amy_make_plan(const amy_problem* p, Plan* pl);
void amy_layout(Plan* pl, int mode);
amy_status amy_resolve(const amy_problem* p, uint64_t budget, Plan* pl);
amy_status amy_enqueue(const Plan& pl, hipStream_t st, void* ws, double* V_out, int16_t* pol, int horizon,
                       bool want_tail, Timing* tm);
hipError_t amy_enqueue_prepare(const Plan& pl, hipStream_t st, void* ws, int horizon);
// tail_memo: the first step forms the row tails inside the factored sweep
// from the memoised tables (built, amy_fac_fuses_tail true for the plan)
hipError_t amy_enqueue_step(const Plan& pl, hipStream_t st, void* ws, double* V_out, int16_t* pol, int horizon,
                            int k, bool want_tail, bool tail_memo = false);

#include <string>
#include <vector>

// Batched launch: per-system plans, the longest-horizon-first order, the
// tile prefix sums, the active-system counts per global step and the
// workspace layout (tables, control block, then one region per system).
struct BatchPlan {
  std::vector<Plan> plans;        // input order
  std::vector<int> order;         // launch order (horizon descending) -> input index
  std::vector<int32_t> tprefix;   // tile prefix sums in launch order (tiles of the sweep variant)
  std::vector<int32_t> tp64;      // 64-state tile prefix sums in launch order (init, tail)
  std::vector<int32_t> active;    // systems still running at each global step
  bool f64 = false;
  int maxT = 0;
  int fs = 0;                     // family set compiled into the launch (0: 2-D / 3-D, 1: all)
  size_t lds = 0;                 // dynamic LDS of the launch
  uint64_t off_sys = 0, off_tp = 0, off_tp64 = 0, off_act = 0, off_ctl = 0, ws_bytes = 0;
  std::vector<uint64_t> base;     // per system (input order): its region
};

// Launch parameters of the persistent batched kernel chosen by the tuner.
struct BatchTune {
  int chunk = 4;          // tiles taken per work-queue grab
  int blocks_per_cu = 0;  // resident workgroups per CU (0: as many as fit)
  int xcd_order = 1;      // one work queue per XCD over a contiguous tile range
};

amy_status amy_batch_plan(const amy_problem* probs, int32_t count, BatchPlan& bp);
// Workgroups of `lds` bytes of LDS resident on one CU of device dev.
int amy_lds_blocks_per_cu(int dev, size_t lds);
// lanes_lds_cap > 0: LANES systems whose per-lane tables exceed it run
// GROUP64 instead (the persistent launch reserves its largest system's LDS
// for every workgroup)
amy_status amy_batch_normalise(const amy_problem* p, Plan* pl, int lanes_lds_cap = 0);
amy_status amy_batch_run(const amy_problem* probs, const BatchPlan& bp, hipStream_t hs, char* ws,
                         double* const* V_out, int16_t* const* policy_out, bool want_tail, const BatchTune& tune,
                         float* ms_out);
