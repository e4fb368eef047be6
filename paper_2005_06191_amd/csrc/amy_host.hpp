// amy_host.hpp -- host driver internals shared by the solve, batch and server code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/amytiss.h"
#include "amy_plan.hpp"

struct Plan {
  DevProblem dev;
  int64_t W;        // slots per row (may exceed INT32 for huge windows)
  int64_t rows;     // n_x * n_u
  bool f64;         // FP64 path
  int mode;         // resolved amy_mode
  uint64_t off_label, off_v0, off_v1, off_tail, off_T, off_org;
  uint64_t stored_bytes, ws_bytes;
};

// ev[0] start, ev[1] sweeps begin, ev[2] after the first T_d - 1 sweeps,
// ev[3] after the last sweep, ev[4] end.
struct Timing {
  static const int N = 5;
  hipEvent_t ev[N];
};

amy_status amy_fail(amy_status st, const char* fmt, ...);
amy_status amy_hip_fail(hipError_t e, const char* what);
amy_status amy_validate(const amy_problem* p);
void amy_make_plan(const amy_problem* p, Plan* pl);
void amy_layout(Plan* pl, int mode);
amy_status amy_resolve(const amy_problem* p, uint64_t budget, Plan* pl);
amy_status amy_enqueue(const Plan& pl, hipStream_t st, void* ws, double* V_out, int16_t* pol, int horizon,
                       bool want_tail, Timing* tm);
