// amy_kernels.hpp -- host-side entry points of the kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "amy_plan.hpp"

enum SweepKind {
  SWEEP_F64 = 0,      // FP64 masses, sums and values
  SWEEP_F32 = 1,      // FP32 masses and sums, FP32 values in and out
  SWEEP_F32_LAST = 2  // FP32 masses, FP64 sums, FP32 values in, FP64 out (k = 1)
};

hipError_t amy_launch_init(const DevProblem& P, uint8_t* label, void* V0, bool v0_double, double* Vout,
                           unsigned long long* tailmax, hipStream_t st);
hipError_t amy_launch_copy_out(int64_t n, const void* src, bool src_double, double* dst, hipStream_t st);
hipError_t amy_launch_tail(const DevProblem& P, const uint8_t* label, unsigned long long* tailmax,
                           hipStream_t st);
// tailmax != NULL: the launch also computes the FP64 max row tail (first step).
hipError_t amy_launch_sweep_otf(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                                const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                                hipStream_t st);
// Group variant (P.grp_g lanes per state).
hipError_t amy_launch_sweep_group(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                                  const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                                  hipStream_t st);
hipError_t amy_launch_build(const DevProblem& P, bool f64, const uint8_t* label, void* T, int32_t* org,
                            unsigned long long* tailmax, hipStream_t st);
hipError_t amy_launch_sweep_stored(const DevProblem& P, SweepKind sk, const void* T, const int32_t* org,
                                   const void* Vin, void* Vout, const uint8_t* label, int16_t* pol,
                                   hipStream_t st);

// Fixed-window-shape sweep (amy_fixed.hip): available for the instantiated
// window shapes only.
bool amy_fixed_available(const DevProblem& P);
// every step of a solve with memoised tables runs a sweep that reads its
// masses from those tables alone (so they may hold any noise model's masses)
bool amy_fixed_memo_complete(const DevProblem& P, bool f64);
// tables: the memoised tables (P.tables == 2) for the steps without the
// FP64 tail, or nullptr.
hipError_t amy_launch_sweep_fixed(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                                  const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                                  const void* tables, hipStream_t st);
hipError_t amy_launch_memo_build(const DevProblem& P, bool f64, void* tables, hipStream_t st);
// The first step's FP64 row tails from memoised tables (P planned for them,
// tables built by amy_launch_memo_build with the same P).
// LDS of that pass per workgroup (every dimension's entries of a state, per lane)
size_t amy_tail_memo_lds(const DevProblem& P);
hipError_t amy_launch_tail_memo(const DevProblem& P, bool f64, const uint8_t* label, const void* tables,
                                unsigned long long* tailmax, hipStream_t st);
// Factored compiled-shape sweep (inputs sharing the outer dimensions' windows).
// rel: the shared relative tables (when P.rel_entries > 0).  A step given
// tailmax forms the FP64 row tails: from the memoised tables (tail_dev, the
// plan of amy_launch_tail_memo, and tail_tab, built by amy_launch_memo_build
// with it) inside the sweep when amy_fac_fuses_tail says so, else in a pass
// of its own that builds the tables per state.
bool amy_fac_available(const DevProblem& P);
int amy_rel_plan(DevProblem& P);
hipError_t amy_launch_rel_build(const DevProblem& P, bool f64, void* rel, hipStream_t st);
bool amy_fac_fuses_tail(const DevProblem& P, const DevProblem& tail_dev, bool f64);
hipError_t amy_launch_sweep_fac(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                                const uint8_t* label, int16_t* pol, unsigned long long* tailmax, const void* rel,
                                hipStream_t st, const DevProblem* tail_dev = nullptr,
                                const void* tail_tab = nullptr);
