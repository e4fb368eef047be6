// amy_batch.hpp -- host-side entry points of the batched kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "amy_plan.hpp"

bool amy_batch_supports(int kind, int n, int mode);
// family set a system needs: 0 = the 2-D / 3-D set, 1 = every family
int amy_batch_family_set(int kind, int n);
const void* amy_batch_persistent_kernel(bool f64, int fs);
hipError_t amy_launch_batch_persistent(bool f64, int fs, unsigned grid, size_t lds, const BatchSys* sys, int nsys,
                                       const int32_t* tprefix, const int32_t* active, int max_steps,
                                       BatchCtl* ctl, int chunk, int xcd_order, hipStream_t st);
const void* amy_batch_step_kernel(bool f64, int fs);
// meta[0] = number of systems, meta[1..] = tile prefix sums (device memory)
hipError_t amy_launch_batch_step(bool f64, int fs, unsigned grid, size_t lds, const BatchSys* sys,
                                 const int32_t* meta, hipStream_t st);
// tp64: prefix sums of the systems' 64-state tiles
hipError_t amy_launch_batch_init(bool f64, const BatchSys* sys, int nsys, const int32_t* tp64, unsigned grid,
                                 hipStream_t st);
hipError_t amy_launch_batch_tail(int fs, const BatchSys* sys, int nsys, const int32_t* tp64, unsigned grid,
                                 hipStream_t st);
hipError_t amy_launch_fill_u32(unsigned* p, size_t n, hipStream_t st);
// NaN into every system's V_out when the launch's control block has err set
hipError_t amy_launch_batch_poison(const BatchSys* sys, int nsys, const BatchCtl* ctl, hipStream_t st);
