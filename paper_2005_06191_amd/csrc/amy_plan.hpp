// amy_plan.hpp -- problem plan shared by the host driver and the kernels.
//
// The host turns an amy_problem into a DevProblem once (FP64 sizing of the
// cutting region, strides, reciprocals); kernels receive it by value as a
// kernel argument (< 4 KB), so every field is uniform across a launch and
// lives in scalar registers.
#pragma once
#include <stdint.h>

#define AMY_MAXD 8
#define AMY_MAXI 4
#define AMY_MAXP 128

enum { LBL_FREE = 0, LBL_ZERO = 1, LBL_ONE = 2 };

struct DevProblem {
  int32_t n, m, kind, spec;
  int32_t count[AMY_MAXD];
  int32_t L[AMY_MAXD];        // fixed window length per dimension
  int32_t Loff[AMY_MAXD + 1]; // offsets of the per-dimension 1-D tables
  int32_t ucount[AMY_MAXI];
  int32_t n_u;
  int32_t W;                  // prod L
  int32_t nocut;              // cutoff == 0: the window is the whole grid
  int32_t n_x;                // states (< 2^31)
  int64_t stride[AMY_MAXD];   // state index strides, last dimension fastest
  double lo[AMY_MAXD], h[AMY_MAXD], inv_h[AMY_MAXD];
  double inv_sigma[AMY_MAXD], xstar[AMY_MAXD];
  double ulo[AMY_MAXI], ustep[AMY_MAXI], uhi[AMY_MAXI];
  double tlo[AMY_MAXD], thi[AMY_MAXD];
  double alo[AMY_MAXD], ahi[AMY_MAXD];
  double slo[AMY_MAXD], shi[AMY_MAXD];
  double params[AMY_MAXP];
};

static_assert(sizeof(DevProblem) < 4096, "kernel argument limit");
