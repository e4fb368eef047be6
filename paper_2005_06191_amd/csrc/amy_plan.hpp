// amy_plan.hpp -- problem plan shared by the host driver and the kernels.
//
// The host turns an amy_problem into a DevProblem once (FP64 sizing of the
// cutting region, strides, reciprocals); kernels receive it by value as a
// kernel argument (< 4 KB), so every field is uniform across a launch and
// lives in scalar registers.
#pragma once
#ifndef __HIPCC_RTC__
#include <stdint.h>
#endif

#define AMY_MAXD 8
#define AMY_MAXI 4
#define AMY_MAXP 128
#define AMY_TABLE_SLOTS 8  // masses per entry of the shared / memoised 1-D tables

// Slots of one memoised-table record: the window's masses, then the origin's
// bits in the last slot, padded to a power of two so that a record is one
// aligned vector load.
static inline constexpr int amy_memo_rec(int lmax) {
  return lmax + 1 <= 2 ? 2 : lmax + 1 <= 4 ? 4 : lmax + 1 <= 8 ? 8 : 16;
}

enum { LBL_FREE = 0, LBL_ZERO = 1, LBL_ONE = 2 };

struct DevProblem {
  int32_t n, m, kind, spec;
  // Disturbance (Def. 3.1): the input walk runs over nd = m + pd digits,
  // the m inputs then the pd disturbance dimensions (their counts, lower
  // ends and steps in ucount / ulo / ustep from index m on); every state has
  // n_rows = n_u n_w rows (x, u, w), disturbance fastest.
  int32_t pd, nd, n_w, n_rows;
  // Noise model: 0 normal (sigma from the variance), 1 uniform on [a, b],
  // 2 exponential with rate lambda, 3 beta(alpha, beta) on [a, b].  The
  // standardised edge coordinate is z = (edge - mu) inv_sigma with
  // inv_sigma = 1/sigma, 1/(b - a), lambda, 1/(b - a); zoff = a/(b - a)
  // for the supports that start at a (the support is z - zoff in [0, 1]).
  // wrule: 0 keeps the cells whose centre lies in the cutting interval,
  // 1 the cells that intersect it.  mult: normal noise scaled by the
  // state's own coordinate (Eq. 3.2, multiplicative), no cut.
  int32_t noise, wrule, mult, pad0;
  double zoff[AMY_MAXD], balpha[AMY_MAXD], bbeta[AMY_MAXD];
  int32_t count[AMY_MAXD];
  int32_t L[AMY_MAXD];        // fixed window length per dimension
  int32_t ucount[AMY_MAXI];
  int32_t n_u;
  int32_t W;                  // prod L
  int32_t nocut;              // cutoff == 0: the window is the whole grid
  int32_t n_x;                // states (< 2^31)
  // Table caching.  Dimension i's mean depends only on the input dimensions
  // k with dep_mult[i][k] > 0; its 1-D table for input digits d is table
  // number c = sum_k d_k dep_mult[i][k] of that dimension.  ccount[i] > 0:
  // all ccount[i] tables of the state are built once before the input loop;
  // ccount[i] == 0: the table is rebuilt inside the loop when mu_i changes.
  int32_t dep_mult[AMY_MAXD][AMY_MAXI];
  int32_t ccount[AMY_MAXD];
  // The same numbering for every dimension, cached or not: table c of
  // dimension i for digits d is c = sum_k d_k rmult[i][k], of rcount[i].
  int32_t rmult[AMY_MAXD][AMY_MAXI];
  int32_t rcount[AMY_MAXD];
  // Shared relative tables (factored sweep of a family whose mean in
  // dimension i, minus the state's own cell centre, depends only on the
  // inputs and on the state's cell centre in dimension rctx[i], or on the
  // inputs alone when rctx[i] < 0): entry j * rcount[i] + c + rel_off[i]
  // holds the 1-D masses of the kept cells relative to the state's cell
  // (zero past the kept count) and their first cell's relative index.
  int32_t rctx[AMY_MAXD];
  int32_t rel_off[AMY_MAXD];
  int32_t rel_entries;        // 0: no shared tables
  // Memoised tables (compiled-shape sweep): dimension i's mean depends only
  // on the inputs and on the state's coordinates in dimensions mctx[i][0 ..
  // mctx_n[i]); entry rel_off[i] + cx * rcount[i] + c holds the absolute
  // window origin and masses for context cells cx = sum_k j_k mmult[i][k].
  int32_t mctx_n[AMY_MAXD];
  int32_t mctx[AMY_MAXD][4];
  int32_t mmult[AMY_MAXD][4];
  int32_t tables;             // 0 none, 1 relative (factored sweep), 2 memoised (compiled-shape sweep)
  int32_t toff[AMY_MAXD];     // first LDS table entry of dimension i
  int32_t ooff[AMY_MAXD];     // first cached-origin slot of dimension i
  int32_t lds_int_off;        // byte offset of the origin slots in a block's LDS
  int32_t lds_tail_off;       // byte offset of the FP64 (window, grid) masses
  int32_t lds_bytes;          // generic sweep: block LDS without / with the tail region
  int32_t lds_bytes_tail;
  int32_t lds_bytes_fixed;    // compiled-shape sweep without the tail region
  int32_t variant;            // resolved amy_variant of the OTF sweeps
  // Group variant (G lanes per state): 1-D tables of a state at goff[i]
  // inside its group's LDS region of gsl entries; the innermost dimensions
  // from index grp_nout on form the lane space split across the G lanes.
  int32_t grp_g;
  int32_t grp_nout;
  int32_t gsl;
  int32_t goff[AMY_MAXD];
  int32_t lds_bytes_group;    // group variant: (64 / grp_g) states x gsl entries
  int64_t stride[AMY_MAXD];   // state index strides, last dimension fastest
  double lo[AMY_MAXD], h[AMY_MAXD], inv_h[AMY_MAXD];
  double inv_sigma[AMY_MAXD], xstar[AMY_MAXD];
  // window rule precomputed per dimension for the cutting interval
  // [mu + zl, mu + zh] (normal: zl = -x*, zh = x*): the centre rule keeps
  // ceil(mu inv_h - win_a) .. floor(mu inv_h - win_b) with
  // win_a = (lo - zl) inv_h + 1/2 and win_b = (lo - zh) inv_h + 1/2; the
  // intersect rule keeps floor(mu inv_h - win_a) .. ceil(mu inv_h - win_b) - 1
  // with win_a = (lo - zl) inv_h and win_b = (lo - zh) inv_h;
  // edge j sits at z = (lo - mu) inv_sigma + j hs, hs = h inv_sigma.
  double win_a[AMY_MAXD], win_b[AMY_MAXD], hs[AMY_MAXD];
  double ulo[AMY_MAXI], ustep[AMY_MAXI], uhi[AMY_MAXI];
  double tlo[AMY_MAXD], thi[AMY_MAXD];
  double alo[AMY_MAXD], ahi[AMY_MAXD];
  double slo[AMY_MAXD], shi[AMY_MAXD];
  double params[AMY_MAXP];
};

static_assert(sizeof(DevProblem) < 4096, "kernel argument limit");

// ------------------------------------------------------------------ batch

#define AMY_BATCH_MAX 4096       // systems per batched launch
#define AMY_BATCH_MAX_STEPS 1024 // global steps per batched launch (max horizon)

// One system of a batched launch (device copy; pointers into the workspace
// or the caller's outputs).
struct BatchSys {
  DevProblem P;                  // plan, variant LANES
  uint8_t* label;
  void* V0;                      // working-precision ping-pong
  void* V1;
  double* Vout;                  // FP64 V at k = 1 (caller's buffer)
  int16_t* pol;                  // caller's policy (T_d * n_x) or null
  unsigned long long* tailmax;   // FP64 max row tail (bits)
  void* T;                       // stored rows (mode STORED) or null
  int32_t* org;
  int32_t horizon;
  int32_t tiles;                 // 64-state tiles
  int32_t mode;                  // AMY_MODE_STORED / AMY_MODE_OTF
  int32_t want_tail;
  int32_t step_base;             // server: global step at which the system's step T_d runs
  int32_t pad[3];
};

// Control words of a batched launch (zeroed before the launch).
struct BatchCtl {
  unsigned bar_count;            // grid barrier arrivals
  unsigned bar_gen;              // grid barrier generation
  unsigned err;                  // 1: a barrier wait gave up
  unsigned pad;
  unsigned ctr[(AMY_BATCH_MAX_STEPS + 1) * 8];  // work-queue counters [phase][XCD] (phase 0 = init)
};
