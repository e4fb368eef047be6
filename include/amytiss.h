/*
 * amytiss.h -- C ABI of libamytiss_hip.so: finite-MDP abstraction and
 * finite-horizon Bellman synthesis of stochastic control systems on gfx950.
 *
 * Method (AMYTISS, arXiv 2005.06191):
 *   - Abstraction, Sec. 4 (Eq. 4.1) and Alg. 2: for every state cell x and
 *     input u the next state is f(x_bar, u_bar) + N(0, diag(var)); the
 *     transition probability to a target cell is the Gaussian mass of that
 *     cell.  Only cells whose centre lies in the cutting region
 *     [[mu - x*, mu + x*]] (Sec. 5.2 and its Remark; x* solves
 *     PDF(x*|0, var_i) = cutoff per dimension) carry probability; every row
 *     has the same number W = prod_i L_i of slots, L_i = floor(2 x*_i/h_i)+1
 *     (clamped to the grid).
 *   - Synthesis, Alg. 4: backward value iteration k = T_d .. 1 for safety,
 *     reachability and reach-avoid, V_k(x) = max_u sum_{x'} T(x'|x,u) V_{k+1}(x')
 *     (plus the one-step target mass T0 for reach / reach-avoid), and the
 *     maximising input per state and step.
 *   - Two modes: STORED builds the rows once (Alg. 2) and streams them in
 *     every step; OTF recomputes them inside every step (Sec. 6.1,
 *     on-the-fly abstraction).
 *
 * Readings of points the paper leaves open (each is part of the contract):
 *   - a state is represented by its cell centre; it belongs to a box when its
 *     centre does (closed boxes, +-INFINITY allowed);
 *   - probability mass that leaves the grid is lost (value 0);
 *   - safety uses the safe box S (default: the whole grid); states outside S
 *     have value 0;
 *   - reach and reach-avoid follow Alg. 4; a cell in both T and A counts as
 *     A; the returned V is 1 on T\A and 0 on A, policy -1 there;
 *   - policy ties go to the lowest input index;
 *   - the mean mu = f(x_bar, u_bar) is evaluated in FP64 in the order written
 *     next to each dynamics kind below, without fused multiply-adds.
 *
 * Conventions of every call:
 *   - all functions return amy_status and never throw; amy_last_error()
 *     gives a thread-local message for the last failure;
 *   - the caller owns every struct and buffer; nothing is retained after a
 *     call returns (the server copies problems at submit);
 *   - "device" pointers are HIP device memory on the current device; the
 *     library allocates no device memory on the solve path: it uses the
 *     caller's workspace, sized by amy_query;
 *   - problems are validated before any device work; outputs are undefined
 *     after an error.
 */
#ifndef AMYTISS_H
#define AMYTISS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AMY_MAX_DIM 8
#define AMY_MAX_IN 4
#define AMY_MAX_PARAMS 128

typedef enum {
  AMY_OK = 0,
  AMY_E_INVALID = 1,     /* bad problem or argument                          */
  AMY_E_NOMEM = 2,       /* workspace / budget too small                     */
  AMY_E_DEVICE = 3,      /* a HIP runtime call failed                        */
  AMY_E_UNSUPPORTED = 4, /* valid but not supported by this build            */
  AMY_E_BUSY = 5,        /* server queue full                                */
  AMY_E_NOTREADY = 6,    /* server: result not ready yet                     */
  AMY_E_CANCELLED = 7    /* server: the request was cancelled                */
} amy_status;

typedef enum { AMY_SAFETY = 0, AMY_REACH = 1, AMY_REACH_AVOID = 2 } amy_spec;
typedef enum { AMY_MODE_AUTO = 0, AMY_MODE_STORED = 1, AMY_MODE_OTF = 2 } amy_mode;

/* FP64: every mass, sum and value in FP64 (the plain GPU path).
 * FP32: cell masses and Bellman sums in FP32 (erfc-differenced tails,
 * compensated outer sums); FP64 kept for the mean and window, the per-row
 * truncated-tail mass and the last step, whose sums and output are FP64. */
typedef enum { AMY_FP64 = 0, AMY_FP32 = 1 } amy_precision;

/* Dynamics mu = f(x, u) (x = cell centre, u = input point):
 *  AMY_DYN_AFFINE    x+ = A x + B u + c; params = A[n*n], B[n*m], c[n]
 *                    (row-major); mu_i = (sum_j A_ij x_j + c_i) + sum_k B_ik u_k,
 *                    each sum taken left to right.
 *  AMY_DYN_UNICYCLE  n = 3, m = 2, u = (v, omega); params = {tau};
 *                    mu = (x + (tau v) cos th, y + (tau v) sin th, th + tau omega).
 *  AMY_DYN_ROOM      ring of n rooms, m = 1 shared heater or m = n heaters;
 *                    params = {alpha, beta, gam, T_e, T_h};
 *                    mu_i = ((c0 x_i + alpha (x_{i-1} + x_{i+1})) + beta T_e)
 *                           + u_i (gam (T_h - x_i)),  c0 = (1 - 2 alpha) - beta,
 *                    indices modulo n (rooms on a circle).
 *  AMY_DYN_VEHICLE7  n = 7, m = 2: the single-track model of the paper's
 *                    Sec. 8.4.1 with its printed right-hand sides, saturations
 *                    = clamps to the input box; params = {tau, l_wb, m, mu_bar,
 *                    l_f, l_r, h_cg, I_z, C_Sf, C_Sr, g}.
 *  AMY_DYN_ROBOT     n = 2, m = 2, p <= 1: the robot of Sec. 7, params = {tau},
 *                    mu = (x1 + (tau u1) cos u2 + w, x2 + (tau u1) sin u2 + w)
 *                    (the printed second row's factor u2 read as the speed u1;
 *                    no w term without a disturbance).
 * With a disturbance (p > 0) only AFFINE and ROBOT take it: AFFINE appends
 * D[n*p] (row-major) to its params and adds (sum_l D_il w_l) last. */
/* Bellman-sweep kernel variant.  AUTO lets the library (and its autotuner
 * cache) choose; the others force one, for tests and tuning:
 *   LANES    one lane per state, window lengths at run time (any shape whose
 *            per-lane 1-D tables fit in LDS);
 *   FIXED    one lane per state, window shape compiled in (the instantiated
 *            shapes of the built-in workload families only);
 *   GROUP16  16 lanes per state (4 states per wave) share the state's tables
 *            and split its window -- for windows of hundreds to thousands
 *            of cells;
 *   GROUP64  one wavefront per (state, input) row -- the largest windows;
 *   FACTORED compiled shape whose innermost dimension alone moves with the
 *            last input digit (the unicycle's heading with the turn rate):
 *            the outer contraction is shared by all values of that digit.
 *            Same values up to summation order (not bitwise equal to LANES).
 *   INPUTS   one wavefront per state, its lanes splitting the state's inputs
 *            (Alg. 4's parallel loop over X x U): for problems with few
 *            states and many (input, disturbance) rows; normal noise only.
 * LANES, FIXED, INPUTS and the GROUP variants give bitwise equal results. */
typedef enum {
  AMY_VARIANT_AUTO = 0,
  AMY_VARIANT_LANES = 1,
  AMY_VARIANT_FIXED = 2,
  AMY_VARIANT_GROUP16 = 3,
  AMY_VARIANT_GROUP64 = 4,
  AMY_VARIANT_FACTORED = 5,
  AMY_VARIANT_INPUTS = 6
} amy_variant;

typedef enum {
  AMY_DYN_AFFINE = 0,
  AMY_DYN_UNICYCLE = 1,
  AMY_DYN_ROOM = 2,
  AMY_DYN_VEHICLE7 = 3,
  AMY_DYN_ROBOT = 4,
  AMY_DYN_USER = 5     /* right-hand side given as source text: amy_user_dynamics_create */
} amy_dyn_kind;

/* Noise distributions (Sec. 3 after Eq. 3.2 and Sec. 6.2: normal, uniform,
 * exponential and beta), independent across dimensions:
 *  NORMAL       zero mean, variance noise_var[i] (the default);
 *  UNIFORM      uniform on [a[i], b[i]];
 *  EXPONENTIAL  density rate e^{-rate t} for t >= 0, rate = a[i] > 0;
 *  BETA         beta(alpha[i], beta[i]) stretched onto [a[i], b[i]],
 *               alpha, beta >= 1 (a bounded density). */
typedef enum {
  AMY_NOISE_NORMAL = 0,
  AMY_NOISE_UNIFORM = 1,
  AMY_NOISE_EXPONENTIAL = 2,
  AMY_NOISE_BETA = 3
} amy_noise_kind;

/* Which cells a row keeps around its mean mu (Sec. 5.2):
 *  CENTRE     the paper's rule: cells whose centre lies in the cutting
 *             interval [mu - x*, mu + x*] (normal noise only);
 *  INTERSECT  cells that meet the cutting interval, so that no cell with
 *             mass inside it is dropped.  The other distributions always
 *             use INTERSECT with their support as the interval (Sec. 6.2:
 *             the cut is tuned to the support of the density); the
 *             exponential's support [0, inf) is cut where its density
 *             falls to the cutoff gamma. */
typedef enum { AMY_WINDOW_CENTRE = 0, AMY_WINDOW_INTERSECT = 1 } amy_window_rule;

/* State grid: dimension i has count[i] cells [lo[i] + j h[i], lo[i] + (j+1) h[i]);
 * states are numbered row-major, the last dimension fastest. */
typedef struct {
  int32_t n;
  int32_t count[AMY_MAX_DIM];
  double lo[AMY_MAX_DIM];
  double h[AMY_MAX_DIM];
} amy_grid;

/* Input set: dimension k is the inclusive linspace lo[k] .. hi[k] with
 * count[k] points, u = lo + j * ((hi - lo)/(count - 1)); one point is lo.
 * Inputs are numbered row-major, the last dimension fastest. */
typedef struct {
  int32_t m;
  int32_t count[AMY_MAX_IN];
  double lo[AMY_MAX_IN];
  double hi[AMY_MAX_IN];
} amy_inputs;

/* Disturbance set W-hat (Def. 3.1, its representative points): dimension l
 * is the inclusive linspace lo[l] .. hi[l] with count[l] points (one point
 * is lo); p = 0 means no disturbance.  The disturbance is an adversary
 * (the Remark after Def. 3.2): a step takes V(x) = max_u min_w V_in(x,u,w)
 * (Alg. 3 and Alg. 4).  m + p <= AMY_MAX_IN. */
typedef struct {
  int32_t p;
  int32_t count[AMY_MAX_IN];
  double lo[AMY_MAX_IN];
  double hi[AMY_MAX_IN];
} amy_disturbance;

/* Noise model; all zero = additive normal noise with the paper's cut. */
typedef struct {
  int32_t kind;                  /* amy_noise_kind                           */
  int32_t window;                /* amy_window_rule (NORMAL only)            */
  int32_t multiplicative;        /* NORMAL only: Upsilon = varsigma x (Eq. 3.2):
                                    dimension i's noise has standard deviation
                                    sqrt(noise_var[i]) |x_i| at state x; the
                                    cut is disabled (Sec. 6.2), rows span the
                                    whole grid                               */
  int32_t reserved;
  double a[AMY_MAX_DIM], b[AMY_MAX_DIM];        /* support / rate            */
  double alpha[AMY_MAX_DIM], beta[AMY_MAX_DIM]; /* BETA shapes               */
} amy_noise;

/* Closed box; set lo > hi in any dimension for the empty box. */
typedef struct {
  double lo[AMY_MAX_DIM];
  double hi[AMY_MAX_DIM];
} amy_box;

typedef struct {
  int32_t kind;        /* amy_dyn_kind */
  int32_t n_params;
  double params[AMY_MAX_PARAMS];
} amy_dynamics;

typedef struct {
  amy_grid grid;
  amy_inputs inputs;
  amy_dynamics dyn;
  double noise_var[AMY_MAX_DIM]; /* diag of the covariance (variances)       */
  double cutoff;                 /* gamma >= 0; 0 keeps every cell           */
  int32_t horizon;               /* T_d >= 0                                 */
  int32_t spec;                  /* amy_spec                                 */
  amy_box target;                /* reach / reach-avoid                      */
  amy_box avoid;                 /* reach-avoid                              */
  amy_box safe;                  /* safety                                   */
  int32_t mode;                  /* amy_mode                                 */
  int32_t precision;             /* amy_precision                            */
  int32_t variant;               /* amy_variant (0 = AUTO)                   */
  amy_disturbance dist;          /* p = 0: none                              */
  amy_noise noise;               /* zero: additive normal, centre rule       */
} amy_problem;

typedef struct {
  int32_t mode_used;             /* AMY_MODE_STORED or AMY_MODE_OTF          */
  int32_t window[AMY_MAX_DIM];   /* L_i                                      */
  int32_t kernel;                /* amy_variant the sweeps ran with          */
  int32_t table_cache_mask;      /* bit i: dimension i's 1-D tables are built
                                    once per state for every input-digit
                                    combination its mean depends on          */
  int32_t lds_bytes;             /* dynamic LDS per 64-state workgroup       */
  int64_t n_x, n_u, rows, W;     /* states, inputs, rows = n_x n_u n_w, slots*/
  uint64_t workspace_bytes;      /* bytes amy_solve needs for this problem   */
  uint64_t stored_bytes;         /* of which transition rows (STORED mode)   */
  double max_row_tail;           /* max over rows of the cut-off mass (FP64) */
  double tail_bound_E;           /* T_d * max_row_tail: V_{no cut} <= V + E  */
  /* phase times (HIP events on the solve's stream), filled when info != NULL:
   * build = labels, tail and (STORED) row construction; sweeps = all T_d
   * Bellman steps; main_sweeps = steps k = T_d - 1 .. 2, the T_d - 2 launches
   * of the working-precision sweep alone (the first step also computes the
   * FP64 tail, the last one writes FP64 V; 0 when T_d < 3). */
  double t_build_ms, t_sweeps_ms, t_main_sweeps_ms, t_readout_ms, t_total_ms;
  int64_t n_w;                   /* disturbance points (1 without)           */
} amy_info;

/* Cells of the paper's quantisation convention (the robot example of
 * Sec. 7, the case studies of Sec. 8 and the pair counts of Table 4): a box
 * [lb, ub] with quantisation parameter q has the representative points
 * lb + j q, j = 0 .. floor((ub - lb)/q + 1e-9), both ends included.  As
 * cells: lo = lb - q/2, h = q, count = floor((ub - lb)/q + 1e-9) + 1 (the
 * 1e-9 absorbs the binary rounding of ratios such as 0.6/0.1 = 5.999...).
 * lb, ub, q: host arrays of n doubles (caller-owned, read only); out: host
 * struct, filled on success (its other fields zeroed).  Pure host
 * arithmetic, no device work.  AMY_E_INVALID when n is outside 1..8, an
 * array or out is NULL, q <= 0, ub < lb, a value is not finite or a count
 * exceeds 2^31 - 1. */
amy_status amy_grid_from_quantization(int32_t n, const double* lb, const double* ub, const double* q,
                                      amy_grid* out);

/* The same convention for an input set (Sec. 7: input quantisation
 * parameter): m dimensions (1..4), points lb + j q as the inclusive linspace
 * lo = lb, hi = lb + (count - 1) q.  Errors as above. */
amy_status amy_inputs_from_quantization(int32_t m, const double* lb, const double* ub, const double* q,
                                        amy_inputs* out);

/* Problem statement of Alg. 2 and Alg. 4 (state, input and noise sets,
 * cutoff gamma of Sec. 5.2, horizon T_d, specification and its sets):
 * validate p and fill sizes, the mode AUTO resolves to for a workspace of
 * at most ws_budget bytes (0 = unlimited) and the workspace size.
 * p, out: host structs owned by the caller (out may be NULL).  No device
 * work.  AMY_E_INVALID for a malformed problem; AMY_E_NOMEM when even the
 * OTF mode needs more than ws_budget; AMY_E_UNSUPPORTED for a valid problem
 * this build cannot solve (window tables larger than LDS, more than 2^31
 * states, more than 32767 inputs). */
amy_status amy_query(const amy_problem* p, uint64_t ws_budget, amy_info* out);

/* Alg. 4 (synthesis) over the abstraction of Alg. 2 -- rows built once and
 * streamed (STORED) or rebuilt inside every step (OTF, Sec. 6.1) -- for the
 * specification of Alg. 3: backward value iteration k = T_d .. 1, the max
 * over inputs and its argmax of the collect step.
 * Solve p on the HIP stream `stream` (hipStream_t; NULL = default stream).
 * workspace: device memory of ws_bytes >= amy_query's workspace_bytes
 * (computed with the same budget).  V_out: device double[n_x], V at k = 1.
 * policy_out: device int16[T_d * n_x] or NULL; entry (k-1)*n_x + x is the
 * maximising input at step k (-1 where the value is fixed).
 * info == NULL: the call only enqueues work and returns.  info != NULL: the
 * call waits for the stream and fills info, including the FP64 tail bound
 * and the phase times (HIP events on `stream`). */
amy_status amy_solve(const amy_problem* p, void* stream, void* workspace, uint64_t ws_bytes,
                     double* V_out, int16_t* policy_out, amy_info* info);

/* ------------------------------------------------- allocation-free solve
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid allocation): amy_solve
 * without a workspace argument.  The library keeps one static workspace of
 * AMY_STATIC_WORKSPACE_BYTES in the memory of every device it runs on (held
 * until the process ends) and runs amy_solve's kernels on it.  The call
 * only enqueues work on `stream`, like amy_solve with info == NULL, and
 * allocates nothing.  V_out, policy_out: as for amy_solve (device buffers,
 * caller-owned).  AMY_E_NOMEM when the problem's workspace (amy_query's
 * workspace_bytes) exceeds the limit; other errors as amy_solve.  All calls
 * on one device share that workspace: calls ordered on one stream are safe,
 * calls whose work can overlap on one device (other streams, other threads)
 * race and give undefined results. */
#define AMY_STATIC_WORKSPACE_BYTES (96ull << 20)
amy_status amy_solve_static(const amy_problem* p, void* stream, double* V_out, int16_t* policy_out);

/* ------------------------------------------------- dynamics as source text
 * Sec. 3: the user gives the right-hand side of the difference equation as
 * text.  rhs is the body of a device function
 *     void rhs(const double* x, const double* u, const double* w,
 *              const double* params, double* mu)
 * that reads the state's cell centre x[0..n), the input u[0..m), the
 * disturbance w[0..p) and the problem's dyn.params[0..n_params), and writes
 * the mean mu[0..n) (C++ in FP64, the C math functions available; it is
 * compiled without fused multiply-adds).  The text is compiled for gfx950
 * with hipRTC and loaded on the current device; it runs with the library's
 * privileges, so it must come from a trusted source.  create: AMY_E_INVALID
 * when the text does not compile (the compiler's message in
 * amy_last_error), AMY_E_DEVICE when the module cannot be loaded.  The
 * handle is owned by the caller until destroy. */
typedef struct amy_user_dynamics amy_user_dynamics;
amy_status amy_user_dynamics_create(const char* rhs, int32_t n, int32_t m, int32_t p, amy_user_dynamics** out);
amy_status amy_user_dynamics_destroy(amy_user_dynamics* f);

/* amy_solve for a problem whose dyn.kind is AMY_DYN_USER (amy_solve refuses
 * those), with the rows built by the compiled right-hand side f: on the
 * fly, with the run-time-window sweeps (one lane per state, or 16 or 64
 * lanes per state for large windows; amy_query sizes the workspace).  p's n, m and
 * dist.p must be those f was compiled for, on the current device.  Other
 * arguments and errors as amy_solve. */
amy_status amy_solve_user(const amy_user_dynamics* f, const amy_problem* p, void* stream, void* workspace,
                          uint64_t ws_bytes, double* V_out, int16_t* policy_out, amy_info* info);

/* ---------------------------------------------------------------- batch
 * Many independent systems (uneven grids, inputs and horizons) in ONE
 * cooperative persistent launch (the batched form of Alg. 4): workgroups
 * take 64-state tiles from per-XCD work queues, a grid-wide barrier
 * separates the Bellman steps, and each system's rows are computed exactly
 * as amy_solve computes them with AMY_VARIANT_LANES (bitwise equal).
 * All systems share one precision and run on the fly (mode AUTO or OTF);
 * the compiled families are affine n = 1..4, unicycle, room n = 2..5 and
 * the 7-D vehicle.  Horizons up to 1024, up to 4096 systems. */

/* Workspace bytes of a batch of count problems (host array, caller-owned;
 * each validated as amy_query does).  No device work.  AMY_E_INVALID for a
 * malformed problem or count outside 1..4096, AMY_E_UNSUPPORTED for a
 * family, mode or horizon the batched kernel does not take. */
amy_status amy_batch_query(const amy_problem* probs, int32_t count, uint64_t* ws_bytes);

/* Alg. 4 for count independent systems in one launch (the batched form of
 * the synthesis loop; every system's rows as amy_solve computes them).
 * workspace: device memory of ws_bytes >= amy_batch_query's size.
 * Solve count systems.  V_out[i]: device double[n_x(i)]; policy_out: NULL
 * or count device int16 buffers (each T_d(i) * n_x(i), entries may be NULL).
 * infos: NULL (asynchronous) or count amy_info, filled after waiting for the
 * stream (including each system's FP64 tail bound; t_total_ms is the time
 * of the whole launch).  AMY_E_DEVICE if a grid-barrier wait gave up; in
 * the asynchronous mode (infos == NULL) every V_out then holds NaN. */
amy_status amy_batch_solve(const amy_problem* probs, int32_t count, void* stream, void* workspace,
                           uint64_t ws_bytes, double* const* V_out, int16_t* const* policy_out,
                           amy_info* infos);

/* --------------------------------------------------------------- autotuner
 * Measures candidate launch configurations on the device and caches the
 * fastest per shape class (dynamics, dimension, window, precision, size
 * buckets); later calls with mode/variant AUTO use the cached choice.
 * Single solve: sweep variant.  Batch: tiles per work-queue grab, resident
 * workgroups per CU, XCD-partitioned queues.  Tuning overwrites V_out. */
typedef struct {
  int32_t chunk, blocks_per_cu, xcd_order, variant;
  int32_t candidates;
  double best_ms, worst_ms;
} amy_tune_result;

/* The paper leaves the mapping of Alg. 4's parallel loops onto the device
 * to its runtime; these calls pick it by measurement.
 * amy_tune_solve: times every feasible sweep variant of p (each a full solve
 * on `stream` in the caller's workspace, sized by amy_query) and caches the
 * fastest for p's shape class.  amy_tune_batch: the same for a batch's
 * launch parameters; a candidate whose grid barrier gave up is discarded.
 * Synchronous; AMY_E_DEVICE on a HIP failure. */
amy_status amy_tune_solve(const amy_problem* p, void* stream, void* workspace, uint64_t ws_bytes,
                          double* V_out, amy_tune_result* out);
amy_status amy_tune_batch(const amy_problem* probs, int32_t count, void* stream, void* workspace,
                          uint64_t ws_bytes, double* const* V_out, amy_tune_result* out);
/* The cache as JSON {"<shape class>": {"chunk":..,"blocks_per_cu":..,"xcd_order":..,
 * "variant":..,"ms":..}}; load merges into the in-process cache. */
amy_status amy_tune_save(const char* path);
amy_status amy_tune_load(const char* path);
amy_status amy_tune_clear(void);
int32_t amy_tune_entries(void);

/* ----------------------------------------------------------------- server
 * Request loop with continuous batching.  A worker thread owns one HIP
 * stream and one device arena of hbm_budget_bytes (the only device
 * allocation, made here).  Requests are admitted in arrival order while a
 * slot (max_slots) and arena space for their footprint are free; each
 * request's mode (stored rows vs on the fly) is picked by memory and a
 * cost model when its mode is AUTO.  Every iteration advances all admitted
 * requests by one Bellman step in a single replay of a captured graph, so
 * requests that arrive while others run join at the next step and their
 * work overlaps on the device; finished requests leave, freeing their slot
 * and memory.  A request's result is bitwise equal to amy_solve of the same
 * problem with the variant its info reports (LANES or GROUP*).
 * Supported: the dynamics families of amy_batch_solve. */
typedef struct amy_server amy_server;
typedef struct {
  uint64_t hbm_budget_bytes;     /* device arena (>= 1 MiB)                  */
  int32_t max_slots;             /* requests on the device at once (1..4096) */
  int32_t device;                /* HIP device ordinal                       */
} amy_server_cfg;

typedef struct {
  uint64_t submitted, completed, failed;
  int32_t queued, active, max_active;
  uint64_t hbm_in_use, hbm_peak;
  uint64_t steps;                /* batched step launches (graph replays)    */
  double row_updates;            /* completed requests' n_x n_u T_d          */
  double busy_s;                 /* worker time with work on the device      */
  double p50_ms, p99_ms, mean_ms;/* submit-to-result latency, completed      */
  uint64_t cancelled;            /* requests cancelled before finishing      */
} amy_server_stats;

/* Serving form of Alg. 4 with the memory trade-off of Sec. 6.1 (stored rows
 * when they fit, on-the-fly rows otherwise) decided per request.
 * create: allocates the arena on cfg->device and starts the worker;
 * AMY_E_INVALID for a bad cfg, AMY_E_DEVICE / AMY_E_NOMEM when the arena
 * cannot be allocated.  *out is owned by the caller until amy_server_destroy. */
amy_status amy_server_create(const amy_server_cfg* cfg, amy_server** out);
/* Queue a request (validated as amy_query does; AMY_E_NOMEM when it can never
 * fit the arena, AMY_E_UNSUPPORTED for a family the batched step lacks).
 * Copies the problem; want_policy != 0 keeps the T_d x n_x policy. */
amy_status amy_server_submit(amy_server* s, const amy_problem* p, int32_t want_policy, uint64_t* ticket);
/* Result of a finished request into host buffers (V_host: n_x doubles;
 * policy_host: T_d * n_x int16 or NULL); the ticket is then released.
 * info: mode, variant, tail bound; t_build_ms = queueing time,
 * t_sweeps_ms = time admitted, t_total_ms = latency.
 * poll: AMY_E_NOTREADY while running.  wait: blocks up to timeout_ms
 * (< 0: no limit) before answering AMY_E_NOTREADY. */
amy_status amy_server_poll(amy_server* s, uint64_t ticket, double* V_host, int16_t* policy_host,
                           amy_info* info);
amy_status amy_server_wait(amy_server* s, uint64_t ticket, int32_t timeout_ms, double* V_host,
                           int16_t* policy_host, amy_info* info);
/* Cancel a queued or running request.  A queued request leaves the queue at
 * once; a running one leaves at the next step boundary (its steps already
 * launched complete first), and its slot and arena space are freed then.
 * poll / wait on the ticket then answer AMY_E_CANCELLED (and release it).
 * AMY_E_INVALID for an unknown ticket or a request that has already finished
 * (its result stays available). */
amy_status amy_server_cancel(amy_server* s, uint64_t ticket);
amy_status amy_server_get_stats(amy_server* s, amy_server_stats* out);
amy_status amy_server_reset_stats(amy_server* s);
/* Finishes the admitted requests, drops the queued ones, frees everything. */
amy_status amy_server_destroy(amy_server* s);

/* Message of the last failed call on this thread ("" if none); the string
 * is owned by the library and valid until the thread's next failing call. */
const char* amy_last_error(void);

/* Library version string (static storage). */
const char* amy_version(void);

#ifdef __cplusplus
}
#endif
#endif /* AMYTISS_H */
