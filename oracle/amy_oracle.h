/*
 * amy_oracle.h -- FP64 CPU oracle for the AMYTISS hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU path is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header, table or
 * helper with the HIP library (include/amytiss.h); the two only read the same
 * problem descriptions.
 *
 * What it computes (paper, Sec. 4-6):
 *   - the finite-MDP abstraction of x+ = f(x,u) + N(0, diag(var)) on a grid
 *     of cells (Eq. 4.1 and Alg. 1), each transition probability being the
 *     Gaussian mass of a target cell, restricted to the cutting region of
 *     Sec. 5.2 (Remark after Fig. 1);
 *   - finite-horizon Bellman value iteration for safety, reachability and
 *     reach-avoid (Alg. 3 / Alg. 4), returning V at k = 1 and the maximising
 *     input of every step.
 * With a disturbance set W (Def. 3.1 and the Remark after Def. 3.2: the
 * disturbance is a rational adversary), every row is (x, u, w) and the
 * update is V(x) = max_u min_w V_in(x, u, w) (Alg. 3 and Alg. 4).
 * Everything is FP64.  Every cell probability is computed directly as a
 * product of 1-D normal-CDF differences (glibc erf/erfc); no table is shared
 * between cells.
 *
 * Pins of the model means: the affine family by the separable-product
 * identity and the one-step closed form; the unicycle, the room ring
 * (Sec. 8.2) and the 7-D single-track vehicle (Sec. 8.4.1) by properties
 * their physics fixes (motion geometry, equilibria, locality, symmetry and
 * energy balance of conduction, mirror symmetry and static axle loads of a
 * car).  The vehicle's slip-angle equation is used as printed: its slip term
 * has the sign of a growing, not a restoring, slip; no pin depends on it.
 */
#ifndef AMY_ORACLE_H
#define AMY_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_DIM 8
#define ORC_MAX_IN 4
#define ORC_MAX_PARAMS 128

enum { ORC_AFFINE = 0, ORC_UNICYCLE = 1, ORC_ROOM = 2, ORC_VEHICLE7 = 3, ORC_ROBOT = 4, ORC_USER = 5 };

/* A right-hand side given by the user (Sec. 3: f as text, compiled by the
 * host compiler for the oracle): mu = f(x, u, w) with the problem's params. */
typedef void (*orc_user_fn)(const double* x, const double* u, const double* w, const double* params, double* mu);
enum { ORC_SAFETY = 0, ORC_REACH = 1, ORC_REACH_AVOID = 2 };

typedef struct {
  int32_t n;                       /* state dimensions, 1..8                 */
  int32_t count[ORC_MAX_DIM];      /* cells per dimension                    */
  double lo[ORC_MAX_DIM];          /* lower edge of cell 0                   */
  double h[ORC_MAX_DIM];           /* cell width                             */
  int32_t m;                       /* input dimensions, 1..4                 */
  int32_t ucount[ORC_MAX_IN];      /* points per input dimension             */
  double ulo[ORC_MAX_IN];          /* inclusive linspace ends                */
  double uhi[ORC_MAX_IN];
  int32_t dyn;                     /* ORC_AFFINE ...                         */
  int32_t n_params;
  double params[ORC_MAX_PARAMS];
  double var[ORC_MAX_DIM];         /* noise variances                        */
  double cutoff;                   /* gamma; 0 = no cut                      */
  int32_t horizon;                 /* T_d >= 0                               */
  int32_t spec;                    /* ORC_SAFETY ...                         */
  double tlo[ORC_MAX_DIM], thi[ORC_MAX_DIM];   /* target box               */
  double alo[ORC_MAX_DIM], ahi[ORC_MAX_DIM];   /* avoid box (empty: lo>hi) */
  double slo[ORC_MAX_DIM], shi[ORC_MAX_DIM];   /* safe box                 */
  int32_t p;                       /* disturbance dimensions, 0 = none       */
  int32_t wcount[ORC_MAX_IN];      /* points per disturbance dimension       */
  double wlo[ORC_MAX_IN];          /* inclusive linspace ends                */
  double whi[ORC_MAX_IN];
  /* noise model: 0 normal (var), 1 uniform on [na, nb], 2 exponential with
   * rate na, 3 beta(nalpha, nbeta) on [na, nb]; window: 0 centre rule,
   * 1 intersect rule (the other distributions always intersect their
   * support, the exponential's cut where its density falls to the cutoff);
   * mult: multiplicative normal noise, standard deviation sqrt(var) |x_i|
   * at state x, no cut */
  int32_t noise, window, mult;
  double na[ORC_MAX_DIM], nb[ORC_MAX_DIM], nalpha[ORC_MAX_DIM], nbeta[ORC_MAX_DIM];
  orc_user_fn user_f;              /* ORC_USER only                          */
} orc_problem;

/* Full solve.  V_out[n_x] (host) receives V at k = 1.  policy_out (may be
 * NULL) receives T_d * n_x int16: entry (k-1)*n_x + x is the lowest-index
 * maximising input at step k, -1 where the state's value is fixed.  gap_out
 * (may be NULL) has the same layout: best minus second-best Q (+inf with a
 * single input, 0 where fixed).  max_tail_out (may be NULL) receives the
 * largest per-row cut-off tail over the rows of non-fixed states.
 * threads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad input. */
int orc_solve(const orc_problem* p, int threads, double* V_out, int16_t* policy_out,
              double* gap_out, double* max_tail_out);

/* One Bellman step (k given V_{k+1}) at the listed states.  V_next is the
 * full V_{k+1} vector in the paper's representation (target/avoid entries
 * are ignored); NULL means the terminal vector V_{T_d+1}.  Outputs are per
 * listed state, with the readout convention of orc_solve (fixed states get
 * their fixed value and policy -1). */
int orc_step(const orc_problem* p, const double* V_next, const int64_t* states,
             int64_t n_states, int threads, double* V_out, int16_t* policy_out,
             double* gap_out);

/* Building blocks, exposed for the oracle's own unit tests. */
double orc_mass1d(double a, double b);              /* Phi(b) - Phi(a)      */
/* Mass of the noise of dimension i between offsets ta < tb from the mean
 * (edge - mu), for a state whose coordinate i is xi (multiplicative noise). */
double orc_noise_mass(const orc_problem* p, int i, double xi, double ta, double tb);
double orc_xstar(double var, double cutoff);         /* cutting half-width   */
/* mu = f(x, u, w) (w: the disturbance point, ignored / may be NULL when p == 0). */
int orc_mean(const orc_problem* p, const double* x, const double* u, const double* w, double* mu);
/* Kept cells [jlo[i], jhi[i]] of each dimension for mean mu; returns 1 if
 * the window is non-empty in every dimension, else 0. */
int orc_window(const orc_problem* p, const double* mu, int32_t* jlo, int32_t* jhi);
/* Row (state, input): sum of the kept cell probabilities (cell by cell) and
 * the row's tail (mass on the grid outside the kept window).  With a
 * disturbance, "input" numbers the (input, disturbance) pairs, u * n_w + w. */
int orc_row_mass(const orc_problem* p, int64_t state, int64_t input, double* sum_out,
                 double* tail_out);
/* Dense transition row over all n_x cells (cut applied), for tiny grids. */
int orc_row_dense(const orc_problem* p, int64_t state, int64_t input, double* row_out);
/* Label of every state: 0 free, 1 fixed at 0 (avoid / unsafe), 2 fixed at 1 (target). */
int orc_labels(const orc_problem* p, uint8_t* labels_out);

#ifdef __cplusplus
}
#endif
#endif
