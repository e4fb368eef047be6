/*
 * amy_oracle.c -- FP64 CPU oracle (test infrastructure only; see the header).
 *
 * Written from the paper's description, in its order:
 *   Sec. 4, Eq. 4.1 / Alg. 1  : T(x'|x,u) = Gaussian mass of the cell of x'
 *                               around the mean mu = f(x_bar, u_bar).
 *   Sec. 5.2 and its Remark   : cutting region = cells whose representative
 *                               point lies in [[mu - x*, mu + x*]], x* solving
 *                               PDF(x*|0, Sigma) = gamma per dimension.
 *   Alg. 3 / Alg. 4           : backward value iteration k = T_d .. 1 with
 *                               V_in = T V (+ T0 for reach / reach-avoid),
 *                               V = max over inputs of the min over
 *                               disturbances (Def. 3.1 and its Remark: the
 *                               disturbance plays against the controller),
 *                               policy = argmax over inputs.
 * No blocking, fusion or table sharing: each cell's probability is the
 * product of its 1-D normal-CDF differences, computed on its own.
 *
 * Readings (where the paper is silent):
 *   - a state is represented by its cell centre, and is in a set when the
 *     centre is (closed boxes);
 *   - gamma is a density level of each 1-D marginal; gamma = 0 keeps all cells;
 *   - probability mass leaving the grid is lost (value 0);
 *   - safety keeps the optional safe box S; states outside S have value 0;
 *   - reach and reach-avoid share Alg. 4's recursion: T0 = mass into T\A,
 *     post-states in T u A contribute nothing else, V_{T_d+1} = 0; a cell in
 *     both T and A counts as A;
 *   - the reported V is 1 on T\A and 0 on A (policy -1 there);
 *   - policy ties go to the lowest input index;
 *   - with a disturbance, each input's value is its minimum over the
 *     disturbance points (the adversary sees the input);
 *   - the robot of Sec. 7 moves along the heading u2 by tau u1 in both rows
 *     (the printed second row's factor u2 read as the speed u1);
 *   - uniform, exponential and beta noise keep the cells that meet their
 *     support (the exponential's support cut where its density falls to
 *     gamma); the intersect rule for normal noise keeps the cells that meet
 *     [mu - x*, mu + x*];
 *   - multiplicative noise scales dimension i's standard deviation by the
 *     state's |x_i| and keeps every cell; at x_i = 0 the whole mass sits in
 *     the cell holding the mean.
 * Compiled with -ffp-contract=off so that every product and sum is rounded
 * as written.
 */
#include "amy_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SQRT_2PI 2.5066282746310002
#define INV_SQRT2 0.70710678118654752440

enum { LBL_FREE = 0, LBL_ZERO = 1, LBL_ONE = 2 };

/* ---------------------------------------------------------------- basics */

/* Standard normal mass between a <= b (Alg. 1's cell integral in one
 * dimension).  Both ends on one side of 0: difference of upper tails via erfc,
 * so that tail cells keep relative accuracy; straddling 0: difference of erf. */
double orc_mass1d(double a, double b) {
  if (a >= 0.0) return 0.5 * (erfc(a * INV_SQRT2) - erfc(b * INV_SQRT2));
  if (b <= 0.0) return 0.5 * (erfc(-b * INV_SQRT2) - erfc(-a * INV_SQRT2));
  return 0.5 * (erf(b * INV_SQRT2) - erf(a * INV_SQRT2));
}

/* Zero-mean cutting point (Remark after Fig. 1): the x* > 0 where the 1-D
 * normal density with variance var equals gamma.  INFINITY for gamma == 0,
 * -1 when gamma is at or above the peak density (no such point). */
double orc_xstar(double var, double cutoff) {
  if (cutoff <= 0.0) return INFINITY;
  double s = sqrt(var);
  double t = (cutoff * s) * SQRT_2PI;
  if (!(t < 1.0)) return -1.0;
  return s * sqrt(-2.0 * log(t));
}

static int valid(const orc_problem* p) {
  if (p->n < 1 || p->n > ORC_MAX_DIM || p->m < 1 || p->m > ORC_MAX_IN) return 0;
  if (p->noise < 0 || p->noise > 3 || p->window < 0 || p->window > 1 || p->mult < 0 || p->mult > 1) return 0;
  if (p->noise != 0 && (p->window != 0 || p->mult != 0)) return 0;
  for (int i = 0; i < p->n; ++i) {
    if (p->count[i] < 1 || !(p->h[i] > 0)) return 0;
    if (p->noise == 0 && !(p->var[i] > 0)) return 0;
    if ((p->noise == 1 || p->noise == 3) && !(p->nb[i] > p->na[i])) return 0;
    if (p->noise == 3 && !(p->nalpha[i] >= 1.0 && p->nbeta[i] >= 1.0)) return 0;
    if (p->noise == 2 && (!(p->na[i] > 0) || (p->cutoff > 0 && !(p->cutoff < p->na[i])))) return 0;
  }
  for (int k = 0; k < p->m; ++k) if (p->ucount[k] < 1) return 0;
  if (p->p < 0 || p->p > ORC_MAX_IN) return 0;
  for (int l = 0; l < p->p; ++l) if (p->wcount[l] < 1) return 0;
  if (p->horizon < 0 || p->cutoff < 0) return 0;
  if (p->noise == 0 && !p->mult)
    for (int i = 0; i < p->n; ++i) if (orc_xstar(p->var[i], p->cutoff) < 0) return 0;
  switch (p->dyn) {
    case ORC_AFFINE: if (p->n_params != p->n * p->n + p->n * p->m + p->n + p->n * p->p) return 0; break;
    case ORC_UNICYCLE: if (p->n != 3 || p->m != 2 || p->n_params != 1 || p->p != 0) return 0; break;
    case ORC_ROOM: if (p->n_params != 5 || !(p->m == 1 || p->m == p->n) || p->p != 0) return 0; break;
    case ORC_VEHICLE7: if (p->n != 7 || p->m != 2 || p->n_params != 11 || p->p != 0) return 0; break;
    case ORC_ROBOT: if (p->n != 2 || p->m != 2 || p->n_params != 1 || p->p > 1) return 0; break;
    case ORC_USER: if (!p->user_f || p->n_params < 0 || p->n_params > ORC_MAX_PARAMS) return 0; break;
    default: return 0;
  }
  return 1;
}

static double centre(const orc_problem* p, int i, int64_t j) {
  return p->lo[i] + ((double)j + 0.5) * p->h[i];
}

static double edge(const orc_problem* p, int i, int64_t j) {
  return p->lo[i] + (double)j * p->h[i];
}

static double input_value(const orc_problem* p, int k, int64_t j) {
  if (p->ucount[k] == 1) return p->ulo[k];
  double step = (p->uhi[k] - p->ulo[k]) / (double)(p->ucount[k] - 1);
  return p->ulo[k] + (double)j * step;
}

static double dist_value(const orc_problem* p, int l, int64_t j) {
  if (p->wcount[l] == 1) return p->wlo[l];
  double step = (p->whi[l] - p->wlo[l]) / (double)(p->wcount[l] - 1);
  return p->wlo[l] + (double)j * step;
}

/* Disturbance point number w (row-major, last dimension fastest). */
static void dist_point(const orc_problem* p, int64_t w, double* wv) {
  for (int l = p->p - 1; l >= 0; --l) {
    int64_t j = w % p->wcount[l];
    w /= p->wcount[l];
    wv[l] = dist_value(p, l, j);
  }
}

static void state_point(const orc_problem* p, int64_t s, double* x) {
  for (int i = p->n - 1; i >= 0; --i) {
    int64_t j = s % p->count[i];
    s /= p->count[i];
    x[i] = centre(p, i, j);
  }
}

static void input_point(const orc_problem* p, int64_t u, double* uv) {
  for (int k = p->m - 1; k >= 0; --k) {
    int64_t j = u % p->ucount[k];
    u /= p->ucount[k];
    uv[k] = input_value(p, k, j);
  }
}

static double clampd(double v, double a, double b) { return v < a ? a : (v > b ? b : v); }

/* Mean mu = f(x_bar, u_bar, w_bar) with the noise set to 0 (Alg. 1, first
 * step).  Each family's evaluation order is fixed here as written. */
int orc_mean(const orc_problem* p, const double* x, const double* u, const double* w, double* mu) {
  const double* q = p->params;
  const int n = p->n, m = p->m;
  switch (p->dyn) {
    case ORC_AFFINE: {
      /* x+ = A x + B u + c + D w, evaluated as ((A x + c) + B u) + D w,
       * sums left to right (no D term without a disturbance) */
      const double* A = q;
      const double* B = q + n * n;
      const double* c = q + n * n + n * m;
      const double* D = q + n * n + n * m + n;
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s = s + A[i * n + j] * x[j];
        s = s + c[i];
        double t = 0.0;
        for (int k = 0; k < m; ++k) t = t + B[i * m + k] * u[k];
        mu[i] = s + t;
        if (p->p > 0) {
          double d = 0.0;
          for (int l = 0; l < p->p; ++l) d = d + D[i * p->p + l] * w[l];
          mu[i] = mu[i] + d;
        }
      }
      return 0;
    }
    case ORC_UNICYCLE: {
      /* x + tau v cos(theta), y + tau v sin(theta), theta + tau omega */
      double tau = q[0];
      double a = tau * u[0];
      mu[0] = x[0] + a * cos(x[2]);
      mu[1] = x[1] + a * sin(x[2]);
      mu[2] = x[2] + tau * u[1];
      return 0;
    }
    case ORC_ROOM: {
      /* ring of rooms: (1-2a-b-g u) x_i + a (x_{i-1} + x_{i+1}) + b Te + g Th u,
       * evaluated as ((c0 x_i + a (left + right)) + b Te) + u (g (Th - x_i)),
       * c0 = (1 - 2a) - b; one shared heater (m == 1) or one per room. */
      double al = q[0], be = q[1], ga = q[2], Te = q[3], Th = q[4];
      double c0 = (1.0 - 2.0 * al) - be;
      for (int i = 0; i < n; ++i) {
        double left = x[(i + n - 1) % n], right = x[(i + 1) % n];
        double ui = (m == 1) ? u[0] : u[i];
        double s = (c0 * x[i] + al * (left + right)) + be * Te;
        double g = ga * (Th - x[i]);
        mu[i] = s + ui * g;
      }
      return 0;
    }
    case ORC_USER:
      p->user_f(x, u, w, q, mu);
      return 0;
    case ORC_ROBOT: {
      /* the robot of Sec. 7: x1 + tau v1 cos(v2) + w, x2 + tau v1 sin(v2) + w
       * (the printed second row multiplies by v2; read as v1, the speed, as
       * in the first row); without a disturbance w = 0 and no w term. */
      double tau = q[0];
      double a = tau * u[0];
      mu[0] = x[0] + a * cos(u[1]);
      mu[1] = x[1] + a * sin(u[1]);
      if (p->p > 0) {
        mu[0] = mu[0] + w[0];
        mu[1] = mu[1] + w[0];
      }
      return 0;
    }
    case ORC_VEHICLE7: {
      /* single-track model of Sec. 8.4.1 with the printed right-hand sides;
       * the input saturations are clamps to the input box. */
      double tau = q[0], lwb = q[1], mass = q[2], mub = q[3], lf = q[4], lr = q[5];
      double hcg = q[6], Iz = q[7], CSf = q[8], CSr = q[9], g = q[10];
      double x1 = x[0], x2 = x[1], x3 = x[2], x4 = x[3], x5 = x[4], x6 = x[5], x7 = x[6];
      double v1 = clampd(u[0], p->ulo[0], p->uhi[0]);
      double v2 = clampd(u[1], p->ulo[1], p->uhi[1]);
      double f1, f2, f5, f6, f7;
      if (fabs(x4) < 0.1) {
        f1 = x4 * cos(x5);
        f2 = x4 * sin(x5);
        f5 = (x4 / lwb) * tan(x3);
        double c3 = cos(x3);
        f6 = (v2 / lwb) * tan(x3) + (x4 / (lwb * (c3 * c3))) * v1;
        f7 = 0.0;
      } else {
        double Ff = g * lr - v2 * hcg;
        double Fr = g * lf + v2 * hcg;
        f1 = x4 * cos(x5 + x7);
        f2 = x4 * sin(x5 + x7);
        f5 = x6;
        double r64 = x6 / x4;
        f6 = ((mub * mass) / (Iz * (lr + lf))) *
             ((lf * CSf * Ff * x3 + (lr * CSr * Fr - lf * CSf * Ff) * x7) -
              (lf * lf * CSf * Ff + lr * lr * CSr * Fr) * r64);
        f7 = (mub / (x4 * (lr + lf))) *
                 ((CSf * Ff * x3 + (CSr * Fr + CSf * Ff) * x7) - (lf * CSf * Ff - lr * CSr * Fr) * r64) -
             x6;
      }
      mu[0] = x1 + tau * f1;
      mu[1] = x2 + tau * f2;
      mu[2] = x3 + tau * v1;
      mu[3] = x4 + tau * v2;
      mu[4] = x5 + tau * f5;
      mu[5] = x6 + tau * f6;
      mu[6] = x7 + tau * f7;
      return 0;
    }
  }
  return -1;
}

/* Cutting interval of dimension i as offsets [zl, zh] from the mean
 * (Sec. 5.2 for the normal density; Sec. 6.2 for the others: their support,
 * the exponential's cut where its density falls to the cutoff).  Returns 0
 * when nothing is cut (gamma = 0 for normal noise; multiplicative noise). */
static int cut_interval(const orc_problem* p, int i, double* zl, double* zh) {
  switch (p->noise) {
    case 1:
    case 3:
      *zl = p->na[i];
      *zh = p->nb[i];
      return 1;
    case 2:
      *zl = 0.0;
      *zh = (p->cutoff > 0) ? log(p->na[i] / p->cutoff) / p->na[i] : INFINITY;
      return 1;
  }
  if (p->mult || p->cutoff <= 0.0) return 0;
  double xs = orc_xstar(p->var[i], p->cutoff);
  *zl = -xs;
  *zh = xs;
  return 1;
}

/* Cutting region (Sec. 5.2): per dimension, the cells whose centre lies in
 * the closed interval [mu + zl, mu + zh] (the paper's rule), or with the
 * intersect rule the cells whose open interval meets it; every cell is
 * tested. */
int orc_window(const orc_problem* p, const double* mu, int32_t* jlo, int32_t* jhi) {
  int ok = 1;
  for (int i = 0; i < p->n; ++i) {
    double zl = -INFINITY, zh = INFINITY;
    const int cut = cut_interval(p, i, &zl, &zh);
    const int intersect = (p->noise != 0) || p->window == 1;
    int32_t a = -1, b = -2;
    for (int32_t j = 0; j < p->count[i]; ++j) {
      int keep = 1;
      if (cut) {
        if (intersect) keep = (edge(p, i, j + 1) - mu[i] > zl) && (edge(p, i, j) - mu[i] < zh);
        else keep = (centre(p, i, j) - mu[i] >= zl) && (centre(p, i, j) - mu[i] <= zh);
      }
      if (keep) {
        if (a < 0) a = j;
        b = j;
      }
    }
    jlo[i] = a;
    jhi[i] = b;
    if (a < 0) ok = 0;
  }
  return ok;
}

static int in_box(const orc_problem* p, const double* x, const double* lo, const double* hi) {
  for (int i = 0; i < p->n; ++i)
    if (!(x[i] >= lo[i] && x[i] <= hi[i])) return 0;
  return 1;
}

static int label_of(const orc_problem* p, int64_t s) {
  double x[ORC_MAX_DIM];
  state_point(p, s, x);
  if (p->spec == ORC_SAFETY) return in_box(p, x, p->slo, p->shi) ? LBL_FREE : LBL_ZERO;
  if (p->spec == ORC_REACH_AVOID && in_box(p, x, p->alo, p->ahi)) return LBL_ZERO;
  if (in_box(p, x, p->tlo, p->thi)) return LBL_ONE;
  return LBL_FREE;
}

int orc_labels(const orc_problem* p, uint8_t* out) {
  if (!valid(p)) return -1;
  int64_t nx = 1;
  for (int i = 0; i < p->n; ++i) nx *= p->count[i];
  for (int64_t s = 0; s < nx; ++s) out[s] = (uint8_t)label_of(p, s);
  return 0;
}

/* ----------------------------------------------------------- one row (x,u) */

typedef struct {
  const orc_problem* p;
  int64_t nx, nu, nw;
  int64_t stride[ORC_MAX_DIM];
  uint8_t* label;
} ctx_t;

static int ctx_init(ctx_t* C, const orc_problem* p) {
  if (!valid(p)) return -1;
  C->p = p;
  C->nx = 1;
  for (int i = p->n - 1; i >= 0; --i) {
    C->stride[i] = C->nx;
    C->nx *= p->count[i];
  }
  C->nu = 1;
  for (int k = 0; k < p->m; ++k) C->nu *= p->ucount[k];
  C->nw = 1;
  for (int l = 0; l < p->p; ++l) C->nw *= p->wcount[l];
  C->label = (uint8_t*)malloc((size_t)C->nx);
  if (!C->label) return -1;
  for (int64_t s = 0; s < C->nx; ++s) C->label[s] = (uint8_t)label_of(p, s);
  return 0;
}

static void ctx_free(ctx_t* C) { free(C->label); }

/* Beta(al, be) density on [0, 1] (al, be >= 1, so it is bounded). */
static double beta_pdf(double y, double al, double be, double lnorm) {
  if (y <= 0.0 || y >= 1.0) {
    if (y == 0.0 && al == 1.0) return exp(-lnorm) * pow(1.0 - y, be - 1.0);
    if (y == 1.0 && be == 1.0) return exp(-lnorm) * pow(y, al - 1.0);
    return 0.0;
  }
  return exp((al - 1.0) * log(y) + (be - 1.0) * log1p(-y) - lnorm);
}

/* Adaptive Simpson quadrature of the beta density over [a, b] within [0, 1]. */
static double beta_simpson(double a, double b, double fa, double fm, double fb, double whole, double al,
                           double be, double lnorm, int depth) {
  double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
  double flm = beta_pdf(lm, al, be, lnorm), frm = beta_pdf(rm, al, be, lnorm);
  double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
  double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
  double diff = left + right - whole;
  if (depth <= 0 || fabs(diff) <= 1e-16 * 15.0) return left + right + diff / 15.0;
  return beta_simpson(a, m, fa, flm, fm, left, al, be, lnorm, depth - 1) +
         beta_simpson(m, b, fm, frm, fb, right, al, be, lnorm, depth - 1);
}

static double beta_mass(double y0, double y1, double al, double be) {
  if (y0 < 0.0) y0 = 0.0;
  if (y1 > 1.0) y1 = 1.0;
  if (!(y1 > y0)) return 0.0;
  double lnorm = lgamma(al) + lgamma(be) - lgamma(al + be);
  double fa = beta_pdf(y0, al, be, lnorm), fb = beta_pdf(y1, al, be, lnorm);
  double fm = beta_pdf(0.5 * (y0 + y1), al, be, lnorm);
  double whole = (y1 - y0) / 6.0 * (fa + 4.0 * fm + fb);
  return beta_simpson(y0, y1, fa, fm, fb, whole, al, be, lnorm, 48);
}

/* Mass of dimension i's noise between offsets ta < tb from the mean: the
 * integral of its density (Alg. 1), in closed form except for the beta
 * density, which is integrated numerically. */
double orc_noise_mass(const orc_problem* p, int i, double xi, double ta, double tb) {
  switch (p->noise) {
    case 1: {
      double w = p->nb[i] - p->na[i];
      double fa = clampd((ta - p->na[i]) / w, 0.0, 1.0), fb = clampd((tb - p->na[i]) / w, 0.0, 1.0);
      return fb - fa;
    }
    case 2: {
      double sa = ta <= 0.0 ? 1.0 : exp(-p->na[i] * ta);
      double sb = tb <= 0.0 ? 1.0 : exp(-p->na[i] * tb);
      return sa - sb;
    }
    case 3: {
      double w = p->nb[i] - p->na[i];
      return beta_mass((ta - p->na[i]) / w, (tb - p->na[i]) / w, p->nalpha[i], p->nbeta[i]);
    }
  }
  double s = sqrt(p->var[i]);
  if (p->mult) {
    s = s * fabs(xi);
    if (s == 0.0) return (ta <= 0.0 && 0.0 < tb) ? 1.0 : 0.0; /* all mass at the mean */
  }
  return orc_mass1d(ta / s, tb / s);
}

/* Probability of one target cell (multi-index j) for mean mu from state x:
 * the product of the per-dimension masses of the cell's edges (Alg. 1
 * integral with independent noise components). */
static double cell_prob(const ctx_t* C, const double* x, const double* mu, const int32_t* j) {
  const orc_problem* p = C->p;
  double t = 1.0;
  for (int i = 0; i < p->n; ++i)
    t *= orc_noise_mass(p, i, x[i], edge(p, i, j[i]) - mu[i], edge(p, i, j[i] + 1) - mu[i]);
  return t;
}

/* V_in(x,u) of Alg. 4: sum over the cutting region of T * V_{k+1}, plus T0
 * for reach / reach-avoid (mass into T\A; post-states in T u A are zeroed
 * in T).  Vnext == NULL means the terminal vector. */
static double row_value(const ctx_t* C, const double* x, const double* mu, const double* Vnext) {
  const orc_problem* p = C->p;
  int32_t lo[ORC_MAX_DIM], hi[ORC_MAX_DIM], j[ORC_MAX_DIM];
  if (!orc_window(p, mu, lo, hi)) return 0.0;
  const int safety = (p->spec == ORC_SAFETY);
  double q = 0.0, t0 = 0.0;
  for (int i = 0; i < p->n; ++i) j[i] = lo[i];
  for (;;) {
    int64_t cell = 0;
    for (int i = 0; i < p->n; ++i) cell += (int64_t)j[i] * C->stride[i];
    double t = cell_prob(C, x, mu, j);
    int lbl = C->label[cell];
    if (safety) {
      /* V_{T_d+1} = 1 on S, 0 outside; V_k = 0 outside S */
      double v = (lbl == LBL_FREE) ? (Vnext ? Vnext[cell] : 1.0) : 0.0;
      q += t * v;
    } else {
      if (lbl == LBL_ONE) t0 += t;
      else if (lbl == LBL_FREE) q += t * (Vnext ? Vnext[cell] : 0.0);
    }
    int i = p->n - 1;
    while (i >= 0) {
      if (++j[i] <= hi[i]) break;
      j[i] = lo[i];
      --i;
    }
    if (i < 0) break;
  }
  return safety ? q : q + t0;
}

/* Tail of one row: grid mass minus kept-window mass (both as products of
 * 1-D masses, exact for independent noise components). */
static double row_tail(const ctx_t* C, const double* x, const double* mu) {
  const orc_problem* p = C->p;
  int32_t lo[ORC_MAX_DIM], hi[ORC_MAX_DIM];
  int ok = orc_window(p, mu, lo, hi);
  double grid = 1.0, win = 1.0;
  for (int i = 0; i < p->n; ++i) {
    grid *= orc_noise_mass(p, i, x[i], edge(p, i, 0) - mu[i], edge(p, i, p->count[i]) - mu[i]);
    if (ok) win *= orc_noise_mass(p, i, x[i], edge(p, i, lo[i]) - mu[i], edge(p, i, hi[i] + 1) - mu[i]);
  }
  if (!ok) win = 0.0;
  return grid - win;
}

/* Bellman update of one state: max over inputs of the min over
 * disturbances of V_in, lowest maximising input. */
static void state_update(const ctx_t* C, const double* Vnext, int64_t s, double* v_out,
                         int16_t* pol_out, double* gap_out, double* tail_out) {
  const orc_problem* p = C->p;
  int lbl = C->label[s];
  if (lbl != LBL_FREE) {
    *v_out = (lbl == LBL_ONE) ? 1.0 : 0.0;
    if (pol_out) *pol_out = -1;
    if (gap_out) *gap_out = 0.0;
    if (tail_out) *tail_out = 0.0;
    return;
  }
  double x[ORC_MAX_DIM], uv[ORC_MAX_IN], wv[ORC_MAX_IN], mu[ORC_MAX_DIM];
  state_point(p, s, x);
  double best = -1.0, second = -1.0, tmax = 0.0;
  int64_t arg = 0;
  for (int64_t u = 0; u < C->nu; ++u) {
    input_point(p, u, uv);
    double q = INFINITY;
    for (int64_t w = 0; w < C->nw; ++w) {
      dist_point(p, w, wv);
      orc_mean(p, x, uv, wv, mu);
      double qw = row_value(C, x, mu, Vnext);
      if (qw < q) q = qw;
      if (tail_out) {
        double t = row_tail(C, x, mu);
        if (t > tmax) tmax = t;
      }
    }
    if (q > best) {
      second = best;
      best = q;
      arg = u;
    } else if (q > second) {
      second = q;
    }
  }
  *v_out = best;
  if (pol_out) *pol_out = (int16_t)arg;
  if (gap_out) *gap_out = (C->nu > 1) ? best - second : INFINITY;
  if (tail_out) *tail_out = tmax;
}

/* ------------------------------------------------------------- public API */

int orc_solve(const orc_problem* p, int threads, double* V_out, int16_t* policy_out,
              double* gap_out, double* max_tail_out) {
  ctx_t C;
  if (ctx_init(&C, p) != 0) return -1;
  if (threads <= 0) threads = 0;
  const int64_t nx = C.nx;
  double* Vn = (double*)malloc((size_t)nx * sizeof(double));
  double* Vk = (double*)malloc((size_t)nx * sizeof(double));
  double* tl = max_tail_out ? (double*)calloc((size_t)nx, sizeof(double)) : NULL;
  if (!Vn || !Vk || (max_tail_out && !tl)) {
    free(Vn); free(Vk); free(tl); ctx_free(&C);
    return -1;
  }
  /* terminal vector in the paper's representation */
  for (int64_t s = 0; s < nx; ++s) {
    if (p->spec == ORC_SAFETY) Vn[s] = (C.label[s] == LBL_FREE) ? 1.0 : 0.0;
    else Vn[s] = 0.0;
  }
  for (int k = p->horizon; k >= 1; --k) {
    int16_t* pol = policy_out ? policy_out + (int64_t)(k - 1) * nx : NULL;
    double* gap = gap_out ? gap_out + (int64_t)(k - 1) * nx : NULL;
    const int want_tail = (tl && k == p->horizon);
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads > 0 ? threads : omp_get_max_threads())
    for (int64_t s = 0; s < nx; ++s) {
      double v;
      state_update(&C, Vn, s, &v, pol ? pol + s : NULL, gap ? gap + s : NULL,
                   want_tail ? tl + s : NULL);
      /* internal representation: T u A entries of V are never read */
      Vk[s] = (C.label[s] == LBL_FREE) ? v : 0.0;
    }
    double* t = Vn; Vn = Vk; Vk = t;
  }
  /* readout (V at k = 1): 1 on T\A, 0 on A / outside S */
  for (int64_t s = 0; s < nx; ++s) {
    int lbl = C.label[s];
    V_out[s] = (lbl == LBL_FREE) ? Vn[s] : (lbl == LBL_ONE ? 1.0 : 0.0);
  }
  if (max_tail_out) {
    double m = 0.0;
    if (p->horizon == 0) {
      /* no sweep ran; compute the tails directly */
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads > 0 ? threads : omp_get_max_threads())
      for (int64_t s = 0; s < nx; ++s) {
        double v;
        state_update(&C, NULL, s, &v, NULL, NULL, tl + s);
      }
    }
    for (int64_t s = 0; s < nx; ++s) if (tl[s] > m) m = tl[s];
    *max_tail_out = m;
  }
  free(Vn); free(Vk); free(tl); ctx_free(&C);
  return 0;
}

int orc_step(const orc_problem* p, const double* V_next, const int64_t* states, int64_t n_states,
             int threads, double* V_out, int16_t* policy_out, double* gap_out) {
  ctx_t C;
  if (ctx_init(&C, p) != 0) return -1;
  for (int64_t r = 0; r < n_states; ++r)
    if (states[r] < 0 || states[r] >= C.nx) { ctx_free(&C); return -1; }
  double* Vn = NULL;
  if (!V_next && p->spec == ORC_SAFETY) {
    Vn = (double*)malloc((size_t)C.nx * sizeof(double));
    if (!Vn) { ctx_free(&C); return -1; }
    for (int64_t s = 0; s < C.nx; ++s) Vn[s] = (C.label[s] == LBL_FREE) ? 1.0 : 0.0;
  }
  const double* src = V_next ? V_next : Vn;
#pragma omp parallel for schedule(dynamic, 16) num_threads(threads > 0 ? threads : omp_get_max_threads())
  for (int64_t r = 0; r < n_states; ++r) {
    state_update(&C, src, states[r], V_out + r, policy_out ? policy_out + r : NULL,
                 gap_out ? gap_out + r : NULL, NULL);
  }
  free(Vn);
  ctx_free(&C);
  return 0;
}

int orc_row_mass(const orc_problem* p, int64_t state, int64_t input, double* sum_out,
                 double* tail_out) {
  ctx_t C;
  if (ctx_init(&C, p) != 0) return -1;
  if (state < 0 || state >= C.nx || input < 0 || input >= C.nu * C.nw) { ctx_free(&C); return -1; }
  double x[ORC_MAX_DIM], uv[ORC_MAX_IN], wv[ORC_MAX_IN], mu[ORC_MAX_DIM];
  int32_t lo[ORC_MAX_DIM], hi[ORC_MAX_DIM], j[ORC_MAX_DIM];
  state_point(p, state, x);
  input_point(p, input / C.nw, uv);
  dist_point(p, input % C.nw, wv);
  orc_mean(p, x, uv, wv, mu);
  double sum = 0.0;
  if (orc_window(p, mu, lo, hi)) {
    for (int i = 0; i < p->n; ++i) j[i] = lo[i];
    for (;;) {
      sum += cell_prob(&C, x, mu, j);
      int i = p->n - 1;
      while (i >= 0) {
        if (++j[i] <= hi[i]) break;
        j[i] = lo[i];
        --i;
      }
      if (i < 0) break;
    }
  }
  *sum_out = sum;
  *tail_out = row_tail(&C, x, mu);
  ctx_free(&C);
  return 0;
}

int orc_row_dense(const orc_problem* p, int64_t state, int64_t input, double* row_out) {
  ctx_t C;
  if (ctx_init(&C, p) != 0) return -1;
  if (state < 0 || state >= C.nx || input < 0 || input >= C.nu * C.nw) { ctx_free(&C); return -1; }
  double x[ORC_MAX_DIM], uv[ORC_MAX_IN], wv[ORC_MAX_IN], mu[ORC_MAX_DIM];
  int32_t lo[ORC_MAX_DIM], hi[ORC_MAX_DIM], j[ORC_MAX_DIM];
  state_point(p, state, x);
  input_point(p, input / C.nw, uv);
  dist_point(p, input % C.nw, wv);
  orc_mean(p, x, uv, wv, mu);
  int ok = orc_window(p, mu, lo, hi);
  for (int64_t c = 0; c < C.nx; ++c) {
    int64_t r = c;
    int inside = ok;
    for (int i = p->n - 1; i >= 0; --i) {
      j[i] = (int32_t)(r % p->count[i]);
      r /= p->count[i];
      if (j[i] < lo[i] || j[i] > hi[i]) inside = 0;
    }
    row_out[c] = inside ? cell_prob(&C, x, mu, j) : 0.0;
  }
  ctx_free(&C);
  return 0;
}
