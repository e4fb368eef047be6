// amy_host.cpp -- C ABI: validation, planning, workspace layout and the
// single-problem solve driver (one HIP stream, no allocation).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "../../include/amytiss.h"
#include "amy_host.hpp"
#include "amy_kernels.hpp"
#include "amy_tune.hpp"

static thread_local std::string g_err;

amy_status amy_fail(amy_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

amy_status amy_hip_fail(hipError_t e, const char* what) {
  return amy_fail(AMY_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char* amy_last_error(void) { return g_err.c_str(); }
extern "C" const char* amy_version(void) { return "amytiss-hip 0.1 (gfx950)"; }

// ------------------------------------------------------- quantisation

// The paper's quantisation convention: points lb + j q, both ends of
// [lb, ub] included; as cells lo = lb - q/2, h = q.
static amy_status quant_count(const double* lb, const double* ub, const double* q, int k, int32_t* count) {
  if (!isfinite(lb[k]) || !isfinite(ub[k]) || !isfinite(q[k]))
    return amy_fail(AMY_E_INVALID, "quantisation of dimension %d not finite", k);
  if (!(q[k] > 0)) return amy_fail(AMY_E_INVALID, "quantisation parameter q[%d] <= 0", k);
  if (ub[k] < lb[k]) return amy_fail(AMY_E_INVALID, "ub[%d] < lb[%d]", k, k);
  const double c = floor((ub[k] - lb[k]) / q[k] + 1e-9) + 1.0;
  if (c > 2147483647.0) return amy_fail(AMY_E_INVALID, "dimension %d has more than 2^31 - 1 points", k);
  *count = (int32_t)c;
  return AMY_OK;
}

extern "C" amy_status amy_grid_from_quantization(int32_t n, const double* lb, const double* ub, const double* q,
                                                 amy_grid* out) {
  if (n < 1 || n > AMY_MAX_DIM) return amy_fail(AMY_E_INVALID, "n=%d not in [1,%d]", n, AMY_MAX_DIM);
  if (!lb || !ub || !q || !out) return amy_fail(AMY_E_INVALID, "NULL argument");
  amy_grid g;
  memset(&g, 0, sizeof g);
  g.n = n;
  for (int i = 0; i < n; ++i) {
    const amy_status st = quant_count(lb, ub, q, i, &g.count[i]);
    if (st != AMY_OK) return st;
    g.lo[i] = lb[i] - q[i] / 2.0;
    g.h[i] = q[i];
  }
  *out = g;
  return AMY_OK;
}

extern "C" amy_status amy_inputs_from_quantization(int32_t m, const double* lb, const double* ub, const double* q,
                                                   amy_inputs* out) {
  if (m < 1 || m > AMY_MAX_IN) return amy_fail(AMY_E_INVALID, "m=%d not in [1,%d]", m, AMY_MAX_IN);
  if (!lb || !ub || !q || !out) return amy_fail(AMY_E_INVALID, "NULL argument");
  amy_inputs u;
  memset(&u, 0, sizeof u);
  u.m = m;
  for (int k = 0; k < m; ++k) {
    const amy_status st = quant_count(lb, ub, q, k, &u.count[k]);
    if (st != AMY_OK) return st;
    u.lo[k] = lb[k];
    u.hi[k] = lb[k] + (double)(u.count[k] - 1) * q[k];
  }
  *out = u;
  return AMY_OK;
}

// ---------------------------------------------------------------- planning

static const double SQRT_2PI = 2.5066282746310002;

// Cutting half-width x* of Sec. 5.2: the 1-D normal density with variance
// var equals the cutoff gamma at +-x*.
static double xstar_of(double var, double cutoff) {
  const double s = sqrt(var);
  const double t = (cutoff * s) * SQRT_2PI;
  return s * sqrt(-2.0 * log(t));
}

static int expected_params(const amy_problem* p) {
  const int n = p->grid.n, m = p->inputs.m;
  switch (p->dyn.kind) {
    case AMY_DYN_AFFINE: return n * n + n * m + n + n * p->dist.p;
    case AMY_DYN_UNICYCLE: return 1;
    case AMY_DYN_ROOM: return 5;
    case AMY_DYN_VEHICLE7: return 11;
    case AMY_DYN_ROBOT: return 1;
    case AMY_DYN_USER: return (p->dyn.n_params >= 0 && p->dyn.n_params <= AMY_MAX_PARAMS) ? p->dyn.n_params : -1;
  }
  return -1;
}

// Exponential noise: the support [0, inf) cut where the density rate e^{-rate t}
// falls to the cutoff; INFINITY without a cut.
static double exp_cut(double rate, double cutoff) {
  if (cutoff <= 0.0) return INFINITY;
  return log(rate / cutoff) / rate;
}

static amy_status validate_noise(const amy_problem* p) {
  const amy_noise& z = p->noise;
  const int n = p->grid.n;
  if (z.kind < AMY_NOISE_NORMAL || z.kind > AMY_NOISE_BETA) return amy_fail(AMY_E_INVALID, "bad noise kind %d", z.kind);
  if (z.window != AMY_WINDOW_CENTRE && z.window != AMY_WINDOW_INTERSECT)
    return amy_fail(AMY_E_INVALID, "bad window rule %d", z.window);
  if (z.multiplicative != 0 && z.multiplicative != 1) return amy_fail(AMY_E_INVALID, "multiplicative must be 0 or 1");
  if (z.kind != AMY_NOISE_NORMAL && (z.multiplicative || z.window != AMY_WINDOW_CENTRE))
    return amy_fail(AMY_E_INVALID, "window rule and multiplicative noise apply to normal noise only");
  for (int i = 0; i < n; ++i) {
    switch (z.kind) {
      case AMY_NOISE_UNIFORM:
      case AMY_NOISE_BETA:
        if (!isfinite(z.a[i]) || !isfinite(z.b[i]) || !(z.b[i] > z.a[i]))
          return amy_fail(AMY_E_INVALID, "noise support [a, b] of dimension %d is empty or not finite", i);
        if (z.kind == AMY_NOISE_BETA && (!(z.alpha[i] >= 1.0) || !(z.beta[i] >= 1.0) || !isfinite(z.alpha[i]) ||
                                         !isfinite(z.beta[i]) || z.alpha[i] > 1e6 || z.beta[i] > 1e6))
          return amy_fail(AMY_E_INVALID, "beta shapes of dimension %d must lie in [1, 1e6]", i);
        break;
      case AMY_NOISE_EXPONENTIAL:
        if (!(z.a[i] > 0.0) || !isfinite(z.a[i])) return amy_fail(AMY_E_INVALID, "exponential rate a[%d] <= 0", i);
        if (p->cutoff > 0.0 && !(p->cutoff < z.a[i]))
          return amy_fail(AMY_E_INVALID, "cutoff %g is at or above the peak density of dimension %d", p->cutoff, i);
        break;
    }
  }
  return AMY_OK;
}

amy_status amy_validate(const amy_problem* p) {
  if (!p) return amy_fail(AMY_E_INVALID, "problem is NULL");
  const int n = p->grid.n, m = p->inputs.m;
  if (n < 1 || n > AMY_MAX_DIM) return amy_fail(AMY_E_INVALID, "grid.n=%d not in [1,%d]", n, AMY_MAX_DIM);
  if (m < 1 || m > AMY_MAX_IN) return amy_fail(AMY_E_INVALID, "inputs.m=%d not in [1,%d]", m, AMY_MAX_IN);
  double nx = 1;
  for (int i = 0; i < n; ++i) {
    if (p->grid.count[i] < 1) return amy_fail(AMY_E_INVALID, "grid.count[%d]=%d < 1", i, p->grid.count[i]);
    if (!(p->grid.h[i] > 0) || !isfinite(p->grid.h[i])) return amy_fail(AMY_E_INVALID, "grid.h[%d] <= 0", i);
    if (!isfinite(p->grid.lo[i])) return amy_fail(AMY_E_INVALID, "grid.lo[%d] not finite", i);
    if (p->noise.kind == AMY_NOISE_NORMAL && (!(p->noise_var[i] > 0) || !isfinite(p->noise_var[i])))
      return amy_fail(AMY_E_INVALID, "noise_var[%d] <= 0", i);
    nx *= p->grid.count[i];
  }
  if (nx >= 2147483647.0) return amy_fail(AMY_E_UNSUPPORTED, "n_x=%.0f >= 2^31 states", nx);
  double nu = 1;
  for (int k = 0; k < m; ++k) {
    if (p->inputs.count[k] < 1) return amy_fail(AMY_E_INVALID, "inputs.count[%d] < 1", k);
    if (!isfinite(p->inputs.lo[k]) || !isfinite(p->inputs.hi[k]))
      return amy_fail(AMY_E_INVALID, "inputs bounds of dim %d not finite", k);
    if (p->inputs.count[k] > 1 && !(p->inputs.hi[k] >= p->inputs.lo[k]))
      return amy_fail(AMY_E_INVALID, "inputs.hi[%d] < inputs.lo[%d]", k, k);
    nu *= p->inputs.count[k];
  }
  if (nu > 32767) return amy_fail(AMY_E_UNSUPPORTED, "n_u=%.0f > 32767 (int16 policy)", nu);
  const int pd = p->dist.p;
  if (pd < 0 || m + pd > AMY_MAX_IN)
    return amy_fail(AMY_E_INVALID, "dist.p=%d: inputs plus disturbance dimensions exceed %d", pd, AMY_MAX_IN);
  double nw = 1;
  for (int l = 0; l < pd; ++l) {
    if (p->dist.count[l] < 1) return amy_fail(AMY_E_INVALID, "dist.count[%d] < 1", l);
    if (!isfinite(p->dist.lo[l]) || !isfinite(p->dist.hi[l]))
      return amy_fail(AMY_E_INVALID, "disturbance bounds of dim %d not finite", l);
    if (p->dist.count[l] > 1 && !(p->dist.hi[l] >= p->dist.lo[l]))
      return amy_fail(AMY_E_INVALID, "dist.hi[%d] < dist.lo[%d]", l, l);
    nw *= p->dist.count[l];
  }
  if (nu * nw > 1e6) return amy_fail(AMY_E_UNSUPPORTED, "%.0f (input, disturbance) rows per state > 1e6", nu * nw);
  if (pd > 0 && p->dyn.kind != AMY_DYN_AFFINE && p->dyn.kind != AMY_DYN_ROBOT && p->dyn.kind != AMY_DYN_USER)
    return amy_fail(AMY_E_INVALID, "dynamics kind %d takes no disturbance", p->dyn.kind);
  {
    const amy_status sn = validate_noise(p);
    if (sn != AMY_OK) return sn;
  }
  if (!(p->cutoff >= 0) || !isfinite(p->cutoff)) return amy_fail(AMY_E_INVALID, "cutoff < 0");
  if (p->cutoff > 0 && p->noise.kind == AMY_NOISE_NORMAL && !p->noise.multiplicative) {
    for (int i = 0; i < n; ++i) {
      const double t = (p->cutoff * sqrt(p->noise_var[i])) * SQRT_2PI;
      if (!(t < 1.0))
        return amy_fail(AMY_E_INVALID, "cutoff %g is at or above the peak density of dimension %d",
                        p->cutoff, i);
    }
  }
  if (p->horizon < 0) return amy_fail(AMY_E_INVALID, "horizon < 0");
  if (p->spec < AMY_SAFETY || p->spec > AMY_REACH_AVOID) return amy_fail(AMY_E_INVALID, "bad spec");
  if (p->mode < AMY_MODE_AUTO || p->mode > AMY_MODE_OTF) return amy_fail(AMY_E_INVALID, "bad mode");
  if (p->precision != AMY_FP64 && p->precision != AMY_FP32) return amy_fail(AMY_E_INVALID, "bad precision");
  if (p->variant < AMY_VARIANT_AUTO || p->variant > AMY_VARIANT_INPUTS) return amy_fail(AMY_E_INVALID, "bad variant");
  const int ep = expected_params(p);
  if (ep < 0) return amy_fail(AMY_E_INVALID, "bad dynamics kind %d", p->dyn.kind);
  if (p->dyn.kind == AMY_DYN_UNICYCLE && (n != 3 || m != 2))
    return amy_fail(AMY_E_INVALID, "unicycle needs n=3, m=2");
  if (p->dyn.kind == AMY_DYN_VEHICLE7 && (n != 7 || m != 2))
    return amy_fail(AMY_E_INVALID, "vehicle7 needs n=7, m=2");
  if (p->dyn.kind == AMY_DYN_ROOM && !(m == 1 || m == n))
    return amy_fail(AMY_E_INVALID, "room needs m=1 (shared heater) or m=n");
  if (p->dyn.kind == AMY_DYN_ROBOT && (n != 2 || m != 2 || pd > 1))
    return amy_fail(AMY_E_INVALID, "robot needs n=2, m=2 and at most one disturbance dimension");
  if (p->dyn.n_params != ep)
    return amy_fail(AMY_E_INVALID, "dynamics needs %d params, got %d", ep, p->dyn.n_params);
  for (int k = 0; k < p->dyn.n_params; ++k)
    if (!isfinite(p->dyn.params[k])) return amy_fail(AMY_E_INVALID, "param %d not finite", k);
  return AMY_OK;
}

// Input-walk digits each state dimension's mean depends on (bit k = digit
// k: the inputs, then the disturbance dimensions), from the structure of
// each dynamics family.
static uint32_t dep_mask(const amy_problem* p, int i) {
  const int n = p->grid.n, m = p->inputs.m, pd = p->dist.p;
  uint32_t all = (1u << (m + pd)) - 1u;
  switch (p->dyn.kind) {
    case AMY_DYN_AFFINE: {
      uint32_t d = 0;
      for (int k = 0; k < m; ++k)
        if (p->dyn.params[n * n + i * m + k] != 0.0) d |= 1u << k;
      for (int l = 0; l < pd; ++l)
        if (p->dyn.params[n * n + n * m + n + i * pd + l] != 0.0) d |= 1u << (m + l);
      return d;
    }
    case AMY_DYN_ROBOT: return all;
    case AMY_DYN_USER: return all;
    case AMY_DYN_UNICYCLE: return i < 2 ? 1u : 2u;  // x, y: speed; theta: turn rate
    case AMY_DYN_ROOM: return m == 1 ? 1u : (1u << i);
    case AMY_DYN_VEHICLE7: {
      // mu_3 <- v1; mu_4, mu_7 <- v2; mu_6 <- v1, v2 (either branch); others none
      static const uint32_t d[7] = {0u, 0u, 1u, 2u, 0u, 3u, 2u};
      return d[i];
    }
  }
  return all;
}

static const int LDS_BUDGET = 64 * 1024;  // bytes of dynamic LDS per 64-lane block

// State coordinates the mean of dimension i reads (besides the inputs), as
// the dynamics families are written; 0 when more than 4 or not known.
static int memo_ctx(const amy_problem* p, int i, int* ctx) {
  const int n = p->grid.n;
  int c = 0;
  auto add = [&](int d) {
    for (int k = 0; k < c; ++k)
      if (ctx[k] == d) return;
    if (c < 4) ctx[c] = d;
    ++c;
  };
  switch (p->dyn.kind) {
    case AMY_DYN_AFFINE:
      for (int j = 0; j < n; ++j)
        if (p->dyn.params[i * n + j] != 0.0) add(j);
      break;
    case AMY_DYN_UNICYCLE: add(i); if (i < 2) add(2); break;
    case AMY_DYN_ROOM: add((i + n - 1) % n); add(i); add((i + 1) % n); break;
    case AMY_DYN_VEHICLE7: {
      // x, y: speed, heading, slip angle; steering, speed: themselves;
      // heading, yaw rate, slip angle: steering, speed, yaw rate, slip angle
      static const int d[7][4] = {{0, 3, 4, 6}, {1, 3, 4, 6}, {2, -1, -1, -1}, {3, -1, -1, -1},
                                  {2, 3, 4, 5}, {2, 3, 5, 6}, {2, 3, 5, 6}};
      for (int k = 0; k < 4; ++k)
        if (d[i][k] >= 0) add(d[i][k]);
      break;
    }
    default: return 0;
  }
  if (c == 0) add(i);
  return c <= 4 ? c : 0;
}

static const int64_t MEMO_BUDGET = 1 << 21;  // entries of memoised tables per solve

// Memoised tables of a compiled-shape plan: false if some dimension's
// context is unknown or the entries exceed the budget.
static bool plan_memo(const amy_problem* p, DevProblem& D) {
  int64_t off = 0;
  for (int i = 0; i < D.n; ++i) {
    if (D.L[i] > AMY_TABLE_SLOTS) return false;  // an entry holds at most that many masses
    int ctx[4];
    const int c = memo_ctx(p, i, ctx);
    if (c <= 0) return false;
    int64_t cells = 1;
    for (int k = c - 1; k >= 0; --k) {
      D.mmult[i][k] = (int32_t)cells;
      cells *= D.count[ctx[k]];
    }
    D.mctx_n[i] = c;
    for (int k = 0; k < 4; ++k) D.mctx[i][k] = k < c ? ctx[k] : 0;
    D.rel_off[i] = (int32_t)off;
    off += cells * D.rcount[i];
    if (off > MEMO_BUDGET) return false;
  }
  D.rel_entries = (int32_t)off;
  return true;
}

// Which dimensions get all their tables built once per state (the others
// are rebuilt in the input loop when their mean changes), and the LDS layout.
// no_cache: none are (the INPUTS variant, whose lanes walk different inputs).
static amy_status plan_tables(const amy_problem* p, Plan* pl, bool no_cache = false) {
  DevProblem& D = pl->dev;
  const int n = D.n, m = D.nd;  // digits of the input walk (inputs, then disturbance)
  const int msz = pl->f64 ? 8 : 4;
  int runs[AMY_MAX_DIM], C[AMY_MAX_DIM];
  uint32_t dep[AMY_MAX_DIM];
  for (int i = 0; i < n; ++i) {
    dep[i] = dep_mask(p, i);
    C[i] = 1;
    int kmax = -1;
    for (int k = 0; k < m; ++k)
      if (dep[i] >> k & 1u) {
        C[i] *= D.ucount[k];
        kmax = k;
      }
    // consecutive-input runs of an unchanged mean in the natural input order
    runs[i] = 1;
    for (int k = 0; k <= kmax; ++k) runs[i] *= D.ucount[k];
    D.ccount[i] = 0;
  }
  auto bytes = [&](bool tail) {
    int64_t ent = 0, slots = 0;
    for (int i = 0; i < n; ++i) {
      ent += (D.ccount[i] > 0) ? (int64_t)D.ccount[i] * D.L[i] : D.L[i];
      if (D.ccount[i] > 0) slots += D.ccount[i];
    }
    // regions plus their alignment padding (at most one table row + 32 B)
    int64_t b = ent * msz * 64 + slots * 4 * 64 + msz * 64 + 32;
    if (tail) b += slots * 2 * 8 * 64;
    return b;
  };
  if (bytes(true) > LDS_BUDGET)
    return amy_fail(AMY_E_UNSUPPORTED, "window tables need %lld B of LDS per 64 lanes (> %d)",
                    (long long)bytes(true), LDS_BUDGET);
  // greedy: cache the dimension saving the most edge evaluations per byte
  for (; !no_cache;) {
    int best = -1;
    double best_gain = 0.0;
    for (int i = 0; i < n; ++i) {
      if (D.ccount[i] > 0 || C[i] >= runs[i]) continue;
      D.ccount[i] = C[i];
      const int64_t b = bytes(true);
      D.ccount[i] = 0;
      if (b > LDS_BUDGET) continue;
      const double gain = (double)(runs[i] - C[i]) * (D.L[i] + 1) / (double)(C[i] * D.L[i] + 1);
      if (gain > best_gain) {
        best_gain = gain;
        best = i;
      }
    }
    if (best < 0) break;
    D.ccount[best] = C[best];
  }
  // LDS layout of a 64-lane block (each region [entry][lane]):
  //   cached tables | cached origins | uncached tables | FP64 tail masses
  // The compiled-shape sweep keeps uncached tables in registers and
  // allocates only the first two regions (plus the last on the tail pass).
  int64_t ent_c = 0, ent_u = 0, slots = 0;
  for (int i = 0; i < n; ++i) {
    if (D.ccount[i] > 0) {
      ent_c += (int64_t)D.ccount[i] * D.L[i];
      slots += D.ccount[i];
    } else {
      ent_u += D.L[i];
    }
  }
  const int64_t row = (int64_t)msz * 64;   // bytes per table entry across the block
  D.lds_int_off = (int32_t)(((ent_c * row + 15) / 16) * 16);
  const int64_t unc_off = D.lds_int_off + ((slots * 4 * 64 + 15) / 16) * 16;
  const int64_t unc_entry0 = (unc_off + row - 1) / row;
  D.lds_tail_off = (int32_t)((((unc_entry0 + ent_u) * row) + 15) / 16 * 16);
  D.lds_bytes = D.lds_tail_off;
  D.lds_bytes_tail = D.lds_tail_off + (int32_t)(slots * 2 * 8 * 64);
  D.lds_bytes_fixed = (int32_t)unc_off;
  int64_t ec = 0, eu = unc_entry0, sl = 0;
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < AMY_MAXI; ++k) D.dep_mult[i][k] = 0;
    D.ooff[i] = (int32_t)sl;
    if (D.ccount[i] > 0) {
      D.toff[i] = (int32_t)ec;
      ec += (int64_t)D.ccount[i] * D.L[i];
      sl += D.ccount[i];
      int mult = 1;
      for (int k = m - 1; k >= 0; --k)
        if (dep[i] >> k & 1u) {
          D.dep_mult[i][k] = mult;
          mult *= D.ucount[k];
        }
    } else {
      D.toff[i] = (int32_t)eu;
      eu += D.L[i];
    }
  }
  for (int i = 0; i < n; ++i) {
    D.rcount[i] = C[i];
    int mult = 1;
    for (int k = m - 1; k >= 0; --k) {
      D.rmult[i][k] = 0;
      if (dep[i] >> k & 1u) {
        D.rmult[i][k] = mult;
        mult *= D.ucount[k];
      }
    }
    for (int k = m; k < AMY_MAXI; ++k) D.rmult[i][k] = 0;
  }
  if (D.lds_bytes_tail > LDS_BUDGET)
    return amy_fail(AMY_E_UNSUPPORTED, "window tables need %d B of LDS per 64 lanes (> %d)", D.lds_bytes_tail,
                    LDS_BUDGET);
  return AMY_OK;
}

void amy_make_plan(const amy_problem* p, Plan* pl) {
  DevProblem& D = pl->dev;
  memset(&D, 0, sizeof D);
  const int n = p->grid.n, m = p->inputs.m;
  D.n = n;
  D.m = m;
  D.kind = p->dyn.kind;
  D.spec = p->spec;
  const amy_noise& nz = p->noise;
  D.noise = nz.kind;
  D.wrule = (nz.kind == AMY_NOISE_NORMAL) ? nz.window : AMY_WINDOW_INTERSECT;
  D.mult = nz.multiplicative;
  // multiplicative noise disables the cut (Sec. 6.2); bounded supports are
  // cut by their support whatever gamma is
  D.nocut = (nz.kind == AMY_NOISE_NORMAL && (p->cutoff == 0.0 || nz.multiplicative));
  int64_t nx = 1;
  for (int i = n - 1; i >= 0; --i) {
    D.stride[i] = nx;
    nx *= p->grid.count[i];
  }
  D.n_x = (int32_t)nx;
  int64_t W = 1;
  for (int i = 0; i < n; ++i) {
    D.count[i] = p->grid.count[i];
    D.lo[i] = p->grid.lo[i];
    D.h[i] = p->grid.h[i];
    D.inv_h[i] = 1.0 / p->grid.h[i];
    // standardised edge coordinate z = (edge - mu) inv_sigma and the cutting
    // interval [mu + zl, mu + zh] of each noise model
    double zl = -INFINITY, zh = INFINITY;
    switch (nz.kind) {
      case AMY_NOISE_UNIFORM:
      case AMY_NOISE_BETA:
        D.inv_sigma[i] = 1.0 / (nz.b[i] - nz.a[i]);
        D.zoff[i] = nz.a[i] * D.inv_sigma[i];
        D.balpha[i] = nz.alpha[i];
        D.bbeta[i] = nz.beta[i];
        zl = nz.a[i];
        zh = nz.b[i];
        break;
      case AMY_NOISE_EXPONENTIAL:
        D.inv_sigma[i] = nz.a[i];
        zl = 0.0;
        zh = exp_cut(nz.a[i], p->cutoff);
        break;
      default: {
        const double sigma = sqrt(p->noise_var[i]);
        D.inv_sigma[i] = 1.0 / sigma;
        if (!D.nocut) {
          const double xs = xstar_of(p->noise_var[i], p->cutoff);
          zl = -xs;
          zh = xs;
        }
      }
    }
    D.hs[i] = p->grid.h[i] * D.inv_sigma[i];
    int L = p->grid.count[i];
    D.xstar[i] = INFINITY;
    if (!D.nocut) {
      if (nz.kind == AMY_NOISE_NORMAL) D.xstar[i] = zh;
      const double len = (zh - zl) / p->grid.h[i];
      // cells kept: centres in an interval of length len h (at most
      // floor(len) + 1), or cells meeting it (at most ceil(len) + 1)
      const double l = (D.wrule == AMY_WINDOW_CENTRE) ? floor(len) + 1.0 : ceil(len) + 1.0;
      if (l < (double)L) L = (int)l;
      const double half = (D.wrule == AMY_WINDOW_CENTRE) ? 0.5 : 0.0;
      D.win_a[i] = (D.lo[i] - zl) * D.inv_h[i] + half;
      D.win_b[i] = (D.lo[i] - zh) * D.inv_h[i] + half;
    }
    D.L[i] = L;
    W *= L;
  }
  D.W = (int32_t)(W < 2147483647 ? W : 2147483647);
  int nu = 1;
  for (int k = 0; k < m; ++k) {
    D.ucount[k] = p->inputs.count[k];
    D.ulo[k] = p->inputs.lo[k];
    D.uhi[k] = p->inputs.hi[k];
    D.ustep[k] = (p->inputs.count[k] > 1) ? (p->inputs.hi[k] - p->inputs.lo[k]) / (double)(p->inputs.count[k] - 1)
                                          : 0.0;
    nu *= p->inputs.count[k];
  }
  D.n_u = nu;
  // disturbance digits follow the inputs in the walk
  D.pd = p->dist.p;
  D.nd = m + D.pd;
  int nw = 1;
  for (int l = 0; l < D.pd; ++l) {
    const int k = m + l;
    D.ucount[k] = p->dist.count[l];
    D.ulo[k] = p->dist.lo[l];
    D.uhi[k] = p->dist.hi[l];
    D.ustep[k] = (p->dist.count[l] > 1) ? (p->dist.hi[l] - p->dist.lo[l]) / (double)(p->dist.count[l] - 1) : 0.0;
    nw *= p->dist.count[l];
  }
  D.n_w = nw;
  D.n_rows = nu * nw;
  for (int i = 0; i < AMY_MAX_DIM; ++i) {
    D.tlo[i] = p->target.lo[i];
    D.thi[i] = p->target.hi[i];
    D.alo[i] = p->avoid.lo[i];
    D.ahi[i] = p->avoid.hi[i];
    D.slo[i] = p->safe.lo[i];
    D.shi[i] = p->safe.hi[i];
  }
  for (int k = 0; k < p->dyn.n_params; ++k) D.params[k] = p->dyn.params[k];
  pl->W = W;
  pl->rows = nx * (int64_t)nu * nw;
  pl->f64 = (p->precision == AMY_FP64);
}

static inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Workspace: labels | V0 | V1 | tail max | (stored: T rows | origins | slot offsets).
// T is kept in the precision of the path (FP32 rows for the FP32 path,
// as the paper's own memory figures imply; FP64 rows for the plain path).
void amy_layout(Plan* pl, int mode) {
  const DevProblem& D = pl->dev;
  const uint64_t nx = (uint64_t)D.n_x;
  const uint64_t vs = pl->f64 ? 8 : 4;
  uint64_t o = 0;
  pl->off_label = o;  o = align256(o + nx);
  pl->off_v0 = o;     o = align256(o + nx * vs);
  pl->off_v1 = o;     o = align256(o + nx * vs);
  pl->off_tail = o;   o = align256(o + 8);
  pl->stored_bytes = 0;
  if (mode == AMY_MODE_STORED) {
    const uint64_t tiles = (nx + 63) / 64;
    const uint64_t rows_p = tiles * 64 * (uint64_t)D.n_rows;
    pl->off_T = o;    o = align256(o + rows_p * (uint64_t)pl->W * vs);
    pl->off_org = o;  o = align256(o + rows_p * 4 + (uint64_t)pl->W * 4);  // + slot offsets
    pl->stored_bytes = o - pl->off_T;
  }
  pl->mode = mode;
  pl->ws_bytes = o;
}

// AUTO: on MI355X the on-the-fly sweep costs ~3W flops plus the edge
// erfc's per row, the stored sweep 4W (8W) bytes of HBM traffic; at the
// chip's ~20 flop/byte balance OTF wins for every built-in family, so AUTO
// takes OTF.  STORED is used only when asked for explicitly.
// Group-variant layout for G lanes per state: the state's 1-D tables back to
// back (gsl entries), 64/G states per block; the lane space is the smallest
// run of innermost dimensions with at least G cells.
static void plan_group(Plan* pl, int G) {
  DevProblem& D = pl->dev;
  int off = 0;
  for (int i = 0; i < D.n; ++i) {
    D.goff[i] = off;
    off += D.L[i];
  }
  D.gsl = (off + 1) & ~1;
  int64_t cells = 1;
  int nout = D.n;
  while (nout > 0 && cells < G) cells *= D.L[--nout];
  D.grp_g = G;
  D.grp_nout = nout;
  D.lds_bytes_group = (64 / G) * D.gsl * (pl->f64 ? 8 : 4);
}

amy_status amy_resolve(const amy_problem* p, uint64_t budget, Plan* pl) {
  amy_make_plan(p, pl);
  int mode = p->mode == AMY_MODE_AUTO ? AMY_MODE_OTF : p->mode;
  const bool user = p->dyn.kind == AMY_DYN_USER;
  if (user && mode == AMY_MODE_STORED)
    return amy_fail(AMY_E_UNSUPPORTED, "dynamics given as text run on the fly only");
  if (mode == AMY_MODE_STORED && (int64_t)pl->dev.W != pl->W)
    return amy_fail(AMY_E_UNSUPPORTED, "window of %lld slots too large to store", (long long)pl->W);
  amy_layout(pl, mode);
  if (budget && pl->ws_bytes > budget)
    return amy_fail(AMY_E_NOMEM, "workspace %llu B exceeds budget %llu B",
                    (unsigned long long)pl->ws_bytes, (unsigned long long)budget);
  // variants that fit: one lane per state needs every lane's 1-D tables in
  // LDS; the group variants need one set per state of the block
  const bool lanes_ok = (plan_tables(p, pl) == AMY_OK);
  // the compiled shapes' own tables, and the factored sweep's shared
  // relative tables, are additive normal masses over the window either rule
  // gives, for rows without a disturbance
  const bool normal_masses = pl->dev.pd == 0 && pl->dev.noise == AMY_NOISE_NORMAL && !pl->dev.mult;
  // the other noise models and the intersect window (additive noise, no
  // disturbance) run a compiled shape when every step of the solve reads its
  // masses from memoised tables, which are built with the general path
  bool memo_only_ok = false;
  if (!normal_masses && !user && pl->dev.pd == 0 && !pl->dev.mult && mode == AMY_MODE_OTF &&
      amy_fixed_memo_complete(pl->dev, pl->f64)) {
    DevProblem q = pl->dev;
    memo_only_ok = plan_memo(p, q);
  }
  const bool fixed_ok = lanes_ok && (normal_masses ? amy_fixed_available(pl->dev) : memo_only_ok);
  const bool fac_ok = fixed_ok && normal_masses && mode == AMY_MODE_OTF && amy_fac_available(pl->dev);
  int64_t sum_l = 0;
  for (int i = 0; i < pl->dev.n; ++i) sum_l += pl->dev.L[i];
  const int64_t msz = pl->f64 ? 8 : 4;
  const bool g16_ok = 4 * ((sum_l + 1) & ~1) * msz <= LDS_BUDGET;
  const bool g64_ok = ((sum_l + 1) & ~1) * msz <= LDS_BUDGET;
  // one wave per state, lanes over inputs: normal noise, on the fly, built-in
  // families, and uncached per-lane tables that fit
  bool inputs_ok = mode == AMY_MODE_OTF && !user && pl->dev.noise == AMY_NOISE_NORMAL && !pl->dev.mult;
  if (inputs_ok) {
    Plan q = *pl;
    inputs_ok = plan_tables(p, &q, true) == AMY_OK;
  }
  auto feasible = [&](int v) {
    if (user && (v == AMY_VARIANT_FIXED || v == AMY_VARIANT_FACTORED)) return false;
    switch (v) {
      case AMY_VARIANT_LANES: return lanes_ok;
      case AMY_VARIANT_FIXED: return fixed_ok;
      case AMY_VARIANT_FACTORED: return fac_ok;
      case AMY_VARIANT_GROUP16: return g16_ok && mode == AMY_MODE_OTF;
      case AMY_VARIANT_GROUP64: return g64_ok && mode == AMY_MODE_OTF;
      case AMY_VARIANT_INPUTS: return inputs_ok;
    }
    return false;
  };
  if (mode == AMY_MODE_STORED && !lanes_ok)
    return amy_fail(AMY_E_UNSUPPORTED, "stored mode: window tables need more LDS than one lane per state allows");
  int v = p->variant;
  if (v != AMY_VARIANT_AUTO && !feasible(v))
    return amy_fail(AMY_E_UNSUPPORTED, "sweep variant %d does not fit this problem", v);
  if (v == AMY_VARIANT_AUTO) {
    const int t = amy_tune_lookup_variant(*pl, p);  // tuned choice, if any
    if (t != AMY_VARIANT_AUTO && feasible(t)) v = t;
  }
  if (v == AMY_VARIANT_AUTO) {
    // one lane per state while its tables leave room for >= 6 waves per CU
    // and the window is small; otherwise lanes share a state's window
    const bool lanes_light = lanes_ok && pl->dev.lds_bytes_tail <= 24 * 1024 && pl->W < 1024;
    // few states with enough rows each to fill a wave's lanes (inputs times
    // disturbance points): one wave per state keeps the GPU busy
    const bool few_states = (pl->dev.n_x + 63) / 64 < 1024 && pl->dev.n_rows >= 64;
    if (fac_ok) v = AMY_VARIANT_FACTORED;
    else if (fixed_ok) v = AMY_VARIANT_FIXED;
    else if (inputs_ok && few_states) v = AMY_VARIANT_INPUTS;
    else if (lanes_light) v = AMY_VARIANT_LANES;
    else if (pl->W >= 4096 && g64_ok) v = AMY_VARIANT_GROUP64;
    else if (g16_ok) v = AMY_VARIANT_GROUP16;
    else if (g64_ok) v = AMY_VARIANT_GROUP64;
    else if (lanes_ok) v = AMY_VARIANT_LANES;
    else
      return amy_fail(AMY_E_UNSUPPORTED, "window tables need %lld B of LDS even for one state per wave",
                      (long long)(sum_l * msz));
  }
  if (v == AMY_VARIANT_INPUTS) plan_tables(p, pl, true);
  pl->dev.variant = v;
  pl->dev.rel_entries = 0;
  pl->dev.tables = 0;
  if ((v == AMY_VARIANT_FACTORED && amy_rel_plan(pl->dev) > 0 && (pl->dev.tables = 1)) ||
      (v == AMY_VARIANT_FIXED && mode == AMY_MODE_OTF && plan_memo(p, pl->dev) && (pl->dev.tables = 2))) {
    // tables after the rest of the workspace: shared relative tables hold
    // masses then origins; memoised tables hold one record per entry
    const uint64_t msz = pl->f64 ? 8 : 4, ne = (uint64_t)pl->dev.rel_entries;
    pl->off_rel = pl->ws_bytes;
    if (pl->dev.tables == 2) {
      int lmax = 1;
      for (int i = 0; i < pl->dev.n; ++i) lmax = pl->dev.L[i] > lmax ? pl->dev.L[i] : lmax;
      // records, then each entry's FP64 kept-window and grid masses
      pl->ws_bytes += ((ne * (uint64_t)amy_memo_rec(lmax) * msz + 255) & ~255ull) + ((ne * 16 + 255) & ~255ull);
    } else {
      pl->ws_bytes += ((ne * 8 * msz + 255) & ~255ull) + ((ne * 4 + 255) & ~255ull);
    }
    if (budget && pl->ws_bytes > budget)
      return amy_fail(AMY_E_NOMEM, "workspace %llu B exceeds budget %llu B",
                      (unsigned long long)pl->ws_bytes, (unsigned long long)budget);
  }
  // the factored sweep forms no row tails: its first step takes them from
  // memoised kept-window and grid masses when those tables can be planned
  pl->tail_memo = false;
  if (pl->dev.variant == AMY_VARIANT_FACTORED && pl->dev.tables == 1) {
    DevProblem q = pl->dev;
    if (plan_memo(p, q)) {
      q.tables = 2;
      int lmax = 1;
      for (int i = 0; i < q.n; ++i) lmax = q.L[i] > lmax ? q.L[i] : lmax;
      const uint64_t msz = pl->f64 ? 8 : 4, ne = (uint64_t)q.rel_entries;
      const uint64_t bytes = ((ne * (uint64_t)amy_memo_rec(lmax) * msz + 255) & ~255ull) + ((ne * 16 + 255) & ~255ull);
      if ((!budget || pl->ws_bytes + bytes <= budget) && amy_tail_memo_lds(q) <= 64 * 1024) {
        pl->tail_memo = true;
        pl->tail_dev = q;
        pl->off_tailtab = pl->ws_bytes;
        pl->ws_bytes += bytes;
      }
    }
  }
  plan_group(pl, v == AMY_VARIANT_GROUP64 ? 64 : 16);
  if (v != AMY_VARIANT_GROUP16 && v != AMY_VARIANT_GROUP64) pl->dev.grp_g = 1;
  return AMY_OK;
}

static void fill_info(const amy_problem* p, const Plan& pl, amy_info* info) {
  memset(info, 0, sizeof *info);
  info->mode_used = pl.mode;
  for (int i = 0; i < p->grid.n; ++i) info->window[i] = pl.dev.L[i];
  info->kernel = pl.dev.variant;
  info->table_cache_mask = 0;
  for (int i = 0; i < p->grid.n; ++i)
    if (pl.dev.ccount[i] > 0) info->table_cache_mask |= 1 << i;
  info->lds_bytes = (pl.dev.grp_g > 1) ? pl.dev.lds_bytes_group
                    : ((pl.dev.variant == AMY_VARIANT_FIXED || pl.dev.variant == AMY_VARIANT_FACTORED)
                           ? pl.dev.lds_bytes_fixed : pl.dev.lds_bytes);
  info->n_x = pl.dev.n_x;
  info->n_u = pl.dev.n_u;
  info->n_w = pl.dev.n_w;
  info->rows = pl.rows;
  info->W = pl.W;
  info->workspace_bytes = pl.ws_bytes;
  info->stored_bytes = pl.stored_bytes;
}

extern "C" amy_status amy_query(const amy_problem* p, uint64_t ws_budget, amy_info* out) {
  amy_status st = amy_validate(p);
  if (st != AMY_OK) return st;
  Plan pl;
  st = amy_resolve(p, ws_budget, &pl);
  if (st != AMY_OK) return st;
  if (out) fill_info(p, pl, out);
  return AMY_OK;
}

// ------------------------------------------------------------------ solve

// Bellman step k (T_d >= k >= 1, Alg. 4's time loop) of a solve whose
// labels and V_{T_d+1} (and stored rows) are in place: reads V buffer
// (T_d - k) & 1 and writes the other one, or V_out at k = 1.
hipError_t amy_enqueue_step(const Plan& pl, hipStream_t st, void* ws, double* V_out, int16_t* pol, int horizon,
                            int k, bool want_tail, bool tail_memo) {
  const DevProblem& D = pl.dev;
  char* base = (char*)ws;
  const uint8_t* label = (const uint8_t*)(base + pl.off_label);
  void* Vb[2] = {base + pl.off_v0, base + pl.off_v1};
  unsigned long long* tail = (want_tail && k == horizon) ? (unsigned long long*)(base + pl.off_tail) : nullptr;
  const int cur = (horizon - k) & 1;
  const bool last = (k == 1);
  const SweepKind sk = pl.f64 ? SWEEP_F64 : (last ? SWEEP_F32_LAST : SWEEP_F32);
  void* out = last ? (void*)V_out : Vb[cur ^ 1];
  int16_t* pk = pol ? pol + (int64_t)(k - 1) * D.n_x : nullptr;
  if (pl.user) return amy_user_launch_sweep(pl.user, D, (int)sk, Vb[cur], out, label, pk, tail, st);
  if (pl.mode == AMY_MODE_STORED)
    return amy_launch_sweep_stored(D, sk, base + pl.off_T, (const int32_t*)(base + pl.off_org), Vb[cur], out,
                                   label, pk, st);
  if (D.variant == AMY_VARIANT_FACTORED) {
    const bool fused = tail && tail_memo;
    return amy_launch_sweep_fac(D, sk, Vb[cur], out, label, pk, tail, D.rel_entries > 0 ? base + pl.off_rel : nullptr,
                                st, fused ? &pl.tail_dev : nullptr, fused ? base + pl.off_tailtab : nullptr);
  }
  if (D.variant == AMY_VARIANT_FIXED)
    return amy_launch_sweep_fixed(D, sk, Vb[cur], out, label, pk, tail, D.rel_entries > 0 ? base + pl.off_rel : nullptr,
                                  st);
  if (D.grp_g > 1) return amy_launch_sweep_group(D, sk, Vb[cur], out, label, pk, tail, st);
  return amy_launch_sweep_otf(D, sk, Vb[cur], out, label, pk, tail, st);
}

// Per-solve tables that the sweeps read (the factored sweep's shared
// relative tables), after the labels and before the first step.
hipError_t amy_enqueue_prepare(const Plan& pl, hipStream_t st, void* ws, int horizon) {
  if (pl.dev.rel_entries <= 0 || horizon < 1) return hipSuccess;
  if (pl.dev.tables == 2) return amy_launch_memo_build(pl.dev, pl.f64, (char*)ws + pl.off_rel, st);
  return amy_launch_rel_build(pl.dev, pl.f64, (char*)ws + pl.off_rel, st);
}

amy_status amy_enqueue(const Plan& pl, hipStream_t st, void* ws, double* V_out, int16_t* pol,
                       int horizon, bool want_tail, Timing* tm) {
  const DevProblem& D = pl.dev;
  char* base = (char*)ws;
  uint8_t* label = (uint8_t*)(base + pl.off_label);
  void* Vb[2] = {base + pl.off_v0, base + pl.off_v1};
  unsigned long long* tailmax = (unsigned long long*)(base + pl.off_tail);
  hipError_t e;
  if (tm) hipEventRecord(tm->ev[0], st);
  if ((e = amy_launch_init(D, label, Vb[0], pl.f64, horizon == 0 ? V_out : nullptr, tailmax, st)) != hipSuccess)
    return amy_hip_fail(e, "init kernel");
  // the FP64 tail pass rides on the first kernel that builds every row
  // (the stored-mode build, else the first sweep); alone only when T_d = 0
  if (want_tail && horizon == 0 &&
      (e = pl.user ? amy_user_launch_tail(pl.user, D, label, tailmax, st) : amy_launch_tail(D, label, tailmax, st)) !=
          hipSuccess)
    return amy_hip_fail(e, "tail kernel");
  const bool stored = (pl.mode == AMY_MODE_STORED);
  if ((e = amy_enqueue_prepare(pl, st, ws, horizon)) != hipSuccess) return amy_hip_fail(e, "table kernel");
  if (stored && horizon > 0) {
    if ((e = amy_launch_build(D, pl.f64, label, base + pl.off_T, (int32_t*)(base + pl.off_org),
                              want_tail ? tailmax : nullptr, st)) != hipSuccess)
      return amy_hip_fail(e, "build kernel");
  }
  // the factored first step's tails from memoised tables, built here: inside
  // the first sweep where it can take them, else in a pass of their own
  const bool tail_tab = want_tail && horizon > 0 && !stored && pl.tail_memo;
  const bool tail_fused = tail_tab && !pl.user && amy_fac_fuses_tail(D, pl.tail_dev, pl.f64);
  if (tail_tab) {
    void* tab = base + pl.off_tailtab;
    if ((e = amy_launch_memo_build(pl.tail_dev, pl.f64, tab, st)) != hipSuccess ||
        (!tail_fused && (e = amy_launch_tail_memo(pl.tail_dev, pl.f64, label, tab, tailmax, st)) != hipSuccess))
      return amy_hip_fail(e, "tail tables");
  }
  if (tm) hipEventRecord(tm->ev[1], st);
  for (int k = horizon; k >= 1; --k) {
    if (tm && k == 1) hipEventRecord(tm->ev[2], st);
    if ((e = amy_enqueue_step(pl, st, ws, V_out, pol, horizon, k, want_tail && (!tail_tab || tail_fused),
                              tail_fused)) != hipSuccess)
      return amy_hip_fail(e, "sweep kernel");
    if (tm && k == horizon) hipEventRecord(tm->ev[5], st);
  }
  if (tm) {
    if (horizon == 0) {
      hipEventRecord(tm->ev[5], st);
      hipEventRecord(tm->ev[2], st);
    }
    hipEventRecord(tm->ev[3], st);
    hipEventRecord(tm->ev[4], st);
  }
  return AMY_OK;
}

static amy_status solve_impl(const amy_problem* p, const amy_user_dynamics* user, void* stream, void* workspace,
                             uint64_t ws_bytes, double* V_out, int16_t* policy_out, amy_info* info) {
  amy_status st = amy_validate(p);
  if (st != AMY_OK) return st;
  if (user && (st = amy_user_check(user, p)) != AMY_OK) return st;
  if (!user && p->dyn.kind == AMY_DYN_USER)
    return amy_fail(AMY_E_INVALID, "dynamics given as text are solved with amy_solve_user");
  Plan pl;
  st = amy_resolve(p, ws_bytes, &pl);
  if (st != AMY_OK) return st;
  pl.user = user;
  if (!workspace || !V_out) return amy_fail(AMY_E_INVALID, "workspace or V_out is NULL");
  if (((uintptr_t)workspace & 255) != 0) return amy_fail(AMY_E_INVALID, "workspace not 256-byte aligned");
  hipStream_t hs = (hipStream_t)stream;
  Timing tm;
  Timing* tp = nullptr;
  if (info) {
    for (int i = 0; i < Timing::N; ++i) {
      hipError_t e = hipEventCreate(&tm.ev[i]);
      if (e != hipSuccess) return amy_hip_fail(e, "hipEventCreate");
    }
    tp = &tm;
  }
  st = amy_enqueue(pl, hs, workspace, V_out, policy_out, p->horizon, info != nullptr, tp);
  if (st == AMY_OK && info) {
    hipError_t e = hipEventSynchronize(tm.ev[4]);
    if (e != hipSuccess) st = amy_hip_fail(e, "solve");
    else {
      fill_info(p, pl, info);
      unsigned long long bits = 0;
      e = hipMemcpy(&bits, (char*)workspace + pl.off_tail, 8, hipMemcpyDeviceToHost);
      if (e != hipSuccess) st = amy_hip_fail(e, "tail readback");
      double t;
      memcpy(&t, &bits, 8);
      info->max_row_tail = t;
      info->tail_bound_E = t * p->horizon;
      float ms;
      hipEventElapsedTime(&ms, tm.ev[0], tm.ev[1]);
      info->t_build_ms = ms;
      hipEventElapsedTime(&ms, tm.ev[1], tm.ev[3]);
      info->t_sweeps_ms = ms;
      ms = 0.f;
      if (p->horizon >= 3) hipEventElapsedTime(&ms, tm.ev[5], tm.ev[2]);
      info->t_main_sweeps_ms = ms;
      hipEventElapsedTime(&ms, tm.ev[3], tm.ev[4]);
      info->t_readout_ms = ms;
      hipEventElapsedTime(&ms, tm.ev[0], tm.ev[4]);
      info->t_total_ms = ms;
    }
  }
  if (tp)
    for (int i = 0; i < Timing::N; ++i) hipEventDestroy(tm.ev[i]);
  return st;
}

extern "C" amy_status amy_solve(const amy_problem* p, void* stream, void* workspace, uint64_t ws_bytes,
                                double* V_out, int16_t* policy_out, amy_info* info) {
  return solve_impl(p, nullptr, stream, workspace, ws_bytes, V_out, policy_out, info);
}

extern "C" amy_status amy_solve_user(const amy_user_dynamics* f, const amy_problem* p, void* stream, void* workspace,
                                     uint64_t ws_bytes, double* V_out, int16_t* policy_out, amy_info* info) {
  if (!f) return amy_fail(AMY_E_INVALID, "user dynamics handle is NULL");
  return solve_impl(p, f, stream, workspace, ws_bytes, V_out, policy_out, info);
}
