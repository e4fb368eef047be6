// amy_device.hpp -- device building blocks of the abstraction + Bellman path.
//
//  * Dyn<KIND,N>   : the mean mu = f(x_bar, u_bar) (Alg. 2, first step), split
//                    into a per-state part (prep) and a per-input part (apply)
//                    so that the inner input loop only redoes what depends on u.
//  * window / dim_table : the cutting region of Sec. 5.2 (cells whose centre
//                    lies in [[mu - x*, mu + x*]]) laid out as a fixed window
//                    of L_i slots that always lies inside the grid; slots
//                    outside the kept range carry mass 0.  The 1-D masses
//                    Phi(b) - Phi(a) of the L_i slots are built from L_i + 1
//                    edge values erfc(|z|/sqrt 2): a diagonal covariance makes
//                    the cell mass of Alg. 1 a product of these 1-D masses.
//  * contract      : Alg. 4's row sum  sum_{x' in window} T(x'|x,u) V(x')
//                    evaluated dimension by dimension (a tensor contraction of
//                    the 1-D tables with the window of V), which needs about
//                    W (1 + 1/L_n + ...) multiply-adds instead of 2W.
// Everything here is compiled with -ffp-contract=off; fused multiply-adds
// appear only where written (fma_).
#pragma once
// (also compiled at run time by hipRTC, which supplies the HIP and math
// declarations itself: __HIPCC_RTC__ marks that build)
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#endif

#include "amy_plan.hpp"

#define AMY_DYN_AFFINE_ 0
#define AMY_DYN_UNICYCLE_ 1
#define AMY_DYN_ROOM_ 2
#define AMY_DYN_VEHICLE7_ 3
#define AMY_DYN_ROBOT_ 4

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Renumber them so that XCD x receives one contiguous run of logical blocks:
// neighbouring states, whose windows overlap, then share an L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G) {
  const uint32_t q = G >> 3, r = G & 7u, x = b & 7u, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Centre of the state's cell, per dimension (state numbering: last dim fastest).
template <int N>
__device__ __forceinline__ void state_centre(const DevProblem& P, uint32_t s, double* x) {
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    const uint32_t c = (uint32_t)P.count[i];
    const uint32_t q = s / c;
    const uint32_t j = s - q * c;
    s = q;
    x[i] = P.lo[i] + ((double)j + 0.5) * P.h[i];
  }
}

// (input, disturbance) points as an odometer over the nd digits: the m
// input dimensions, then the disturbance dimensions (last fastest).  u[k]
// for k < m is the input, u[m + l] the disturbance's dimension l.
struct InputWalk {
  int dig[AMY_MAXI];
  __device__ __forceinline__ void reset() {
#pragma unroll
    for (int k = 0; k < AMY_MAXI; ++k) dig[k] = 0;
  }
  __device__ __forceinline__ void values(const DevProblem& P, double* u) const {
#pragma unroll
    for (int k = 0; k < AMY_MAXI; ++k)
      u[k] = (k < P.nd) ? ((P.ucount[k] == 1) ? P.ulo[k] : P.ulo[k] + (double)dig[k] * P.ustep[k]) : 0.0;
  }
  // the first row of input number u (input digits of u, disturbance digits 0)
  __device__ __forceinline__ void set_input(const DevProblem& P, int u) {
#pragma unroll
    for (int k = AMY_MAXI - 1; k >= 0; --k) {
      if (k >= P.nd) {
        dig[k] = 0;
      } else if (k >= P.m) {
        dig[k] = 0;
      } else {
        dig[k] = u % P.ucount[k];
        u /= P.ucount[k];
      }
    }
  }
  __device__ __forceinline__ void next(const DevProblem& P) {
    bool carry = true;
#pragma unroll
    for (int k = AMY_MAXI - 1; k >= 0; --k) {
      if (carry && k < P.nd) {
        if (++dig[k] >= P.ucount[k]) dig[k] = 0;
        else carry = false;
      }
    }
  }
};

// ----------------------------------------------------------------- dynamics

template <int KIND, int N>
struct Dyn;

template <int N>
struct Dyn<AMY_DYN_AFFINE_, N> {
  struct State { double s[N]; };
  __device__ __forceinline__ static void prep(const DevProblem& P, const double* x, State& st) {
    const double* A = P.params;
    const double* c = P.params + N * N + N * P.m;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < N; ++j) s = s + A[i * N + j] * x[j];
      st.s[i] = s + c[i];
    }
  }
  __device__ __forceinline__ static void apply(const DevProblem& P, const State& st, const double*,
                                               const double* u, double* mu) {
    const double* B = P.params + N * N;
    const double* D = P.params + N * N + N * P.m + N;  // disturbance columns (pd > 0)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < AMY_MAXI; ++k)
        if (k < P.m) t = t + B[i * P.m + k] * u[k];
      mu[i] = st.s[i] + t;
      if (P.pd > 0) {
        double d = 0.0;
#pragma unroll
        for (int l = 0; l < AMY_MAXI; ++l)
          if (l < P.pd) d = d + D[i * P.pd + l] * u[P.m + l];
        mu[i] = mu[i] + d;
      }
    }
  }
};

// The planar robot of Sec. 7: speed u0 along heading u1, pushed by the
// disturbance w on both axes (w = 0 and no w term without a disturbance).
template <>
struct Dyn<AMY_DYN_ROBOT_, 2> {
  struct State { int unused; };
  __device__ __forceinline__ static void prep(const DevProblem&, const double*, State&) {}
  __device__ __forceinline__ static void apply(const DevProblem& P, const State&, const double* x,
                                               const double* u, double* mu) {
    const double a = P.params[0] * u[0];
    mu[0] = x[0] + a * cos(u[1]);
    mu[1] = x[1] + a * sin(u[1]);
    if (P.pd > 0) {
      mu[0] = mu[0] + u[2];
      mu[1] = mu[1] + u[2];
    }
  }
};

template <>
struct Dyn<AMY_DYN_UNICYCLE_, 3> {
  struct State { double c, s; };
  __device__ __forceinline__ static void prep(const DevProblem&, const double* x, State& st) {
    st.c = cos(x[2]);
    st.s = sin(x[2]);
  }
  __device__ __forceinline__ static void apply(const DevProblem& P, const State& st, const double* x,
                                               const double* u, double* mu) {
    const double tau = P.params[0];
    const double a = tau * u[0];
    mu[0] = x[0] + a * st.c;
    mu[1] = x[1] + a * st.s;
    mu[2] = x[2] + tau * u[1];
  }
};

template <int N>
struct Dyn<AMY_DYN_ROOM_, N> {
  struct State { double s[N], g[N]; };
  __device__ __forceinline__ static void prep(const DevProblem& P, const double* x, State& st) {
    const double al = P.params[0], be = P.params[1], ga = P.params[2], Te = P.params[3],
                 Th = P.params[4];
    const double c0 = (1.0 - 2.0 * al) - be;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double left = x[(i + N - 1) % N], right = x[(i + 1) % N];
      st.s[i] = (c0 * x[i] + al * (left + right)) + be * Te;
      st.g[i] = ga * (Th - x[i]);
    }
  }
  __device__ __forceinline__ static void apply(const DevProblem& P, const State& st, const double*,
                                               const double* u, double* mu) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double ui = (P.m == 1) ? u[0] : u[i < AMY_MAXI ? i : 0];
      mu[i] = st.s[i] + ui * st.g[i];
    }
  }
};

template <>
struct Dyn<AMY_DYN_VEHICLE7_, 7> {
  struct State { int unused; };
  __device__ __forceinline__ static void prep(const DevProblem&, const double*, State&) {}
  __device__ __forceinline__ static void apply(const DevProblem& P, const State&, const double* x,
                                               const double* u, double* mu) {
    const double* q = P.params;
    const double tau = q[0], lwb = q[1], mass = q[2], mub = q[3], lf = q[4], lr = q[5];
    const double hcg = q[6], Iz = q[7], CSf = q[8], CSr = q[9], g = q[10];
    const double x3 = x[2], x4 = x[3], x5 = x[4], x6 = x[5], x7 = x[6];
    const double v1 = fmin(fmax(u[0], P.ulo[0]), P.uhi[0]);
    const double v2 = fmin(fmax(u[1], P.ulo[1]), P.uhi[1]);
    double f1, f2, f5, f6, f7;
    if (fabs(x4) < 0.1) {
      f1 = x4 * cos(x5);
      f2 = x4 * sin(x5);
      f5 = (x4 / lwb) * tan(x3);
      const double c3 = cos(x3);
      f6 = (v2 / lwb) * tan(x3) + (x4 / (lwb * (c3 * c3))) * v1;
      f7 = 0.0;
    } else {
      const double Ff = g * lr - v2 * hcg;
      const double Fr = g * lf + v2 * hcg;
      f1 = x4 * cos(x5 + x7);
      f2 = x4 * sin(x5 + x7);
      f5 = x6;
      const double r64 = x6 / x4;
      f6 = ((mub * mass) / (Iz * (lr + lf))) *
           ((lf * CSf * Ff * x3 + (lr * CSr * Fr - lf * CSf * Ff) * x7) -
            (lf * lf * CSf * Ff + lr * lr * CSr * Fr) * r64);
      f7 = (mub / (x4 * (lr + lf))) *
               ((CSf * Ff * x3 + (CSr * Fr + CSf * Ff) * x7) - (lf * CSf * Ff - lr * CSr * Fr) * r64) -
           x6;
    }
    mu[0] = x[0] + tau * f1;
    mu[1] = x[1] + tau * f2;
    mu[2] = x3 + tau * v1;
    mu[3] = x4 + tau * v2;
    mu[4] = x5 + tau * f5;
    mu[5] = x6 + tau * f6;
    mu[6] = x7 + tau * f7;
  }
};

// ---------------------------------------------------------- cutting window

// Kept cells of dimension i for mean mu: [jlo, b-1] (empty when b == jlo),
// and the origin o of the fixed L_i-slot window, o <= jlo, o + L_i <= n_i.
// z0 = (lo - mu) / scale is the edge coordinate of grid edge 0 and hs the
// edge spacing in those units.  isc: the inverse of the state's noise scale
// factor (multiplicative noise: 1/|x_i|, infinite at x_i = 0; 1 otherwise).
struct Win { int jlo, b, o; double z0, hs; };

__device__ __forceinline__ Win window_1d(const DevProblem& P, int i, double mu, double isc = 1.0) {
  const int n = P.count[i], L = P.L[i];
  Win w;
  if (P.nocut) {
    w.jlo = 0;
    w.b = n;
  } else {
    const double m = mu * P.inv_h[i];
    double tl = m - P.win_a[i];
    double th = m - P.win_b[i];
    tl = fmin(fmax(tl, -1.0), (double)n);
    th = fmin(fmax(th, -2.0), (double)n);
    int jlo, jhi;
    if (P.wrule == 0) {
      // cell j is kept iff its centre lo + (j + 1/2) h lies in [mu + zl, mu + zh]
      jlo = max(0, (int)ceil(tl));
      jhi = min(n - 1, (int)floor(th));
    } else {
      // cell j is kept iff (lo + j h, lo + (j + 1) h) meets (mu + zl, mu + zh)
      jlo = max(0, (int)floor(tl));
      jhi = min(n - 1, (int)ceil(th) - 1);
    }
    jhi = min(jhi, jlo + L - 1);  // allocation bound, for rounding at exact ties
    w.jlo = jlo;
    w.b = max(jhi + 1, jlo);
  }
  w.o = min(w.jlo, n - L);
  w.z0 = (P.lo[i] - mu) * P.inv_sigma[i] * isc;
  w.hs = P.hs[i] * isc;
  return w;
}

__device__ __forceinline__ float ec_of(double z, float) {
  return erfcf((float)(fabs(z) * 0.70710678118654752440));
}
__device__ __forceinline__ double ec_of(double z, double) {
  const double a = fabs(z);
  // erfc(a / sqrt 2) underflows to 0 in FP64 beyond a ~ 38.6
  return a > 38.5 ? 0.0 : erfc(a * 0.70710678118654752440);
}

// Phi(z1) - Phi(z0) from e = erfc(|z|/sqrt 2): upper-tail difference when
// both edges are >= 0, lower-tail difference when both are <= 0, else
// 1 minus both tails.  Tail cells keep their relative accuracy.
template <class MT>
__device__ __forceinline__ MT mass_of(double z0, MT e0, double z1, MT e1) {
  if (z0 >= 0.0) return MT(0.5) * (e0 - e1);
  if (z1 <= 0.0) return MT(0.5) * (e1 - e0);
  return MT(1) - MT(0.5) * (e0 + e1);
}

__device__ __forceinline__ double edge_z(const DevProblem&, int, const Win& w, int E) {
  return w.z0 + (double)E * w.hs;
}

// ---------------------------------------------------- other noise models
//
// FP64 lower and upper tail masses at a standardised edge z, for the
// noise models other than additive normal (and for multiplicative normal
// noise); the mass of a cell is the difference of the tail on the side of
// the median away from which both its edges lie, or 1 minus both tails.

struct Tails { double lo, up; };

// Regularised incomplete beta I_x(a, b) by its continued fraction
// (modified Lentz), for x below (a + 1) / (a + b + 2) where it converges fast.
__device__ __noinline__ double ibeta_cf(double x, double a, double b) {
  const double tiny = 1e-300;
  double c = 1.0, d = 1.0 - (a + b) * x / (a + 1.0);
  if (fabs(d) < tiny) d = tiny;
  d = 1.0 / d;
  double f = d;
  for (int k = 1; k <= 400; ++k) {
    const double kk = (double)k;
    // even term k(b - k) x / ((a + 2k - 1)(a + 2k))
    double num = kk * (b - kk) * x / ((a + 2.0 * kk - 1.0) * (a + 2.0 * kk));
    d = 1.0 + num * d;
    if (fabs(d) < tiny) d = tiny;
    c = 1.0 + num / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    f *= d * c;
    // odd term -(a + k)(a + b + k) x / ((a + 2k)(a + 2k + 1))
    num = -(a + kk) * (a + b + kk) * x / ((a + 2.0 * kk) * (a + 2.0 * kk + 1.0));
    d = 1.0 + num * d;
    if (fabs(d) < tiny) d = tiny;
    c = 1.0 + num / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    f *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  const double lbeta = lgamma(a) + lgamma(b) - lgamma(a + b);
  return exp(a * log(x) + b * log1p(-x) - lbeta) * f / a;
}

__device__ __noinline__ Tails noise_tails(const DevProblem& P, int i, double z) {
  Tails t;
  switch (P.noise) {
    case 1: {  // uniform on the unit support
      const double x = fmin(fmax(z - P.zoff[i], 0.0), 1.0);
      t.lo = x;
      t.up = 1.0 - x;
      break;
    }
    case 2: {  // exponential, unit rate in z
      if (z <= 0.0) {
        t.lo = 0.0;
        t.up = 1.0;
      } else {
        t.lo = -expm1(-z);
        t.up = exp(-z);
      }
      break;
    }
    case 3: {  // beta on the unit support
      const double x = fmin(fmax(z - P.zoff[i], 0.0), 1.0);
      const double a = P.balpha[i], b = P.bbeta[i];
      if (x <= 0.0) {
        t.lo = 0.0;
        t.up = 1.0;
      } else if (x >= 1.0) {
        t.lo = 1.0;
        t.up = 0.0;
      } else if (x < (a + 1.0) / (a + b + 2.0)) {
        t.lo = ibeta_cf(x, a, b);
        t.up = 1.0 - t.lo;
      } else {
        t.up = ibeta_cf(1.0 - x, b, a);
        t.lo = 1.0 - t.up;
      }
      break;
    }
    default: {  // normal: the small tail from erfc, exact on either side of 0
      const double a = fabs(z) > 38.5 ? 0.0 : erfc(fabs(z) * 0.70710678118654752440) * 0.5;
      t.lo = z <= 0.0 ? a : 1.0 - a;
      t.up = z <= 0.0 ? 1.0 - a : a;
      break;
    }
  }
  return t;
}

// Median of the standardised noise (the side switch of the differencing).
__device__ __forceinline__ double noise_median(const DevProblem& P, int i) {
  switch (P.noise) {
    case 1: return P.zoff[i] + 0.5;
    case 2: return 0.69314718055994530942;
    case 3: return P.zoff[i] + P.balpha[i] / (P.balpha[i] + P.bbeta[i]);
  }
  return 0.0;
}

__device__ __forceinline__ double tails_mass(double z0, const Tails& t0, double z1, const Tails& t1, double zm) {
  if (z1 <= zm) return t1.lo - t0.lo;
  if (z0 >= zm) return t0.up - t1.up;
  return (1.0 - t0.lo) - t1.up;
}

// Mass of [edge E0, edge E1] of dimension i in the general model (FP64);
// a zero noise scale (multiplicative noise at a zero coordinate, isc
// infinite) puts the whole mass in the cell that holds the mean.
__device__ __noinline__ double general_mass(const DevProblem& P, int i, const Win& w, int E0, int E1,
                                            double mu, double isc) {
  if (E1 <= E0) return 0.0;
  if (isinf(isc)) {
    const double a = P.lo[i] + (double)E0 * P.h[i], b = P.lo[i] + (double)E1 * P.h[i];
    return (a <= mu && mu < b) ? 1.0 : 0.0;
  }
  const double zm = noise_median(P, i);
  const double z0 = edge_z(P, i, w, E0), z1 = edge_z(P, i, w, E1);
  return tails_mass(z0, noise_tails(P, i, z0), z1, noise_tails(P, i, z1), zm);
}

// The slot masses of dim_table in the general noise models: FP64 tails per
// edge, each cell's mass rounded once (out of line: one copy per kernel
// file, not one per inlined call site).
template <class MT>
__device__ __noinline__ void general_table(const DevProblem& P, int i, const Win& w, double mu, double isc, MT* t,
                                           int ts) {
  const int L = P.L[i];
  if (isinf(isc)) {
    for (int k = 0; k < L; ++k)
      t[k * ts] = MT(general_mass(P, i, w, min(max(w.o + k, w.jlo), w.b), min(max(w.o + k + 1, w.jlo), w.b), mu, isc));
    return;
  }
  const double zm = noise_median(P, i);
  double zq = edge_z(P, i, w, min(max(w.o, w.jlo), w.b));
  Tails tq = noise_tails(P, i, zq);
  for (int k = 0; k < L; ++k) {
    const double z = edge_z(P, i, w, min(max(w.o + k + 1, w.jlo), w.b));
    const Tails tz = noise_tails(P, i, z);
    t[k * ts] = MT(z > zq ? tails_mass(zq, tq, z, tz, zm) : 0.0);
    zq = z;
    tq = tz;
  }
}

// 1-D masses of the L_i window slots of dimension i into t[k*ts] (slot k is
// cell o + k; cells outside the kept range get mass 0 because their two
// edges are clamped onto the same kept-range edge).
template <class MT>
__device__ __forceinline__ Win dim_table(const DevProblem& P, int i, double mu, MT* t, int ts) {
  const Win w = window_1d(P, i, mu);
  const int L = P.L[i];
  double zp = edge_z(P, i, w, min(max(w.o, w.jlo), w.b));
  MT ep = ec_of(zp, MT());
  for (int k = 0; k < L; ++k) {
    const double z = edge_z(P, i, w, min(max(w.o + k + 1, w.jlo), w.b));
    const MT e = ec_of(z, MT());
    t[k * ts] = mass_of(zp, ep, z, e);
    zp = z;
    ep = e;
  }
  return w;
}

// FP64 mass of [edge ea, edge eb] of dimension i.
__device__ __forceinline__ double mass_edges(const DevProblem& P, int i, const Win& w, int ea, int eb) {
  const double za = edge_z(P, i, w, ea), zb = edge_z(P, i, w, eb);
  return mass_of(za, ec_of(za, 0.0), zb, ec_of(zb, 0.0));
}

// FP64 kept-window mass and grid mass of dimension i (the per-row tail is
// prod_i grid_i - prod_i win_i).
__device__ __forceinline__ void win_grid_mass(const DevProblem& P, int i, const Win& w, double& win,
                                              double& grid) {
  win = mass_edges(P, i, w, w.jlo, w.b);
  grid = mass_edges(P, i, w, 0, P.count[i]);
}

// The same for the run-time-window sweeps, which also take the other noise
// models and multiplicative noise (isc: the state's inverse noise scale);
// the compiled-shape sweeps, which run additive normal noise only, call
// the plain forms above and carry no call to the general path.
template <class MT>
__device__ __forceinline__ Win dim_table_gen(const DevProblem& P, int i, double mu, MT* t, int ts, double isc) {
  if (P.noise != 0 || P.mult) {
    const Win w = window_1d(P, i, mu, isc);
    general_table<MT>(P, i, w, mu, isc, t, ts);
    return w;
  }
  return dim_table<MT>(P, i, mu, t, ts);
}

__device__ __forceinline__ void win_grid_mass_gen(const DevProblem& P, int i, const Win& w, double& win,
                                                  double& grid, double mu, double isc) {
  if (P.noise != 0 || P.mult) {
    win = general_mass(P, i, w, w.jlo, w.b, mu, isc);
    grid = general_mass(P, i, w, 0, P.count[i], mu, isc);
    return;
  }
  win_grid_mass(P, i, w, win, grid);
}

// Input digits of table c of dimension i (digits the mean does not depend on are 0).
__device__ __forceinline__ void combo_digits(const DevProblem& P, int i, int c, InputWalk& iw) {
#pragma unroll
  for (int k = 0; k < AMY_MAXI; ++k) {
    const int mlt = P.dep_mult[i][k];
    iw.dig[k] = (k < P.nd && mlt > 0) ? (c / mlt) % P.ucount[k] : 0;
  }
}

__device__ __forceinline__ int combo_index(const DevProblem& P, int i, const InputWalk& iw) {
  int c = 0;
#pragma unroll
  for (int k = 0; k < AMY_MAXI; ++k) c += iw.dig[k] * P.dep_mult[i][k];
  return c;
}

// ------------------------------------------------------- tail reduction

// Max of the wave's row tails into *tailmax (non-negative doubles order as
// their bits): one lane per wave updates it, and only when its value exceeds
// what the location already holds.  Every wave of a launch targets the same
// address, so unconditional atomics serialise there (one per wave: about
// 12 ns each, 0.1 ms for the unicycle's 9,375 waves); a stale read can only
// be lower than the location, so no needed update is skipped.
__device__ __forceinline__ void wave_max_to(double tmax, unsigned long long* tailmax) {
  for (int off = 32; off > 0; off >>= 1) tmax = fmax(tmax, __shfl_xor(tmax, off));
  if ((threadIdx.x & 63) == 0 && tmax > 0.0) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(tmax);
    if (b > __hip_atomic_load(tailmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(tailmax, b);
  }
}

// ------------------------------------------------------------- contraction

// sum over the window of prod_i t_i[k_i] * V[base + sum_i k_i stride_i],
// innermost dimension first; t_i starts at table entry toff[i].
// COMP: Kahan-compensated outermost sum.
template <int D, int N, class MT, class AT, class VT, bool COMP>
__device__ __forceinline__ AT contract(const DevProblem& P, const MT* __restrict__ t, int ts,
                                       const int* toff, const VT* __restrict__ V, int64_t base) {
  const int L = P.L[D];
  const MT* td = t + toff[D] * ts;
  AT acc = AT(0), c = AT(0);
  int k0 = 0;
  if constexpr (D == N - 1 && !(COMP && D == 0)) {
    // innermost run: four gathers in flight, summed in slot order
    for (; k0 + 4 <= L; k0 += 4) {
      AT v[4];
      MT m[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[j] = AT(V[base + k0 + j]);
        m[j] = td[(k0 + j) * ts];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) acc = fma_(AT(m[j]), v[j], acc);
    }
  }
  const int64_t step = D == N - 1 ? 1 : (int64_t)P.stride[D];
  int64_t o = base + (int64_t)k0 * step;  // slot k's offset, stepped rather than multiplied
  for (int k = k0; k < L; ++k, o += step) {
    AT inner;
    if constexpr (D == N - 1) inner = AT(V[o]);
    else inner = contract<D + 1, N, MT, AT, VT, COMP>(P, t, ts, toff, V, o);
    if constexpr (COMP && D == 0) {
      const AT y = AT(td[k * ts]) * inner - c;
      const AT s2 = acc + y;
      c = (s2 - acc) - y;
      acc = s2;
    } else {
      acc = fma_(AT(td[k * ts]), inner, acc);
    }
  }
  return acc;
}

// ---------------------------------------------------------------- row engine

// Per-lane LDS views of one 64-lane block: 1-D tables [entry][lane], cached
// window origins [slot][lane], and (tail pass) FP64 window / grid masses of
// the cached tables [2 slot + {0,1}][lane].
template <class MT>
struct LaneLds {
  MT* tab;
  int32_t* org;
  double* wg;
  __device__ __forceinline__ LaneLds(const DevProblem& P, unsigned char* smem, int lane) {
    tab = reinterpret_cast<MT*>(smem) + lane;
    org = reinterpret_cast<int32_t*>(smem + P.lds_int_off) + lane;
    wg = reinterpret_cast<double*>(smem + P.lds_tail_off) + lane;
  }
};

// Inverse noise-scale factors of the state at x: 1 for additive noise,
// 1/|x_i| for multiplicative noise (infinite at x_i = 0).
template <int N>
__device__ __forceinline__ void state_isc(const DevProblem& P, const double* x, double* isc) {
#pragma unroll
  for (int i = 0; i < N; ++i) isc[i] = P.mult ? 1.0 / fabs(x[i]) : 1.0;
}

// Build every cached table of state x (all input-digit combinations of the
// dimensions whose tables are cached); isc: the state's inverse noise
// scales (nullptr: additive noise, all 1).
template <int KIND, int N, class MT, bool TAIL, int LB>
__device__ __forceinline__ void build_cached(const DevProblem& P, const typename Dyn<KIND, N>::State& st,
                                             const double* x, const double* isc, const LaneLds<MT>& S) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int C = P.ccount[i];
    for (int c = 0; c < C; ++c) {
      InputWalk iw;
      combo_digits(P, i, c, iw);
      double uv[AMY_MAXI], mu[N];
      iw.values(P, uv);
      Dyn<KIND, N>::apply(P, st, x, uv, mu);
      Win w;
      if (isc) w = dim_table_gen<MT>(P, i, mu[i], S.tab + (P.toff[i] + c * P.L[i]) * LB, LB, isc[i]);
      else w = dim_table<MT>(P, i, mu[i], S.tab + (P.toff[i] + c * P.L[i]) * LB, LB);
      S.org[(P.ooff[i] + c) * LB] = w.o;
      if constexpr (TAIL) {
        double wm, gm;
        if (isc) win_grid_mass_gen(P, i, w, wm, gm, mu[i], isc[i]);
        else win_grid_mass(P, i, w, wm, gm);
        S.wg[(2 * (P.ooff[i] + c)) * LB] = wm;
        S.wg[(2 * (P.ooff[i] + c) + 1) * LB] = gm;
      }
    }
  }
}

// Tables of the current input: table offsets toff[] and window base index;
// rebuilds uncached tables whose mean changed.  TAIL: returns the row's
// FP64 tail (grid mass - kept-window mass).  isc: the state's inverse noise
// scales, or nullptr for code that runs additive normal noise only.
template <int KIND, int N, class MT, bool TAIL, int LB>
struct RowState {
  double prev[N];
  int o[N];
  double wmem[TAIL ? N : 1], gmem[TAIL ? N : 1];
  __device__ __forceinline__ void reset() {
#pragma unroll
    for (int i = 0; i < N; ++i) prev[i] = __builtin_nan("");
  }
  __device__ __forceinline__ int64_t prepare(const DevProblem& P, const InputWalk& iw, const double* mu,
                                             const double* isc, const LaneLds<MT>& S, int* toff, double& tail) {
    int64_t base = 0;
    double win = 1.0, grid = 1.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      int oi;
      if (P.ccount[i] > 0) {
        const int c = combo_index(P, i, iw);
        toff[i] = P.toff[i] + c * P.L[i];
        oi = S.org[(P.ooff[i] + c) * LB];
        if constexpr (TAIL) {
          win *= S.wg[(2 * (P.ooff[i] + c)) * LB];
          grid *= S.wg[(2 * (P.ooff[i] + c) + 1) * LB];
        }
      } else {
        if (mu[i] != prev[i]) {
          Win w;
          if (isc) w = dim_table_gen<MT>(P, i, mu[i], S.tab + P.toff[i] * LB, LB, isc[i]);
          else w = dim_table<MT>(P, i, mu[i], S.tab + P.toff[i] * LB, LB);
          o[i] = w.o;
          prev[i] = mu[i];
          if constexpr (TAIL) {
            if (isc) win_grid_mass_gen(P, i, w, wmem[i], gmem[i], mu[i], isc[i]);
            else win_grid_mass(P, i, w, wmem[i], gmem[i]);
          }
        }
        toff[i] = P.toff[i];
        oi = o[i];
        if constexpr (TAIL) {
          win *= wmem[i];
          grid *= gmem[i];
        }
      }
      base += (int64_t)oi * P.stride[i];
    }
    if constexpr (TAIL) tail = grid - win;
    return base;
  }
};
