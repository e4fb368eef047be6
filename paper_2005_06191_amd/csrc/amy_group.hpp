// amy_group.hpp -- Bellman sweep with G lanes per state (G = 16 or 64), for
// windows whose per-lane 1-D tables would not fit in LDS (thousands of
// cells per row): a wave holds 64/G states; the G lanes of a state build its
// 1-D tables together (slots split across lanes, kept in the group's LDS
// region), split the window -- each lane takes lane-space indices (the
// innermost dimensions from grp_nout on) and contracts the outer
// dimensions for them -- and combine their partial sums with a butterfly.
// With G = 64 this is one wavefront per (state, input) row.
// Loop trip counts and barriers are uniform across the wave (all states of
// a wave belong to one system); inactive states only skip arithmetic.
#pragma once
#include "amy_device.hpp"

// Mass of window slot k of dimension i (both edges evaluated here; the same
// edge values, clamps and differencing as dim_table).
template <class MT, bool GEN>
__device__ __forceinline__ MT slot_mass(const DevProblem& P, int i, const Win& w, int k, double mu, double isc) {
  const int e0 = min(max(w.o + k, w.jlo), w.b), e1 = min(max(w.o + k + 1, w.jlo), w.b);
  if constexpr (GEN)
    if (P.noise != 0 || P.mult) return MT(general_mass(P, i, w, e0, e1, mu, isc));
  const double z0 = edge_z(P, i, w, e0);
  const double z1 = edge_z(P, i, w, e1);
  return mass_of(z0, ec_of(z0, MT()), z1, ec_of(z1, MT()));
}

// Outer dimensions (D < nout) contracted, inner digits fixed at kin[].
template <int D, int N, class MT, class AT, class VT>
__device__ __forceinline__ AT gsum(const DevProblem& P, int nout, const MT* __restrict__ t, const int* kin,
                                   const VT* __restrict__ V, int64_t off) {
  if constexpr (D == N) {
    return AT(V[off]);
  } else {
    if (D < nout) {
      const MT* td = t + P.goff[D];
      const int64_t sd = P.stride[D];
      AT acc = AT(0);
      int k = 0;
      int64_t o = off;  // offset of slot k (stepped, not multiplied)
      if constexpr (D >= N - 2) {
        // the last levels: four sub-sums (gathers) in flight, added in slot order
        for (; k + 4 <= P.L[D]; k += 4) {
          AT in[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) in[j] = gsum<D + 1, N, MT, AT, VT>(P, nout, t, kin, V, o + j * sd);
#pragma unroll
          for (int j = 0; j < 4; ++j) acc = fma_(AT(td[k + j]), in[j], acc);
          o += 4 * sd;
        }
      }
      for (; k < P.L[D]; ++k, o += sd) acc = fma_(AT(td[k]), gsum<D + 1, N, MT, AT, VT>(P, nout, t, kin, V, o), acc);
      return acc;
    }
    return gsum<D + 1, N, MT, AT, VT>(P, nout, t, kin, V, off + (int64_t)kin[D] * P.stride[D]);
  }
}

template <int KIND, int N, class MT, class AT, class VI, class VO, bool COMP, bool TAIL, int G, bool GEN = true>
__device__ __forceinline__ void sweep_group(const DevProblem& P, uint32_t tile, const VI* __restrict__ Vin,
                                            VO* __restrict__ Vout, const uint8_t* __restrict__ label,
                                            int16_t* __restrict__ pol, unsigned long long* __restrict__ tailmax,
                                            unsigned char* smem) {
  constexpr int NG = 64 / G;
  const int lane = threadIdx.x & 63, g = lane / G, gl = lane % G;
  const uint32_t s = tile * NG + g;
  MT* tab = reinterpret_cast<MT*>(smem) + g * P.gsl;
  const bool inside = s < (uint32_t)P.n_x;
  const uint8_t lb = inside ? label[s] : (uint8_t)LBL_ZERO;
  const bool active = inside && lb == LBL_FREE;
  if (inside && !active && gl == 0) {
    Vout[s] = (lb == LBL_ONE) ? VO(1) : VO(0);
    if (pol) pol[s] = -1;
  }
  double x[N];
  state_centre<N>(P, inside ? s : 0u, x);
  typename Dyn<KIND, N>::State st;
  Dyn<KIND, N>::prep(P, x, st);
  double isc[N];
  state_isc<N>(P, x, isc);
  double prev[N];
  int o[N];
  double wmem[TAIL ? N : 1], gmem[TAIL ? N : 1];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    prev[i] = __builtin_nan("");
    o[i] = 0;
  }
  // lane space: the dimensions from nout on, flattened (last fastest); a
  // lane's first index gl and the stride G as mixed-radix digits, so the
  // lane steps through its indices with carries instead of divisions
  const int nout = P.grp_nout;
  int ls = 1;
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i >= nout) ls *= P.L[i];
  int kin0[N], kinc[N];
  {
    int rr = gl, rg = G;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
      if (i >= nout) {
        kin0[i] = rr % P.L[i];
        rr /= P.L[i];
        kinc[i] = rg % P.L[i];
        rg /= P.L[i];
      } else {
        kin0[i] = 0;
        kinc[i] = 0;
      }
    }
  }
  InputWalk iw;
  iw.reset();
  AT best = AT(-1), qmin = AT(0);
  int arg = 0, wd = 0;
  double tmax = 0.0;
  for (int r = 0; r < P.n_rows; ++r) {
    double uv[AMY_MAXI], mu[N];
    iw.values(P, uv);
    Dyn<KIND, N>::apply(P, st, x, uv, mu);
    double win = 1.0, grid = 1.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (mu[i] != prev[i]) {
        const Win w = window_1d(P, i, mu[i], GEN ? isc[i] : 1.0);
        o[i] = w.o;
        prev[i] = mu[i];
        if (active)
          for (int k = gl; k < P.L[i]; k += G) tab[P.goff[i] + k] = slot_mass<MT, GEN>(P, i, w, k, mu[i], isc[i]);
        if constexpr (TAIL) {
          if constexpr (GEN) win_grid_mass_gen(P, i, w, wmem[i], gmem[i], mu[i], isc[i]);
          else win_grid_mass(P, i, w, wmem[i], gmem[i]);
        }
      }
      if constexpr (TAIL) {
        win *= wmem[i];
        grid *= gmem[i];
      }
    }
    __syncthreads();  // tables visible to the whole group (one wave per block)
    int64_t base = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) base += (int64_t)o[i] * P.stride[i];
    AT acc = AT(0), cmp = AT(0);
    if (active) {
      int kin[N];
#pragma unroll
      for (int i = 0; i < N; ++i) kin[i] = kin0[i];
      for (int j = gl; j < ls; j += G) {
        AT mi = AT(1);
#pragma unroll
        for (int i = 0; i < N; ++i)
          if (i >= nout) mi = mi * AT(tab[P.goff[i] + kin[i]]);
        const AT sj = gsum<0, N, MT, AT, VI>(P, nout, tab, kin, Vin, base);
        if constexpr (COMP) {
          const AT y = mi * sj - cmp;
          const AT s2 = acc + y;
          cmp = (s2 - acc) - y;
          acc = s2;
        } else {
          acc = fma_(mi, sj, acc);
        }
        // kin += the digits of G (each digit sum stays below 2 L_i)
        int carry = 0;
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
          if (i >= nout) {
            const int k = kin[i] + kinc[i] + carry;
            carry = k >= P.L[i] ? 1 : 0;
            kin[i] = carry ? k - P.L[i] : k;
          }
        }
      }
    }
    // sum of the group's partials (butterfly inside each group of G lanes)
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    qmin = (wd == 0 || acc < qmin) ? acc : qmin;
    if (++wd == P.n_w) {
      wd = 0;
      if (qmin > best) {
        best = qmin;
        arg = r / P.n_w;
      }
    }
    if constexpr (TAIL)
      if (active) tmax = fmax(tmax, grid - win);
    __syncthreads();  // the group's tables may be rebuilt for the next input
    iw.next(P);
  }
  if (active && gl == 0) {
    Vout[s] = VO(best);
    if (pol) pol[s] = (int16_t)arg;
  }
  if constexpr (TAIL) {
    wave_max_to(tmax, tailmax);
  }
}
