// amy_fixed.hip -- Bellman sweep specialised to a compile-time window shape.
//
// Same row algorithm as k_sweep_otf (one lane per state, inputs walked in
// the lane, running max / argmax, cached or memoised 1-D tables), with the
// window lengths L_0..L_{n-1} known at compile time:
//   * every window loop is unrolled, so all gathers of a row are issued
//     back to back (memory-level parallelism instead of one load in flight);
//   * the 1-D masses of the current row live in registers (cached tables are
//     copied from LDS once per input);
//   * V is read with buffer loads: a per-lane 32-bit byte offset (the
//     window origin), a uniform SGPR offset per outer window index, and the
//     innermost index as an immediate -- no VALU address arithmetic, and
//     the hardware merges consecutive innermost loads into dwordx2/x3/x4.
// Shapes are instantiated for the workload families' windows; any other
// shape runs the generic kernel.
#include <hip/hip_runtime.h>

#include "amy_device.hpp"
#include "amy_kernels.hpp"

#define FIX_BLOCK 64

template <int BLOCK, int... Ls>
struct ShapeT {
  static constexpr int N = sizeof...(Ls);
  static constexpr int L[N] = {Ls...};
  static constexpr int max_of() {
    int m = 0;
    for (int i = 0; i < N; ++i) m = L[i] > m ? L[i] : m;
    return m;
  }
  static constexpr int LMAX = max_of();
  // cells of the window below level d
  static constexpr int inner(int d) {
    int v = 1;
    for (int i = d; i < N; ++i) v *= L[i];
    return v;
  }
  // outermost level whose sub-window holds at most BLOCK_LOADS gathers: the
  // iterations of the level above are issued as separate blocks
  static constexpr int BLOCK_LOADS = BLOCK;
  static constexpr int block_level() {
    int d = 0;
    while (d < N - 1 && inner(d) > BLOCK_LOADS) ++d;
    return d;
  }
  static constexpr int BL = block_level();
};

// Raw buffer view of a V vector (offsets in bytes; out-of-range reads give 0).
template <class VT>
struct VBuf {
  using value_type = VT;
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ VBuf(const VT* p, uint32_t n)
      : r(__builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(n * (uint32_t)sizeof(VT)), 0x00020000)) {}
  __device__ __forceinline__ VT load(uint32_t voff, uint32_t soff) const;
  // byte step of one cell along dimension D
  template <int D>
  __device__ __forceinline__ uint32_t step(const DevProblem& P) const {
    return (uint32_t)P.stride[D] * (uint32_t)sizeof(VT);
  }
};
template <>
__device__ __forceinline__ float VBuf<float>::load(uint32_t voff, uint32_t soff) const {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double VBuf<double>::load(uint32_t voff, uint32_t soff) const {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

// n consecutive values from byte offset voff + soff into v[0 .. n), in
// 8-byte loads where they fit.  (This compiler lowers the 96- and 128-bit
// raw buffer load builtins, and element access on the 64-bit one's vector
// result, to a single dword load; only whole-value casts of the 64-bit
// load are used.)
template <class VT, int n>
__device__ __forceinline__ void vbuf_run(const VBuf<VT>& vb, uint32_t voff, uint32_t soff, VT* v) {
  int t = 0;
  if constexpr (sizeof(VT) == 4) {
#pragma unroll
    for (; t + 2 <= n; t += 2) {
      // whole-value cast: extracting the builtin's vector elements is also miscompiled
      const uint64_t q = __builtin_bit_cast(
          uint64_t, __builtin_amdgcn_raw_buffer_load_b64(vb.r, (int)(voff + (uint32_t)(t * 4)), (int)soff, 0));
      v[t] = __builtin_bit_cast(float, (uint32_t)q);
      v[t + 1] = __builtin_bit_cast(float, (uint32_t)(q >> 32));
    }
  }
#pragma unroll
  for (; t < n; ++t) v[t] = vb.load(voff + (uint32_t)(t * sizeof(VT)), soff);
}

// n consecutive cells of V from a V source, as wide as the source allows.
template <int n, class VT>
__device__ __forceinline__ void v_run(const VBuf<VT>& vb, uint32_t voff, uint32_t soff, VT* v) {
  vbuf_run<VT, n>(vb, voff, soff, v);
}
template <int n, class VS>
__device__ __forceinline__ void v_run(const VS& vs, uint32_t voff, uint32_t soff, typename VS::value_type* v) {
#pragma unroll
  for (int t = 0; t < n; ++t) v[t] = vs.load(voff + (uint32_t)(t * sizeof(typename VS::value_type)), soff);
}

// 1-D masses of an L-slot window into registers (same edges as dim_table).
template <class MT, int L>
__device__ __forceinline__ void fixed_table(const DevProblem& P, int i, const Win& w, MT* m) {
  double zp = edge_z(P, i, w, min(max(w.o, w.jlo), w.b));
  MT ep = ec_of(zp, MT());
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const double z = edge_z(P, i, w, min(max(w.o + k + 1, w.jlo), w.b));
    const MT e = ec_of(z, MT());
    m[k] = mass_of(zp, ep, z, e);
    zp = z;
    ep = e;
  }
}

template <class SH, class MT>
struct FixedRow {
  MT m[SH::N][SH::LMAX];
  uint32_t o[SH::N];
  double prev[SH::N];
  double wm[SH::N], gm[SH::N];
};

// Tables and window origin of dimension I for the current input.
template <int I, class SH, class MT, bool TAIL>
__device__ __forceinline__ void dim_step(const DevProblem& P, const InputWalk& iw, const double* mu,
                                         const LaneLds<MT>& S, FixedRow<SH, MT>& R, uint32_t& base,
                                         double& win, double& grid) {
  if constexpr (I < SH::N) {
    constexpr int L = SH::L[I];
    if (P.ccount[I] > 0) {
      const int c = combo_index(P, I, iw);
      const MT* tp = S.tab + (P.toff[I] + c * L) * FIX_BLOCK;
#pragma unroll
      for (int k = 0; k < L; ++k) R.m[I][k] = tp[k * FIX_BLOCK];
      R.o[I] = (uint32_t)S.org[(P.ooff[I] + c) * FIX_BLOCK];
      if constexpr (TAIL) {
        win *= S.wg[(2 * (P.ooff[I] + c)) * FIX_BLOCK];
        grid *= S.wg[(2 * (P.ooff[I] + c) + 1) * FIX_BLOCK];
      }
    } else {
      if (mu[I] != R.prev[I]) {
        const Win w = window_1d(P, I, mu[I]);
        R.o[I] = (uint32_t)w.o;
        R.prev[I] = mu[I];
        fixed_table<MT, L>(P, I, w, R.m[I]);
        if constexpr (TAIL) win_grid_mass(P, I, w, R.wm[I], R.gm[I]);
      }
      if constexpr (TAIL) {
        win *= R.wm[I];
        grid *= R.gm[I];
      }
    }
    base += R.o[I] * (uint32_t)P.stride[I];
    dim_step<I + 1, SH, MT, TAIL>(P, iw, mu, S, R, base, win, grid);
  }
}

// Window contraction with compile-time lengths; soff accumulates the
// uniform byte offset of the outer indices, voff is the lane's origin.
// Levels below SH::BL are unrolled (their gathers issue together); the
// levels above are loops, one gather block per iteration, which bounds the
// registers a row needs.
// VS is the source of V: VBuf (global memory, the grid's strides) or VLds
// (a box of V staged in LDS, the box's strides).
template <int D, class SH, class MT, class AT, class VS, bool COMP, int LL = 0>
__device__ __forceinline__ AT contract_fixed(const DevProblem& P, const FixedRow<SH, MT>& R,
                                             const VS& vb, uint32_t voff, uint32_t soff,
                                             const MT* ll = nullptr);

// LL > 0: the loop levels' masses are also in the thread's LDS slot ll
// ([level * LMAX + k][thread], LL threads) and are read from there by index.
template <int D, class SH, class MT, class AT, bool COMP, int LL>
__device__ __forceinline__ void accum_step(const FixedRow<SH, MT>& R, int k, AT inner, AT& acc, AT& c,
                                           const MT* ll);

template <int D, class SH, class MT, class AT, class VS, bool COMP, int LL = 0>
__device__ __forceinline__ void contract_step(const DevProblem& P, const FixedRow<SH, MT>& R,
                                              const VS& vb, uint32_t voff, uint32_t soff, int k,
                                              AT& acc, AT& c, const MT* ll) {
  AT inner;
  if constexpr (D == SH::N - 1) {
    inner = AT(vb.load(voff + (uint32_t)(k * sizeof(typename VS::value_type)), soff));
  } else {
    inner = contract_fixed<D + 1, SH, MT, AT, VS, COMP, LL>(P, R, vb, voff,
                                                            soff + (uint32_t)k * vb.template step<D>(P), ll);
  }
  accum_step<D, SH, MT, AT, COMP, LL>(R, k, inner, acc, c, ll);
}

// The value of v, hidden from the optimiser: the select chain below then
// stays a chain of selects instead of being folded back into an indexed
// access of the row's mass array, which would put that array in scratch
// memory (an empty asm statement: no instruction is emitted).
template <class T>
__device__ __forceinline__ T opaque_value(T v) {
  asm("" : "+v"(v));
  return v;
}

// acc += mass of slot k of level D times inner (compensated at level 0).
template <int D, class SH, class MT, class AT, bool COMP, int LL>
__device__ __forceinline__ void accum_step(const FixedRow<SH, MT>& R, int k, AT inner, AT& acc, AT& c,
                                           const MT* ll) {
  // mass of slot k; in a loop level k is a uniform register, so pick it
  // with selects (or from LDS) rather than an indexed register access
  MT mk;
  if constexpr (D < SH::BL) {
    if constexpr (LL > 0) {
      mk = ll[(D * SH::LMAX + k) * LL];
    } else {
      mk = opaque_value(R.m[D][0]);
#pragma unroll
      for (int j = 1; j < SH::L[D]; ++j) mk = (k == j) ? opaque_value(R.m[D][j]) : mk;
    }
  } else {
    mk = R.m[D][k];
  }
  if constexpr (COMP && D == 0) {
    const AT y = AT(mk) * inner - c;
    const AT s2 = acc + y;
    c = (s2 - acc) - y;
    acc = s2;
  } else {
    acc = fma_(AT(mk), inner, acc);
  }
}

template <int D, class SH, class MT, class AT, class VS, bool COMP, int LL>
__device__ __forceinline__ AT contract_fixed(const DevProblem& P, const FixedRow<SH, MT>& R,
                                             const VS& vb, uint32_t voff, uint32_t soff, const MT* ll) {
  constexpr int L = SH::L[D];
  AT acc = AT(0), c = AT(0);
  if constexpr (D < SH::BL) {
#pragma clang loop unroll(disable)
    for (int k = 0; k < L; ++k) contract_step<D, SH, MT, AT, VS, COMP, LL>(P, R, vb, voff, soff, k, acc, c, ll);
  } else if constexpr (D == SH::N - 1) {
    // the innermost run of L cells is contiguous in V: load it whole
    typename VS::value_type v[L];
    v_run<L>(vb, voff, soff, v);
#pragma unroll
    for (int k = 0; k < L; ++k) accum_step<D, SH, MT, AT, COMP, LL>(R, k, AT(v[k]), acc, c, ll);
  } else {
#pragma unroll
    for (int k = 0; k < L; ++k) contract_step<D, SH, MT, AT, VS, COMP, LL>(P, R, vb, voff, soff, k, acc, c, ll);
  }
  return acc;
}

template <int KIND, class SH, class MT, class AT, class VI, class VO, bool COMP, bool TAIL>
__global__ void __launch_bounds__(FIX_BLOCK) k_sweep_fixed(DevProblem P, const VI* __restrict__ Vin,
                                                           VO* __restrict__ Vout,
                                                           const uint8_t* __restrict__ label,
                                                           int16_t* __restrict__ pol,
                                                           unsigned long long* __restrict__ tailmax) {
  constexpr int N = SH::N;
  extern __shared__ __align__(16) unsigned char smem[];
  const LaneLds<MT> S(P, smem, threadIdx.x);
  const uint32_t s = xcd_block(blockIdx.x, gridDim.x) * FIX_BLOCK + threadIdx.x;
  double tmax = 0.0;
  if (s < (uint32_t)P.n_x) {
    const uint8_t lb = label[s];
    if (lb != LBL_FREE) {
      Vout[s] = (lb == LBL_ONE) ? VO(1) : VO(0);
      if (pol) pol[s] = -1;
    } else {
      double x[N];
      state_centre<N>(P, s, x);
      typename Dyn<KIND, N>::State st;
      Dyn<KIND, N>::prep(P, x, st);
      build_cached<KIND, N, MT, TAIL, FIX_BLOCK>(P, st, x, nullptr, S);
      const VBuf<VI> vb(Vin, (uint32_t)P.n_x);
      FixedRow<SH, MT> R;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        R.prev[i] = __builtin_nan("");
        R.o[i] = 0;
      }
      InputWalk iw;
      iw.reset();
      AT best = AT(-1);
      int arg = 0;
      for (int u = 0; u < P.n_u; ++u) {
        double uv[AMY_MAXI], mu[N];
        iw.values(P, uv);
        Dyn<KIND, N>::apply(P, st, x, uv, mu);
        uint32_t base = 0;
        double win = 1.0, grid = 1.0;
        dim_step<0, SH, MT, TAIL>(P, iw, mu, S, R, base, win, grid);
        if constexpr (TAIL) tmax = fmax(tmax, grid - win);
        const AT q = contract_fixed<0, SH, MT, AT, VBuf<VI>, COMP>(P, R, vb, base * (uint32_t)sizeof(VI), 0u);
        if (q > best) {
          best = q;
          arg = u;
        }
        iw.next(P);
      }
      Vout[s] = VO(best);
      if (pol) pol[s] = (int16_t)arg;
    }
  }
  if constexpr (TAIL) {
    wave_max_to(tmax, tailmax);
  }
}

// FP64 row tails alone, for the first step of a solve whose sweep reads the
// shared relative tables (that sweep runs after it).  Per state, the cached
// dimensions' kept-window and grid masses are computed once per input-digit
// combination into LDS ([2 x slot][lane] doubles, no mass tables), the
// others per input when their mean changes; each row's products are taken
// in dimension order with the same window rule and mass routine as the fused
// first step, so the max is that step's, bit for bit.
template <int KIND, int N>
__global__ void __launch_bounds__(FIX_BLOCK) k_tail_cached(DevProblem P, const uint8_t* __restrict__ label,
                                                           unsigned long long* __restrict__ tailmax) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* wg = reinterpret_cast<double*>(smem) + threadIdx.x;
  const uint32_t s = xcd_block(blockIdx.x, gridDim.x) * FIX_BLOCK + threadIdx.x;
  double tmax = 0.0;
  if (s < (uint32_t)P.n_x && label[s] == LBL_FREE) {
    double x[N];
    state_centre<N>(P, s, x);
    typename Dyn<KIND, N>::State st;
    Dyn<KIND, N>::prep(P, x, st);
    bool all_cached = true;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      all_cached = all_cached && P.ccount[i] > 0;
      for (int c = 0; c < P.ccount[i]; ++c) {
        InputWalk iw;
        combo_digits(P, i, c, iw);
        double uv[AMY_MAXI], mu[N];
        iw.values(P, uv);
        Dyn<KIND, N>::apply(P, st, x, uv, mu);
        double m_i = mu[0];
#pragma unroll
        for (int d = 1; d < N; ++d)
          if (d == i) m_i = mu[d];
        const Win w = window_1d(P, i, m_i);
        double wm, gm;
        win_grid_mass(P, i, w, wm, gm);
        wg[(2 * (P.ooff[i] + c)) * FIX_BLOCK] = wm;
        wg[(2 * (P.ooff[i] + c) + 1) * FIX_BLOCK] = gm;
      }
    }
    double prev[N], pw[N], pg[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      prev[i] = __builtin_nan("");
      pw[i] = pg[i] = 0.0;
    }
    InputWalk iw;
    iw.reset();
    for (int u = 0; u < P.n_u; ++u) {
      double mu[N];
#pragma unroll
      for (int i = 0; i < N; ++i) mu[i] = 0.0;
      if (!all_cached) {
        double uv[AMY_MAXI];
        iw.values(P, uv);
        Dyn<KIND, N>::apply(P, st, x, uv, mu);
      }
      double win = 1.0, grid = 1.0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        if (P.ccount[i] > 0) {
          const int c = combo_index(P, i, iw);
          win *= wg[(2 * (P.ooff[i] + c)) * FIX_BLOCK];
          grid *= wg[(2 * (P.ooff[i] + c) + 1) * FIX_BLOCK];
        } else {
          if (mu[i] != prev[i]) {
            const Win w = window_1d(P, i, mu[i]);
            win_grid_mass(P, i, w, pw[i], pg[i]);
            prev[i] = mu[i];
          }
          win *= pw[i];
          grid *= pg[i];
        }
      }
      tmax = fmax(tmax, grid - win);
      iw.next(P);
    }
  }
  wave_max_to(tmax, tailmax);
}

// ---------------------------------------------------------------- factored
//
// Inputs are walked with the last digit fastest.  When that digit moves only
// the innermost dimension's window (dimension N-1 depends on the last digit
// alone, and no other dimension depends on it; the unicycle: the turn rate
// moves the heading, the speed moves x and y), every input of one
// combination of the slower digits shares the outer dimensions' masses and
// window.  The outer contraction is then done once per slow combination for
// each innermost cell that the fast digit's windows can reach -- U cells
// from the smallest of their origins -- giving A[t]; the row value of each
// fast digit is the L_{N-1}-term sum of its innermost masses against A.
// The host admits a problem only when the union of the fast digit's windows
// is provably at most U cells long and dimension N-1's tables are cached.
// Outer contraction for the U innermost cells from the union's origin:
// acc[t] = sum over dimensions D .. N-2 of their masses times V.  Level 0 is
// a loop (its mass read from LDS per iteration); the levels below it are
// unrolled with their masses in registers, so every gather of one level-0
// slice issues back to back.
template <int D, class SH, int U, class MT, class AT, class VS>
__device__ __forceinline__ void contract_fac_in(const DevProblem& P, const FixedRow<SH, MT>& R, const VS& vb,
                                                uint32_t voff, uint32_t soff, AT (&acc)[U]) {
  using VT = typename VS::value_type;
#pragma unroll
  for (int t = 0; t < U; ++t) acc[t] = AT(0);
#pragma unroll
  for (int k = 0; k < SH::L[D]; ++k) {
    const uint32_t sk = soff + (uint32_t)k * vb.template step<D>(P);
    AT inner[U];
    if constexpr (D == SH::N - 2) {
      VT v[U];
      v_run<U>(vb, voff, sk, v);
#pragma unroll
      for (int t = 0; t < U; ++t) inner[t] = AT(v[t]);
    } else {
      contract_fac_in<D + 1, SH, U, MT, AT, VS>(P, R, vb, voff, sk, inner);
    }
#pragma unroll
    for (int t = 0; t < U; ++t) acc[t] = fma_(AT(R.m[D][k]), inner[t], acc[t]);
  }
}

template <class SH, int U, class MT, class AT, class VS, bool COMP>
__device__ __forceinline__ void contract_fac(const DevProblem& P, const FixedRow<SH, MT>& R, const MT* m0,
                                             const VS& vb, uint32_t voff, AT (&acc)[U]) {
  using VT = typename VS::value_type;
  AT c[U];
#pragma unroll
  for (int t = 0; t < U; ++t) acc[t] = c[t] = AT(0);
#pragma clang loop unroll(disable)
  for (int k = 0; k < SH::L[0]; ++k) {
    const uint32_t soff = (uint32_t)k * vb.template step<0>(P);
    AT inner[U];
    if constexpr (SH::N == 2) {
#pragma unroll
      for (int t = 0; t < U; ++t) inner[t] = AT(vb.load(voff + (uint32_t)(t * sizeof(VT)), soff));
    } else {
      contract_fac_in<1, SH, U, MT, AT, VS>(P, R, vb, voff, soff, inner);
    }
    const AT mk = AT(m0[k * FIX_BLOCK]);
#pragma unroll
    for (int t = 0; t < U; ++t) {
      if constexpr (COMP) {
        const AT y = mk * inner[t] - c[t];
        const AT s2 = acc[t] + y;
        c[t] = (s2 - acc[t]) - y;
        acc[t] = s2;
      } else {
        acc[t] = fma_(mk, inner[t], acc[t]);
      }
    }
  }
}

// Masses and window origins of the outer dimensions 0 .. N-2 for the
// current combination of the slow digits: cached tables are read from LDS;
// the others are built from the mean mu.  Dimension 0's masses are left in
// LDS (m0: its cached table, or the lane's slot t0 when it is built here),
// the others go to registers.
template <int I, class SH, class MT, bool TAIL>
__device__ __forceinline__ void fac_outer(const DevProblem& P, const InputWalk& iw, const LaneLds<MT>& S,
                                          MT* t0, const double* mu, FixedRow<SH, MT>& R, const MT*& m0,
                                          uint32_t& base, double& win, double& grid) {
  if constexpr (I < SH::N - 1) {
    constexpr int L = SH::L[I];
    int o;
    if (P.ccount[I] > 0) {
      const int c = combo_index(P, I, iw);
      const MT* tp = S.tab + (P.toff[I] + c * L) * FIX_BLOCK;
      if constexpr (I == 0) {
        m0 = tp;
      } else {
#pragma unroll
        for (int k = 0; k < L; ++k) R.m[I][k] = tp[k * FIX_BLOCK];
      }
      o = S.org[(P.ooff[I] + c) * FIX_BLOCK];
      if constexpr (TAIL) {
        win *= S.wg[(2 * (P.ooff[I] + c)) * FIX_BLOCK];
        grid *= S.wg[(2 * (P.ooff[I] + c) + 1) * FIX_BLOCK];
      }
    } else {
      const Win w = window_1d(P, I, mu[I]);
      fixed_table<MT, L>(P, I, w, R.m[I]);
      if constexpr (I == 0) {
#pragma unroll
        for (int k = 0; k < L; ++k) t0[k * FIX_BLOCK] = R.m[0][k];
        m0 = t0;
      }
      o = w.o;
      if constexpr (TAIL) {
        double wm, gm;
        win_grid_mass(P, I, w, wm, gm);
        win *= wm;
        grid *= gm;
      }
    }
    base += (uint32_t)o * (uint32_t)P.stride[I];
    fac_outer<I + 1, SH, MT, TAIL>(P, iw, S, t0, mu, R, m0, base, win, grid);
  }
}

template <int KIND, class SH, int U, class MT, class AT, class VI, class VO, bool COMP, bool TAIL>
__global__ void __launch_bounds__(FIX_BLOCK) k_sweep_fac(DevProblem P, const VI* __restrict__ Vin,
                                                         VO* __restrict__ Vout, const uint8_t* __restrict__ label,
                                                         int16_t* __restrict__ pol,
                                                         unsigned long long* __restrict__ tailmax,
                                                         uint32_t t0_off) {
  constexpr int N = SH::N;
  constexpr int F = N - 1;
  constexpr int LF = SH::L[F];
  static_assert(N >= 2 && LF <= U, "factored sweep shape");
  extern __shared__ __align__(16) unsigned char smem[];
  const LaneLds<MT> S(P, smem, threadIdx.x);
  const uint32_t s = xcd_block(blockIdx.x, gridDim.x) * FIX_BLOCK + threadIdx.x;
  double tmax = 0.0;
  if (s < (uint32_t)P.n_x) {
    const uint8_t lb = label[s];
    if (lb != LBL_FREE) {
      Vout[s] = (lb == LBL_ONE) ? VO(1) : VO(0);
      if (pol) pol[s] = -1;
    } else {
      double x[N];
      state_centre<N>(P, s, x);
      typename Dyn<KIND, N>::State st;
      Dyn<KIND, N>::prep(P, x, st);
      build_cached<KIND, N, MT, TAIL, FIX_BLOCK>(P, st, x, nullptr, S);
      const VBuf<VI> vb(Vin, (uint32_t)P.n_x);
      const int fd = P.m - 1;                    // the fast digit
      const int nf = P.ucount[fd];
      const int fm = P.dep_mult[F][fd];          // its step in dimension F's combo index
      // smallest innermost origin over the fast digit
      int omin = S.org[P.ooff[F] * FIX_BLOCK];
      for (int f = 1; f < nf; ++f) omin = min(omin, S.org[(P.ooff[F] + f * fm) * FIX_BLOCK]);
      FixedRow<SH, MT> R;
      MT* t0 = reinterpret_cast<MT*>(smem + t0_off) + threadIdx.x;
      bool all_cached = true;
#pragma unroll
      for (int i = 0; i < F; ++i) all_cached = all_cached && P.ccount[i] > 0;
      InputWalk iw;
      iw.reset();
      AT best = AT(-1);
      int arg = 0, u = 0;
      const int nslow = P.n_u / nf;
      for (int sc = 0; sc < nslow; ++sc) {
        uint32_t base = (uint32_t)omin;
        double win = 1.0, grid = 1.0;
        double mu[N];
        if (!all_cached) {  // the slow digits' mean (the fast digit is 0 here)
          double uv[AMY_MAXI];
          iw.values(P, uv);
          Dyn<KIND, N>::apply(P, st, x, uv, mu);
        }
        const MT* m0 = nullptr;
        fac_outer<0, SH, MT, TAIL>(P, iw, S, t0, mu, R, m0, base, win, grid);
        AT A[U];
        contract_fac<SH, U, MT, AT, VBuf<VI>, COMP>(P, R, m0, vb, base * (uint32_t)sizeof(VI), A);
        for (int f = 0; f < nf; ++f, ++u) {
          const int c = f * fm;
          const MT* tp = S.tab + (P.toff[F] + c * LF) * FIX_BLOCK;
          const int d = min(S.org[(P.ooff[F] + c) * FIX_BLOCK] - omin, U - LF);
          AT q = AT(0);
#pragma unroll
          for (int k = 0; k < LF; ++k) {
            AT a = A[k];
#pragma unroll
            for (int j = 1; j <= U - LF; ++j) a = (d == j) ? A[j + k] : a;
            q = fma_(AT(tp[k * FIX_BLOCK]), a, q);
          }
          if constexpr (TAIL) {
            const double wf = S.wg[(2 * (P.ooff[F] + c)) * FIX_BLOCK];
            const double gf = S.wg[(2 * (P.ooff[F] + c) + 1) * FIX_BLOCK];
            tmax = fmax(tmax, grid * gf - win * wf);
          }
          if (q > best) {
            best = q;
            arg = u;
          }
        }
        // next combination of the slow digits (the fast digit stays 0)
#pragma unroll
        for (int k = AMY_MAXI - 1; k >= 0; --k) {
          if (k < fd) {
            if (++iw.dig[k] < P.ucount[k]) break;
            iw.dig[k] = 0;
          }
        }
      }
      Vout[s] = VO(best);
      if (pol) pol[s] = (int16_t)arg;
    }
  }
  if constexpr (TAIL) {
    wave_max_to(tmax, tailmax);
  }
}

// --------------------------------------------------- shared relative tables
//
// For the unicycle the mean minus the state's own cell centre is
// (tau v cos th, tau v sin th, tau omega): in x and y it depends only on the
// heading cell and the speed, in the heading only on the turn rate.  The
// 1-D masses of a window relative to the state's cell are then the same for
// every state with that heading cell, so they are built once per solve
// (k_rel_build) and read by the steps without the FP64 tail (k_sweep_rel).
// A state's window origin is its cell plus the relative origin, clamped to
// the grid as the per-state rule clamps it; slots are matched to the
// relative masses by the clamp's shift, and cells outside the grid or the
// kept range get mass 0 -- the same cells and masses as the per-state rule.
template <int KIND, int N>
struct RelDrift {
  static constexpr bool ok = false;
};

template <>
struct RelDrift<AMY_DYN_UNICYCLE_, 3> {
  static constexpr bool ok = true;
  static constexpr int ctx(int i) { return i < 2 ? 2 : -1; }
  // mean of dimension i minus the state's cell centre; xc: the centre of
  // the context dimension's cell
  __device__ static double drift(const DevProblem& P, int i, double xc, const double* u) {
    const double tau = P.params[0];
    if (i == 2) return tau * u[1];
    const double a = tau * u[0];
    return i == 0 ? a * cos(xc) : a * sin(xc);
  }
};

#define REL_SLOTS AMY_TABLE_SLOTS  // masses per table entry

template <int KIND, int N, class MT>
__global__ void __launch_bounds__(64) k_rel_build(DevProblem P, MT* __restrict__ rm, int32_t* __restrict__ rlo) {
  const int e = blockIdx.x * 64 + threadIdx.x;
  if (e >= P.rel_entries) return;
  int i = 0;
#pragma unroll
  for (int d = 1; d < N; ++d)
    if (e >= P.rel_off[d]) i = d;
  const int jc = e - P.rel_off[i];
  const int j = jc / P.rcount[i], c = jc % P.rcount[i];
  InputWalk iw;
#pragma unroll
  for (int k = 0; k < AMY_MAXI; ++k) {
    const int mlt = P.rmult[i][k];
    iw.dig[k] = (k < P.m && mlt > 0) ? (c / mlt) % P.ucount[k] : 0;
  }
  double u[AMY_MAXI];
  iw.values(P, u);
  const int cx = P.rctx[i];
  const double xc = cx >= 0 ? P.lo[cx] + ((double)j + 0.5) * P.h[cx] : 0.0;
  const double dr = RelDrift<KIND, N>::drift(P, i, xc, u);
  // kept cells r (relative to the state's cell): the centre rule keeps
  // |r h - drift| <= x*; the intersect rule keeps every cell meeting
  // [drift - x*, drift + x*], i.e. (r - 1/2) h < drift + x* and
  // (r + 1/2) h > drift - x*
  const int L = P.L[i];
  const bool inter = P.wrule == 1;
  const int r0 = inter ? (int)floor((dr - P.xstar[i]) * P.inv_h[i] + 0.5)
                       : (int)ceil((dr - P.xstar[i]) * P.inv_h[i]);
  int r1 = inter ? (int)ceil((dr + P.xstar[i]) * P.inv_h[i] + 0.5) - 1 : (int)floor((dr + P.xstar[i]) * P.inv_h[i]);
  r1 = min(r1, r0 + L - 1);
  const int cnt = max(0, r1 - r0 + 1);
  // edge below relative cell r: z = ((r - 1/2) h - drift) / sigma
  double zp = (((double)r0 - 0.5) * P.h[i] - dr) * P.inv_sigma[i];
  MT ep = ec_of(zp, MT());
  for (int k = 0; k < REL_SLOTS; ++k) {
    MT mk = MT(0);
    if (k < cnt) {
      const double z = (((double)(r0 + k) + 0.5) * P.h[i] - dr) * P.inv_sigma[i];
      const MT ez = ec_of(z, MT());
      mk = mass_of(zp, ep, z, ez);
      zp = z;
      ep = ez;
    }
    rm[(int64_t)e * REL_SLOTS + k] = mk;
  }
  rlo[e] = r0;
}

// Outer dimensions from the relative tables, in two passes so that every
// dimension's loads are in flight together: rel_load fetches each entry's
// masses and relative origin, rel_place clamps the origin, shifts the masses
// of a clamped window (zero fill) and leaves dimension 0's in the lane's
// LDS slot t0.
template <int I, class SH, class MT>
__device__ __forceinline__ void rel_load(const DevProblem& P, const InputWalk& iw, const int* j,
                                         const MT* __restrict__ rm, const int32_t* __restrict__ rlo,
                                         FixedRow<SH, MT>& R, int* r) {
  if constexpr (I < SH::N - 1) {
    int c = 0;
#pragma unroll
    for (int k = 0; k < AMY_MAXI; ++k) c += iw.dig[k] * P.rmult[I][k];
    const int e = P.rel_off[I] + (P.rctx[I] >= 0 ? j[P.rctx[I]] : 0) * P.rcount[I] + c;
    const MT* tp = rm + (int64_t)e * REL_SLOTS;
#pragma unroll
    for (int k = 0; k < SH::L[I]; ++k) R.m[I][k] = tp[k];
    r[I] = j[I] + rlo[e];
    rel_load<I + 1, SH, MT>(P, iw, j, rm, rlo, R, r);
  }
}

template <int I, class SH, class MT>
__device__ __forceinline__ void rel_place(const DevProblem& P, const int* r, MT* t0, FixedRow<SH, MT>& R,
                                          uint32_t& base) {
  if constexpr (I < SH::N - 1) {
    constexpr int L = SH::L[I];
    const int o = min(max(r[I], 0), P.count[I] - L);
    const int sh = o - r[I];  // slot k holds relative cell k + sh
    if (sh != 0) {            // window clamped at a grid edge
      MT w[L];
#pragma unroll
      for (int k = 0; k < L; ++k) {
        w[k] = MT(0);
#pragma unroll
        for (int q = 0; q < L; ++q) w[k] = (k + sh == q) ? R.m[I][q] : w[k];
      }
#pragma unroll
      for (int k = 0; k < L; ++k) R.m[I][k] = w[k];
    }
    if constexpr (I == 0) {
#pragma unroll
      for (int k = 0; k < L; ++k) t0[k * FIX_BLOCK] = R.m[0][k];
    }
    base += (uint32_t)o * (uint32_t)P.stride[I];
    rel_place<I + 1, SH, MT>(P, r, t0, R, base);
  }
}

template <int KIND, class SH, int U, class MT, class AT, class VI, class VO, bool COMP>
__global__ void __launch_bounds__(FIX_BLOCK) k_sweep_rel(DevProblem P, const VI* __restrict__ Vin,
                                                         VO* __restrict__ Vout, const uint8_t* __restrict__ label,
                                                         int16_t* __restrict__ pol, const MT* __restrict__ rm,
                                                         const int32_t* __restrict__ rlo) {
  constexpr int N = SH::N;
  constexpr int F = N - 1;
  constexpr int LF = SH::L[F];
  static_assert(N >= 2 && LF <= U && SH::LMAX <= REL_SLOTS, "relative-table sweep shape");
  extern __shared__ __align__(16) unsigned char smem[];
  const int fd = P.m - 1, nf = P.ucount[fd], fm = P.rmult[F][fd];
  // the innermost dimension's tables are the same for every lane: one copy
  // per block in LDS after the lanes' dimension-0 slots
  MT* t0 = reinterpret_cast<MT*>(smem) + threadIdx.x;
  MT* thm = reinterpret_cast<MT*>(smem) + SH::L[0] * FIX_BLOCK;
  int32_t* thr = reinterpret_cast<int32_t*>(thm + nf * LF);
  for (int f = threadIdx.x; f < nf; f += FIX_BLOCK) {
    const int e = P.rel_off[F] + f * fm;
#pragma unroll
    for (int k = 0; k < LF; ++k) thm[f * LF + k] = rm[(int64_t)e * REL_SLOTS + k];
    thr[f] = rlo[e];
  }
  __syncthreads();
  const uint32_t s = xcd_block(blockIdx.x, gridDim.x) * FIX_BLOCK + threadIdx.x;
  if (s >= (uint32_t)P.n_x) return;
  const uint8_t lb = label[s];
  if (lb != LBL_FREE) {
    Vout[s] = (lb == LBL_ONE) ? VO(1) : VO(0);
    if (pol) pol[s] = -1;
    return;
  }
  int j[N];
  {
    uint32_t r = s;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
      j[i] = (int)(r % (uint32_t)P.count[i]);
      r /= (uint32_t)P.count[i];
    }
  }
  const VBuf<VI> vb(Vin, (uint32_t)P.n_x);
  const int nF = P.count[F];
  int omin = nF;
  for (int f = 0; f < nf; ++f) omin = min(omin, min(max(j[F] + thr[f], 0), nF - LF));
  FixedRow<SH, MT> R;
  InputWalk iw;
  iw.reset();
  AT best = AT(-1);
  int arg = 0, u = 0;
  const int nslow = P.n_u / nf;
  for (int sc = 0; sc < nslow; ++sc) {
    uint32_t base = (uint32_t)omin;
    int r[N];
    rel_load<0, SH, MT>(P, iw, j, rm, rlo, R, r);
    rel_place<0, SH, MT>(P, r, t0, R, base);
    AT A[U];
    contract_fac<SH, U, MT, AT, VBuf<VI>, COMP>(P, R, t0, vb, base * (uint32_t)sizeof(VI), A);
    for (int f = 0; f < nf; ++f, ++u) {
      const int g = j[F] + thr[f] - omin;  // A index of the first kept cell
      AT q = AT(0);
#pragma unroll
      for (int k = 0; k < LF; ++k) {
        const int t = g + k;
        AT a = A[0];
#pragma unroll
        for (int jj = 1; jj < U; ++jj) a = (t == jj) ? A[jj] : a;
        const bool ok = t >= 0 && t < U && omin + t < nF;
        const AT qk = fma_(AT(thm[f * LF + k]), a, q);
        q = ok ? qk : q;
      }
      if (q > best) {
        best = q;
        arg = u;
      }
    }
#pragma unroll
    for (int k = AMY_MAXI - 1; k >= 0; --k) {
      if (k < fd) {
        if (++iw.dig[k] < P.ucount[k]) break;
        iw.dig[k] = 0;
      }
    }
  }
  Vout[s] = VO(best);
  if (pol) pol[s] = (int16_t)arg;
}

// ---------------------------------------------------------- memoised tables
//
// A dimension whose mean reads few state coordinates (the room ring: its
// room and the two neighbours; the 7-D vehicle: at most four) has few
// distinct 1-D tables over the whole grid: one per (context cells, input
// digits).  k_memo_build runs the per-state code (mean, window, masses) once
// per such entry, with the context coordinates at their cell centres, so an
// entry holds exactly the bits a state with that context computes;
// k_sweep_memo (the steps without the FP64 tail) loads a row's tables
// instead of computing them.
template <class MT>
__device__ __forceinline__ MT origin_bits(int o) {
  if constexpr (sizeof(MT) == 8) return __builtin_bit_cast(MT, (int64_t)o);
  else return __builtin_bit_cast(MT, (int32_t)o);
}
template <class MT>
__device__ __forceinline__ int origin_of(MT v) {
  if constexpr (sizeof(MT) == 8) return (int)__builtin_bit_cast(int64_t, v);
  else return (int)__builtin_bit_cast(int32_t, v);
}

// Entry e is the record rm[e*REC .. e*REC+REC): the masses of its window, zeros,
// and the window origin's bits in the last slot; wg[2e], wg[2e+1]: its FP64
// kept-window and grid masses (the per-row tail's factors).
// GEN: the masses of the other noise models (one entry's tables cost a few
// hundred FP64 operations there, so memoising them matters most).
template <int KIND, int N, class MT, int REC, bool GEN>
__global__ void __launch_bounds__(64) k_memo_build(DevProblem P, MT* __restrict__ rm, double* __restrict__ wg) {
  const int e = blockIdx.x * 64 + threadIdx.x;
  if (e >= P.rel_entries) return;
  int i = 0;
#pragma unroll
  for (int d = 1; d < N; ++d)
    if (e >= P.rel_off[d]) i = d;
  const int idx = e - P.rel_off[i];
  const int c = idx % P.rcount[i];
  int cx = idx / P.rcount[i];
  double x[N];
#pragma unroll
  for (int d = 0; d < N; ++d) x[d] = P.lo[d] + 0.5 * P.h[d];
  for (int k = P.mctx_n[i] - 1; k >= 0; --k) {
    const int d = P.mctx[i][k];
    const int j = cx % P.count[d];
    cx /= P.count[d];
#pragma unroll
    for (int dd = 0; dd < N; ++dd)
      if (dd == d) x[dd] = P.lo[dd] + ((double)j + 0.5) * P.h[dd];
  }
  InputWalk iw;
#pragma unroll
  for (int k = 0; k < AMY_MAXI; ++k) {
    const int mlt = P.rmult[i][k];
    iw.dig[k] = (k < P.m && mlt > 0) ? (c / mlt) % P.ucount[k] : 0;
  }
  double u[AMY_MAXI], mu[N];
  iw.values(P, u);
  typename Dyn<KIND, N>::State st;
  Dyn<KIND, N>::prep(P, x, st);
  Dyn<KIND, N>::apply(P, st, x, u, mu);
  double m_i = mu[0];
#pragma unroll
  for (int dd = 1; dd < N; ++dd)
    if (dd == i) m_i = mu[dd];
  MT t[REC];
  const Win w = GEN ? dim_table_gen<MT>(P, i, m_i, t, 1, 1.0) : dim_table<MT>(P, i, m_i, t, 1);
  for (int k = P.L[i]; k < REC - 1; ++k) t[k] = MT(0);
  t[REC - 1] = origin_bits<MT>(w.o);
  MT* dst = rm + (int64_t)e * REC;
#pragma unroll
  for (int k = 0; k < REC; ++k) dst[k] = t[k];
  double wm, gm;
  if constexpr (GEN) win_grid_mass_gen(P, i, w, wm, gm, m_i, 1.0);
  else win_grid_mass(P, i, w, wm, gm);
  wg[2 * (int64_t)e] = wm;
  wg[2 * (int64_t)e + 1] = gm;
}

// FP64 row tails alone from the memoised kept-window and grid masses (wg,
// filled by k_memo_build), for the first step of a solve whose sweep forms
// none (the factored sweep on shared relative tables).  The memo entries
// hold the per-state code's masses for the state's own context, and each
// row multiplies them in dimension order as the per-state path does, so
// the max is that path's, bit for bit, at a few loads per row instead of
// the per-state FP64 means, windows and erfc's.  A state's entries (one per
// input-digit combination of each dimension, sum_i rcount_i of them) are
// first loaded into its own LDS column, so the input loop waits on no memory.
#define TAIL_MEMO_BLOCK 64
template <int N>
__global__ void __launch_bounds__(TAIL_MEMO_BLOCK) k_tail_memo(DevProblem P, const uint8_t* __restrict__ label,
                                                               const double* __restrict__ wg,
                                                               unsigned long long* __restrict__ tailmax) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2* ent0 = reinterpret_cast<double2*>(smem);  // [entry][lane]
  double2* ent = ent0 + threadIdx.x;
  const uint32_t s = xcd_block(blockIdx.x, gridDim.x) * TAIL_MEMO_BLOCK + threadIdx.x;
  double tmax = 0.0;
  if (s < (uint32_t)P.n_x && label[s] == LBL_FREE) {
    int j[N];
    uint32_t r = s;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
      j[i] = (int)(r % (uint32_t)P.count[i]);
      r /= (uint32_t)P.count[i];
    }
    int eoff[N];
    const double2* src[N];
    int off = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      int v = 0;
      for (int k = 0; k < P.mctx_n[i]; ++k) {
        int jk = j[0];
#pragma unroll
        for (int d = 1; d < N; ++d)
          if (d == P.mctx[i][k]) jk = j[d];
        v += jk * P.mmult[i][k];
      }
      src[i] = reinterpret_cast<const double2*>(wg) + ((int64_t)P.rel_off[i] + (int64_t)v * P.rcount[i]);
      eoff[i] = off;
      off += P.rcount[i];
    }
    // every entry straight from memory into the state's LDS column (the
    // load-to-LDS form writes lane l's 16 bytes at the given wave-uniform
    // base + 16 l, which is the [entry][lane] layout), all in flight at once
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int rc = P.rcount[i];
      for (int c = 0; c < rc; ++c)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src[i] + c),
                                         (__attribute__((address_space(3))) void*)(ent0 + (eoff[i] + c) * TAIL_MEMO_BLOCK),
                                         16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);  // the loads have landed in LDS
    // walk the inputs (last digit fastest) keeping each dimension's entry
    // index e_i = eoff_i + sum_k dig_k rmult_ik up to date with adds
    int dig[AMY_MAXI], e[N];
#pragma unroll
    for (int k = 0; k < AMY_MAXI; ++k) dig[k] = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) e[i] = eoff[i];
    for (int u = 0; u < P.n_u; ++u) {
      double win = 1.0, grid = 1.0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const double2 w2 = ent[e[i] * TAIL_MEMO_BLOCK];
        win *= w2.x;
        grid *= w2.y;
      }
      tmax = fmax(tmax, grid - win);
      bool carry = true;
#pragma unroll
      for (int k = AMY_MAXI - 1; k >= 0; --k) {
        if (carry && k < P.m) {
          if (++dig[k] >= P.ucount[k]) {
            dig[k] = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) e[i] -= (P.ucount[k] - 1) * P.rmult[i][k];
          } else {
            carry = false;
#pragma unroll
            for (int i = 0; i < N; ++i) e[i] += P.rmult[i][k];
          }
        }
      }
    }
  }
  wave_max_to(tmax, tailmax);
}

// Byte offset of the memoised tables' FP64 window and grid masses.
__host__ __device__ inline uint64_t memo_wg_offset(const DevProblem& P, int rec, uint64_t msz) {
  return ((uint64_t)P.rel_entries * (uint64_t)rec * msz + 255) & ~255ull;
}

template <class MT, int REC>
struct alignas(REC * sizeof(MT)) MemoRec {
  MT v[REC];
};

// Every dimension's record for the current input: masses and origin.  TAIL:
// also the products of the dimensions' FP64 window and grid masses, in
// dimension order (as the per-state path forms them).
template <int I, class SH, class MT, bool TAIL = false>
__device__ __forceinline__ void memo_load(const DevProblem& P, const InputWalk& iw, const int* cx,
                                          const MT* __restrict__ rm, FixedRow<SH, MT>& R, uint32_t& base,
                                          const double* __restrict__ wg = nullptr, double* win = nullptr,
                                          double* grid = nullptr) {
  if constexpr (I < SH::N) {
    constexpr int REC = amy_memo_rec(SH::LMAX);
    int c = 0;
#pragma unroll
    for (int k = 0; k < AMY_MAXI; ++k) c += iw.dig[k] * P.rmult[I][k];
    const int e = P.rel_off[I] + cx[I] * P.rcount[I] + c;
    const MemoRec<MT, REC> r = *reinterpret_cast<const MemoRec<MT, REC>*>(rm + (int64_t)e * REC);
#pragma unroll
    for (int k = 0; k < SH::L[I]; ++k) R.m[I][k] = r.v[k];
    R.o[I] = (uint32_t)origin_of<MT>(r.v[REC - 1]);
    base += R.o[I] * (uint32_t)P.stride[I];
    if constexpr (TAIL) {
      *win *= wg[2 * (int64_t)e];
      *grid *= wg[2 * (int64_t)e + 1];
    }
    memo_load<I + 1, SH, MT, TAIL>(P, iw, cx, rm, R, base, wg, win, grid);
  }
}

// State of lane `lane` of workgroup b.  With at least three dimensions whose
// three innermost counts are multiples of 4, and more than 8 cells in the
// innermost one, a workgroup takes a 4 x 4 x 4 tile of those dimensions
// (their windows overlap, so the gathers share cache lines); otherwise 64
// consecutive states (which already span a 2-D plane of the innermost
// dimensions when those are short).  j[]: the state's cells.
template <int N>
__device__ __forceinline__ uint32_t tiled_state(const DevProblem& P, uint32_t b, int lane, int* j) {
  bool tiled = N >= 3 && P.count[N - 1] > 8;
#pragma unroll
  for (int d = (N >= 3 ? N - 3 : 0); d < N; ++d) tiled = tiled && (P.count[d] & 3) == 0;
  uint32_t s = 0;
  if (tiled) {
    uint32_t r = b;
#pragma unroll
    for (int d = N - 1; d >= 0; --d) {
      const bool inner = d >= N - 3;
      const uint32_t td = inner ? (uint32_t)P.count[d] / 4u : (uint32_t)P.count[d];
      const uint32_t c = r % td;
      r /= td;
      const int part = d == N - 1 ? (lane & 3) : (d == N - 2 ? ((lane >> 2) & 3) : (lane >> 4));
      j[d] = inner ? (int)(c * 4u) + part : (int)c;
      s += (uint32_t)j[d] * (uint32_t)P.stride[d];
    }
    if (r != 0) s = 0xffffffffu;  // past the last tile
  } else {
    s = b * FIX_BLOCK + (uint32_t)lane;
    uint32_t r = s;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
      j[i] = (int)(r % (uint32_t)P.count[i]);
      r /= (uint32_t)P.count[i];
    }
  }
  return s;
}

template <int KIND, class SH, class MT, class AT, class VI, class VO, bool COMP>
__global__ void __launch_bounds__(FIX_BLOCK) k_sweep_memo(DevProblem P, const VI* __restrict__ Vin,
                                                          VO* __restrict__ Vout, const uint8_t* __restrict__ label,
                                                          int16_t* __restrict__ pol, const MT* __restrict__ rm) {
  constexpr int N = SH::N;
  int j[N];
  const uint32_t s = tiled_state<N>(P, xcd_block(blockIdx.x, gridDim.x), threadIdx.x, j);
  if (s >= (uint32_t)P.n_x) return;
  const uint8_t lb = label[s];
  if (lb != LBL_FREE) {
    Vout[s] = (lb == LBL_ONE) ? VO(1) : VO(0);
    if (pol) pol[s] = -1;
    return;
  }
  int cx[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    int v = 0;
    for (int k = 0; k < P.mctx_n[i]; ++k) {
      int jk = j[0];
#pragma unroll
      for (int d = 1; d < N; ++d)
        if (d == P.mctx[i][k]) jk = j[d];
      v += jk * P.mmult[i][k];
    }
    cx[i] = v;
  }
  const VBuf<VI> vb(Vin, (uint32_t)P.n_x);
  extern __shared__ __align__(16) unsigned char smem[];
  MT* ll = reinterpret_cast<MT*>(smem) + threadIdx.x;  // loop levels' masses
  FixedRow<SH, MT> R;
  InputWalk iw;
  iw.reset();
  AT best = AT(-1);
  int arg = 0;
  for (int u = 0; u < P.n_u; ++u) {
    uint32_t base = 0;
    memo_load<0, SH, MT>(P, iw, cx, rm, R, base);
#pragma unroll
    for (int d = 0; d < SH::BL; ++d)
#pragma unroll
      for (int k = 0; k < SH::LMAX; ++k)
        if (k < SH::L[d]) ll[(d * SH::LMAX + k) * FIX_BLOCK] = R.m[d][k];
    const AT q = contract_fixed<0, SH, MT, AT, VBuf<VI>, COMP, FIX_BLOCK>(P, R, vb, base * (uint32_t)sizeof(VI), 0u, ll);
    if (q > best) {
      best = q;
      arg = u;
    }
    iw.next(P);
  }
  Vout[s] = VO(best);
  if (pol) pol[s] = (int16_t)arg;
}

// ------------------------------------------------------- staged V boxes
//
// A workgroup of 256 threads takes a 1 x 4 x 4 x 4 x 4 tile of a 5-D grid.
// For each input the union of its threads' windows, which for the room ring
// (every mean moves less than one cell per cell of its own coordinate and a
// fraction of a cell per neighbour's cell) spans at most T + L - 1 cells in
// a tiled dimension and L + 1 in the untiled one, is copied from V into LDS
// once; the threads then read their windows from the box instead of
// gathering them through the vector memory pipeline.  The box starts at the
// window origin of the tile's first state, clamped to the grid; a thread
// whose window does not fit in it gathers from V as the other sweeps do.
// The contraction is the same code with the same order of operations, so
// the result is bitwise that of k_sweep_memo.
//
// The box is padded in LDS so that one read instruction of a wave hits
// distinct banks.  A wave's 64 lanes are 4 x 4 x 4 states of dimensions
// 2..4, and each LDS cycle serves 32 lanes (a 4 x 4 x 2 block) from 32
// four-byte banks.  Their window origins step by about one cell per lane in
// each of those dimensions, so rows of dimension 4 padded to 8 cells put the
// 4 x 4 block on 16 distinct banks, and a dimension-2 stride of 20 mod 32
// moves the other half of the block onto the remaining ones.  Dense strides
// (6, 36) put pairs of lanes on one bank: the profiler counted 39% of the
// LDS cycles stalled on bank conflicts.
template <class SH, int T0>
struct StageBox {
  static_assert(SH::N == 5, "staged box: 5-D shapes");
  static constexpr int C[5] = {SH::L[0] + T0, SH::L[1] + 3, SH::L[2] + 3, SH::L[3] + 3, SH::L[4] + 3};
  static constexpr int S3 = (C[4] + 7) / 8 * 8;
  // smallest stride >= C3 * S3 that is 20 mod 32
  static constexpr int S2 = C[3] * S3 + ((20 - C[3] * S3) % 32 + 32) % 32;
  static constexpr int S[5] = {C[1] * C[2] * S2, C[2] * S2, S2, S3, 1};
  static constexpr int SIZE = C[0] * S[0];
  static constexpr int PLANE = C[2] * C[3] * C[4];   // cells of dims 2..4: one per staging thread
  static constexpr int PLANES = C[0] * C[1];
  static_assert(PLANE <= 256, "a plane of the box per workgroup pass");
  static_assert(S2 % 32 == 20 && S2 >= C[3] * S3, "padded dimension-2 stride");
};

template <int KIND, class SH>
struct Staged {
  static constexpr bool value = KIND == AMY_DYN_ROOM_ && SH::N == 5 && SH::LMAX <= REL_SLOTS;
};

template <class VT, class BX>
struct VLds {
  using value_type = VT;
  const VT* p;
  __device__ __forceinline__ VT load(uint32_t voff, uint32_t soff) const {
    return *reinterpret_cast<const VT*>(reinterpret_cast<const char*>(p) + voff + soff);
  }
  template <int D>
  __device__ __forceinline__ uint32_t step(const DevProblem&) const {
    return (uint32_t)(BX::S[D] * (int)sizeof(VT));
  }
};

#define STAGE_BLOCK 256  // threads per cell of dimension 0 in a tile
// The loop levels' masses are picked from registers with selects on the
// (uniform) loop index rather than read from per-thread LDS slots: the sweep
// is bound by LDS traffic, and the slots would also cost a fifth of the
// workgroups a CU holds.
#define STAGE_LL 0

// TAIL: also the largest per-row FP64 tail over the launch into *tailmax.
// T0: cells of dimension 0 per tile (T0 x 256 threads); the threads of one
// cell of dimension 0 stage a share of the box's rows of dimension 1.
template <int KIND, class SH, class MT, class AT, class VI, class VO, bool COMP, bool TAIL, int T0>
__global__ void __launch_bounds__(STAGE_BLOCK * T0) k_sweep_stage(DevProblem P, const VI* __restrict__ Vin,
                                                             VO* __restrict__ Vout,
                                                             const uint8_t* __restrict__ label,
                                                             int16_t* __restrict__ pol, const MT* __restrict__ rm,
                                                             const double* __restrict__ wg,
                                                             unsigned long long* __restrict__ tailmax) {
  using BX = StageBox<SH, T0>;
  constexpr int N = 5;
  // the staging groups split the box's rows of dimension 1, or of
  // dimension 0 where dimension 1's do not divide evenly
  constexpr bool SPLIT1 = BX::C[1] % T0 == 0;
  static_assert(SPLIT1 || BX::C[0] % T0 == 0, "whole rows per staging group");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int blo[N];
  VI* box = reinterpret_cast<VI*>(smem);
  MT* ll = STAGE_LL ? reinterpret_cast<MT*>(smem + ((BX::SIZE * sizeof(VI) + 15) & ~(size_t)15)) + threadIdx.x
                    : nullptr;
  const int t = threadIdx.x;
  const int tp = t & (STAGE_BLOCK - 1), grp = t / STAGE_BLOCK;  // cell of a box plane; staging group
  int j[N];
  {
    uint32_t r = xcd_block(blockIdx.x, gridDim.x);
#pragma unroll
    for (int d = N - 1; d >= 1; --d) {
      const uint32_t td = (uint32_t)P.count[d] / 4u;
      const uint32_t c = r % td;
      r /= td;
      j[d] = (int)(c * 4u);
    }
    j[0] = (int)r * T0 + grp;
    j[4] += t & 3;
    j[3] += (t >> 2) & 3;
    j[2] += (t >> 4) & 3;
    j[1] += (t >> 6) & 3;
  }
  uint32_t s = 0;
#pragma unroll
  for (int d = 0; d < N; ++d) s += (uint32_t)j[d] * (uint32_t)P.stride[d];
  // this thread's cell of a box plane (dims 2..4) and its offset in V; the
  // group stages an R0 x R1 block of the box's (dim 0, dim 1) planes
  constexpr int C3C4 = BX::C[3] * BX::C[4];
  constexpr int R0 = SPLIT1 ? BX::C[0] : BX::C[0] / T0, R1 = SPLIT1 ? BX::C[1] / T0 : BX::C[1];
  const int g0 = SPLIT1 ? 0 : grp * R0, g1 = SPLIT1 ? grp * R1 : 0;  // the block's first plane
  const bool stager = tp < BX::PLANE;
  const uint32_t gt = (uint32_t)(tp / C3C4) * (uint32_t)P.stride[2] +
                      (uint32_t)((tp / BX::C[4]) % BX::C[3]) * (uint32_t)P.stride[3] + (uint32_t)(tp % BX::C[4]) +
                      (uint32_t)g0 * (uint32_t)P.stride[0] + (uint32_t)g1 * (uint32_t)P.stride[1];
  const int lt = (tp / C3C4) * BX::S[2] + ((tp / BX::C[4]) % BX::C[3]) * BX::S[3] + tp % BX::C[4] + g0 * BX::S[0] +
                 g1 * BX::S[1];
  const bool free = label[s] == LBL_FREE;
  if (!free) {
    Vout[s] = (label[s] == LBL_ONE) ? VO(1) : VO(0);
    if (pol) pol[s] = -1;
  }
  int cx[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    int v = 0;
    for (int k = 0; k < P.mctx_n[i]; ++k) {
      int jk = j[0];
#pragma unroll
      for (int d = 1; d < N; ++d)
        if (d == P.mctx[i][k]) jk = j[d];
      v += jk * P.mmult[i][k];
    }
    cx[i] = v;
  }
  const VBuf<VI> vb(Vin, (uint32_t)P.n_x);
  const VLds<VI, BX> vl{box};
  FixedRow<SH, MT> R;
  InputWalk iw;
  iw.reset();
  AT best = AT(-1);
  int arg = 0;
  double tmax = 0.0;
  for (int u = 0; u < P.n_u; ++u) {
    uint32_t base = 0;
    double win = 1.0, grid = 1.0;
    memo_load<0, SH, MT, TAIL>(P, iw, cx, rm, R, base, wg, &win, &grid);
    if constexpr (TAIL) {
      if (free) tmax = fmax(tmax, grid - win);
    }
    // every thread has passed the previous input's second barrier, so
    // blo and the box are no longer read
    if (t == 0) {
#pragma unroll
      for (int d = 0; d < N; ++d) blo[d] = min((int)R.o[d], P.count[d] - BX::C[d]);
    }
    __syncthreads();
    int bl[N];
    uint32_t gb = 0;
#pragma unroll
    for (int d = 0; d < N; ++d) {
      bl[d] = blo[d];
      gb += (uint32_t)bl[d] * (uint32_t)P.stride[d];
    }
    if (stager) {
      constexpr int NP = R0 * R1;  // planes per staging group
      VI v[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p)
        v[p] = vb.load((gb + gt) * (uint32_t)sizeof(VI),
                       ((uint32_t)(p / R1) * (uint32_t)P.stride[0] + (uint32_t)(p % R1) * (uint32_t)P.stride[1]) *
                           (uint32_t)sizeof(VI));
#pragma unroll
      for (int p = 0; p < NP; ++p) box[(p / R1) * BX::S[0] + (p % R1) * BX::S[1] + lt] = v[p];
    }
    if constexpr (STAGE_LL > 0) {
#pragma unroll
      for (int d = 0; d < SH::BL; ++d)
#pragma unroll
        for (int k = 0; k < SH::LMAX; ++k)
          if (k < SH::L[d]) ll[(d * SH::LMAX + k) * STAGE_LL] = R.m[d][k];
    }
    __syncthreads();
    if (free) {
      bool in = true;
      uint32_t lo = 0;
#pragma unroll
      for (int d = 0; d < N; ++d) {
        const int o = (int)R.o[d] - bl[d];
        in = in && o >= 0 && o + SH::L[d] <= BX::C[d];
        lo += (uint32_t)o * (uint32_t)BX::S[d];
      }
      AT q;
      if (in)
        q = contract_fixed<0, SH, MT, AT, VLds<VI, BX>, COMP, STAGE_LL>(P, R, vl, lo * (uint32_t)sizeof(VI), 0u, ll);
      else
        q = contract_fixed<0, SH, MT, AT, VBuf<VI>, COMP, STAGE_LL>(P, R, vb, base * (uint32_t)sizeof(VI), 0u, ll);
      if (q > best) {
        best = q;
        arg = u;
      }
    }
    iw.next(P);
  }
  if (free) {
    Vout[s] = VO(best);
    if (pol) pol[s] = (int16_t)arg;
  }
  if constexpr (TAIL) {
    wave_max_to(tmax, tailmax);
  }
}

template <int KIND, class SH, class MT, class VI, int T0>
static constexpr size_t stage_lds_bytes() {
  using BX = StageBox<SH, T0>;
  return ((BX::SIZE * sizeof(VI) + 15) & ~(size_t)15) + (size_t)SH::BL * SH::LMAX * sizeof(MT) * STAGE_LL;
}

// ----------------------------------------------- staged planes (7-D)
//
// The vehicle's grid has 8 x 8 cells in its last two dimensions (yaw rate,
// slip angle), so one such plane of V is 64 contiguous values.  A workgroup
// of 128 threads takes the two planes of states at cells 2b, 2b + 1 of
// dimension 4 (the other coordinates fixed); their windows share the
// origins of dimensions 0 .. 3 (those means do not read the plane's
// coordinates) and spread by at most 2 cells in dimension 4 (the heading
// moves with the yaw rate).  For each input the workgroup copies the
// L0 x L1 x L2 x L3 x (L4 + 2) planes that hold the windows into LDS, one
// 256-byte plane per wave and load, and contracts from there.  As for the
// room, the box starts at the first state's origin clamped to the grid, a
// window outside it is gathered from V, and the result is bitwise that of
// the gather sweep.
//
// TW = 8 (a grid of exactly 8 cells in dimension 4): a workgroup of 8 waves
// takes all 8 planes of states that share cells in dimensions 0 .. 3, and
// its box spans the whole of dimension 4, so the 8 waves share one box
// (a staged plane serves 8 planes of states over 8 box planes in dimension
// 4, where it served 2 over L4 + 2) and a CU holds two
// such workgroups (16 waves, where the 2-wave workgroups' 52 KB allowed 6).
// Wave w stages the box's planes at cell w of dimension 4.  The loop
// levels' masses are then picked from registers (no per-thread LDS slots).
template <class SH, int TW>
struct PlaneBox {
  static_assert(SH::N == 7, "plane box: 7-D shapes");
  static_assert(TW == 2 || TW == 8, "two planes per workgroup, or the whole 8-cell dimension 4");
  static constexpr int C[7] = {SH::L[0], SH::L[1], SH::L[2], SH::L[3], TW == 8 ? 8 : SH::L[4] + 2, 8, 8};
  static constexpr int S[7] = {C[1] * C[2] * C[3] * C[4] * 64, C[2] * C[3] * C[4] * 64, C[3] * C[4] * 64,
                               C[4] * 64, 64, 8, 1};
  static constexpr int PLANES = C[0] * C[1] * C[2] * C[3] * C[4];
  static constexpr int SIZE = PLANES * 64;
};

template <int KIND, class SH>
struct Planed {
  static constexpr bool value = KIND == AMY_DYN_VEHICLE7_ && SH::N == 7 && SH::LMAX <= REL_SLOTS;
};

#define PLANE_BLOCK 128

// Per-thread LDS slots of the loop levels' masses: the 2-wave workgroups'.
template <int TW>
struct PlaneLL {
  static constexpr int value = TW == 2 ? PLANE_BLOCK : 0;
};

template <int KIND, class SH, class MT, class AT, class VI, class VO, bool COMP, bool TAIL, int TW>
__global__ void __launch_bounds__(64 * TW) k_sweep_plane(DevProblem P, const VI* __restrict__ Vin,
                                                         VO* __restrict__ Vout,
                                                         const uint8_t* __restrict__ label,
                                                         int16_t* __restrict__ pol, const MT* __restrict__ rm,
                                                         const double* __restrict__ wg,
                                                         unsigned long long* __restrict__ tailmax) {
  using BX = PlaneBox<SH, TW>;
  constexpr int N = 7;
  constexpr int LLN = PlaneLL<TW>::value;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int blo[N];
  VI* box = reinterpret_cast<VI*>(smem);
  MT* ll = LLN ? reinterpret_cast<MT*>(smem + ((BX::SIZE * sizeof(VI) + 15) & ~(size_t)15)) + threadIdx.x : nullptr;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  int j[N];
  {
    uint32_t r = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t t4 = (uint32_t)P.count[4] / (uint32_t)TW;
    j[4] = (int)(r % t4) * TW + wave;
    r /= t4;
#pragma unroll
    for (int d = 3; d >= 0; --d) {
      const uint32_t c = (uint32_t)P.count[d];
      j[d] = (int)(r % c);
      r /= c;
    }
    j[5] = lane >> 3;
    j[6] = lane & 7;
  }
  uint32_t s = 0;
#pragma unroll
  for (int d = 0; d < N; ++d) s += (uint32_t)j[d] * (uint32_t)P.stride[d];
  const bool free = label[s] == LBL_FREE;
  if (!free) {
    Vout[s] = (label[s] == LBL_ONE) ? VO(1) : VO(0);
    if (pol) pol[s] = -1;
  }
  int cx[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    int v = 0;
    for (int k = 0; k < P.mctx_n[i]; ++k) {
      int jk = j[0];
#pragma unroll
      for (int d = 1; d < N; ++d)
        if (d == P.mctx[i][k]) jk = j[d];
      v += jk * P.mmult[i][k];
    }
    cx[i] = v;
  }
  const VBuf<VI> vb(Vin, (uint32_t)P.n_x);
  const VLds<VI, BX> vl{box};
  FixedRow<SH, MT> R;
  InputWalk iw;
  iw.reset();
  AT best = AT(-1);
  int arg = 0;
  double tmax = 0.0;
  for (int u = 0; u < P.n_u; ++u) {
    uint32_t base = 0;
    double win = 1.0, grid = 1.0;
    memo_load<0, SH, MT, TAIL>(P, iw, cx, rm, R, base, wg, &win, &grid);
    if constexpr (TAIL) {
      if (free) tmax = fmax(tmax, grid - win);
    }
    // every thread has passed the previous input's second barrier
    if (t == 0) {
#pragma unroll
      for (int d = 0; d < 5; ++d) blo[d] = min((int)R.o[d], P.count[d] - BX::C[d]);
    }
    __syncthreads();
    int bl[N];
    uint32_t gb = 0;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      bl[d] = blo[d];
      gb += (uint32_t)bl[d] * (uint32_t)P.stride[d];
    }
    bl[5] = bl[6] = 0;
    // wave w stages the planes with box coordinate w in dimension 0 (the
    // box is 2 cells wide there); plane i of a wave has fixed coordinates
    // (r1 .. r4), so its offset is a fixed combination of the strides.  Each
    // plane is 64 consecutive values of V.  Fully unrolled, CH loads in
    // flight, then their LDS writes, and a scheduling barrier so that the
    // next chunk's loads are not hoisted above them (registers).
    if constexpr (TW == 2) {
      static_assert(BX::C[0] == 2, "one wave per half of the box along dimension 0");
      constexpr int PER = BX::PLANES / 2, CH = 15;
      static_assert(PER % CH == 0, "whole chunks");
      const uint32_t gw = (gb + (uint32_t)wave * (uint32_t)P.stride[0] + (uint32_t)lane) * (uint32_t)sizeof(VI);
      VI* bw = box + wave * PER * 64 + lane;
#pragma unroll
      for (int q0 = 0; q0 < PER; q0 += CH) {
        VI v[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int i = q0 + q;
          const int r4 = i % BX::C[4], r3 = (i / BX::C[4]) % BX::C[3], r2 = (i / (BX::C[4] * BX::C[3])) % BX::C[2];
          const int r1 = i / (BX::C[4] * BX::C[3] * BX::C[2]);
          const uint32_t po = (uint32_t)r1 * (uint32_t)P.stride[1] + (uint32_t)r2 * (uint32_t)P.stride[2] +
                              (uint32_t)r3 * (uint32_t)P.stride[3] + (uint32_t)r4 * (uint32_t)P.stride[4];
          v[q] = vb.load(gw, po * (uint32_t)sizeof(VI));
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) bw[(q0 + q) * 64] = v[q];
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      // wave w: the planes at box cell w of dimension 4, in box order
      constexpr int PER = BX::PLANES / TW, CH = 12;
      static_assert(BX::C[4] == TW && PER % CH == 0, "one wave per cell of dimension 4, whole chunks");
      const uint32_t gw = (gb + (uint32_t)wave * (uint32_t)P.stride[4] + (uint32_t)lane) * (uint32_t)sizeof(VI);
      VI* bw = box + wave * BX::S[4] + lane;
#pragma unroll
      for (int q0 = 0; q0 < PER; q0 += CH) {
        VI v[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int i = q0 + q;  // (r0, r1, r2, r3), r3 fastest
          const int r3 = i % BX::C[3], r2 = (i / BX::C[3]) % BX::C[2], r1 = (i / (BX::C[3] * BX::C[2])) % BX::C[1];
          const int r0 = i / (BX::C[3] * BX::C[2] * BX::C[1]);
          const uint32_t po = (uint32_t)r0 * (uint32_t)P.stride[0] + (uint32_t)r1 * (uint32_t)P.stride[1] +
                              (uint32_t)r2 * (uint32_t)P.stride[2] + (uint32_t)r3 * (uint32_t)P.stride[3];
          v[q] = vb.load(gw, po * (uint32_t)sizeof(VI));
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int i = q0 + q;
          const int r3 = i % BX::C[3], r2 = (i / BX::C[3]) % BX::C[2], r1 = (i / (BX::C[3] * BX::C[2])) % BX::C[1];
          const int r0 = i / (BX::C[3] * BX::C[2] * BX::C[1]);
          bw[r0 * BX::S[0] + r1 * BX::S[1] + r2 * BX::S[2] + r3 * BX::S[3]] = v[q];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if constexpr (LLN > 0) {
#pragma unroll
      for (int d = 0; d < SH::BL; ++d)
#pragma unroll
        for (int k = 0; k < SH::LMAX; ++k)
          if (k < SH::L[d]) ll[(d * SH::LMAX + k) * LLN] = R.m[d][k];
    }
    __syncthreads();
    if (free) {
      bool in = true;
      uint32_t lo = 0;
#pragma unroll
      for (int d = 0; d < N; ++d) {
        const int o = (int)R.o[d] - bl[d];
        in = in && o >= 0 && o + SH::L[d] <= BX::C[d];
        lo += (uint32_t)o * (uint32_t)BX::S[d];
      }
      AT q;
      if (in)
        q = contract_fixed<0, SH, MT, AT, VLds<VI, BX>, COMP, LLN>(P, R, vl, lo * (uint32_t)sizeof(VI), 0u, ll);
      else
        q = contract_fixed<0, SH, MT, AT, VBuf<VI>, COMP, LLN>(P, R, vb, base * (uint32_t)sizeof(VI), 0u, ll);
      if (q > best) {
        best = q;
        arg = u;
      }
    }
    iw.next(P);
  }
  if (free) {
    Vout[s] = VO(best);
    if (pol) pol[s] = (int16_t)arg;
  }
  if constexpr (TAIL) {
    wave_max_to(tmax, tailmax);
  }
}

// ------------------------------------- staged boxes, shared relative tables
//
// The unicycle's steps on the shared relative tables, with one wave per
// (x, y) cell: lane t takes heading cell t (at most 64 cells), and a
// workgroup of CY waves takes CY cells adjacent in y.  Over every heading
// and input, the x and y windows of a cell start within 3 cells of each
// other (the drift is at most one cell), so the workgroup copies the
// (L_x + 2) x (L_y + 1 + CY) rows of all headings that hold its windows from
// V into LDS once per step (each row is contiguous in V; each wave copies a
// share of the rows) and every input contracts from there.  The box starts
// at the smallest origin over its lanes and inputs, clamped to the grid; a
// window outside it is gathered from V.  The order of operations is that of
// k_sweep_rel, so the bits are the same.  Cells of one workgroup share
// their box's overlapping rows: with two, 28 row loads per lane instead of
// 49, and 8 workgroups (16 waves) per CU where one cell each allowed 10
// waves; with four, 18 row loads and 5 workgroups (20 waves) per CU.
template <class SH, int CY>
struct RelBox {
  static_assert(SH::N == 3, "relative-table box: 3-D shapes");
  static constexpr int C[3] = {SH::L[0] + 2, SH::L[1] + 1 + CY, 64};
  static constexpr int S[3] = {C[1] * 64, 64, 1};
  static constexpr int ROWS = C[0] * C[1];
  static constexpr int SIZE = ROWS * 64;
};

// LDS of a relative-box workgroup: the box, then per wave its U partial
// sums behind L_{N-1} zero slots and dimension 0's masses ([slot][lane]
// each), then the shared fast
// digit tables; a first step that forms the row tails adds the heading's
// FP64 memo entries of every fast digit ([digit][lane], 16-byte aligned).
template <class SH, int U, int CY, class MT, class AT, class VI>
static size_t relbox_lds_bytes(int nf, bool tail) {
  const size_t b = (size_t)RelBox<SH, CY>::SIZE * sizeof(VI) + (size_t)CY * (U + SH::L[SH::N - 1]) * 64 * sizeof(AT) +
                   (size_t)CY * SH::L[0] * 64 * sizeof(MT) + (size_t)nf * SH::L[SH::N - 1] * sizeof(MT) + (size_t)nf * 4;
  return tail ? ((b + 15) & ~(size_t)15) + (size_t)nf * 64 * 16 : b;
}

// Where a first step on the relative box finds the memoised FP64 kept-window
// and grid masses that k_tail_memo reads (the same entries, numbered the
// same way): entry off[i] + cx * rc[i] + c of dimension i, with context cell
// cx = sum_k j[ctx[i][k]] mult[i][k].  The last dimension's context is its
// own cell alone, so every wave of a workgroup (the same heading cells on
// its lanes) shares those entries.
struct MemoTail {
  const double2* wg;
  int32_t off[3], rc[3], cn[3], ctx[3][4], mult[3][4];
};

template <int KIND, class SH, int U, class MT, class AT, class VI, class VO, bool COMP, int CY, bool TAIL>
__global__ void __launch_bounds__(64 * CY) k_sweep_relbox(DevProblem P, const VI* __restrict__ Vin,
                                                          VO* __restrict__ Vout, const uint8_t* __restrict__ label,
                                                          int16_t* __restrict__ pol, const MT* __restrict__ rm,
                                                          const int32_t* __restrict__ rlo, MemoTail mt,
                                                          unsigned long long* __restrict__ tailmax) {
  using BX = RelBox<SH, CY>;
  constexpr int N = 3;
  constexpr int F = N - 1;
  constexpr int LF = SH::L[F];
  static_assert(2 * LF <= U && SH::LMAX <= REL_SLOTS, "relative-table sweep shape");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int wlo[2][CY];
  const int fd = P.m - 1, nf = P.ucount[fd], fm = P.rmult[F][fd];
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  VI* box = reinterpret_cast<VI*>(smem);
  // the lane's U partial sums of one slow combination, read back by index,
  // after LF slots that hold zeros (slot t at asl[t * 64], t >= -LF)
  AT* asl = reinterpret_cast<AT*>(smem + BX::SIZE * sizeof(VI)) + (w * (U + LF) + LF) * 64 + lane;
  unsigned char* after_asl = smem + BX::SIZE * sizeof(VI) + (size_t)CY * (U + LF) * 64 * sizeof(AT);
  MT* t0 = reinterpret_cast<MT*>(after_asl) + w * SH::L[0] * 64 + lane;
  MT* thm = reinterpret_cast<MT*>(after_asl) + CY * SH::L[0] * 64;
  int32_t* thr = reinterpret_cast<int32_t*>(thm + nf * LF);
  for (int f = (int)threadIdx.x; f < nf; f += 64 * CY) {
    const int e = P.rel_off[F] + f * fm;
#pragma unroll
    for (int k = 0; k < LF; ++k) thm[f * LF + k] = rm[(int64_t)e * REL_SLOTS + k];
    thr[f] = rlo[e];
  }
  const int nF = P.count[F];
  double2* fent = reinterpret_cast<double2*>(
      (reinterpret_cast<uintptr_t>(thr + nf) + 15) & ~(uintptr_t)15);  // [fast digit][lane]
  if constexpr (TAIL) {
    const int64_t fb = mt.off[F] + (int64_t)min(lane, nF - 1) * mt.mult[F][0] * mt.rc[F];
    for (int f = w; f < nf; f += CY) fent[f * 64 + lane] = mt.wg[fb + (int64_t)f * fm];
  }
  const uint32_t nyb = (uint32_t)P.count[1] / (uint32_t)CY;
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  int j[N];
  j[1] = (int)(blk % nyb) * CY + w;
  j[0] = (int)(blk / nyb);
  j[F] = lane;
  const uint32_t pair = (uint32_t)j[0] * (uint32_t)P.count[1] + (uint32_t)j[1];
  const bool valid = lane < nF;
  const uint32_t s = pair * (uint32_t)nF + (uint32_t)lane;
  const uint8_t lb = valid ? label[s] : (uint8_t)LBL_ZERO;
  const bool free = valid && lb == LBL_FREE;
  if (valid && !free) {
    Vout[s] = (lb == LBL_ONE) ? VO(1) : VO(0);
    if (pol) pol[s] = -1;
  }
  const int nslow = P.n_u / nf;
  // the box origin: the smallest x and y window origin over the free lanes
  // of every wave and the slow digits (the fast digit moves only the heading)
  int lo0 = P.count[0], lo1 = P.count[1];
  if (free) {
    InputWalk iw;
    iw.reset();
    FixedRow<SH, MT> R;
    for (int sc = 0; sc < nslow; ++sc) {
      int r[N];
      rel_load<0, SH, MT>(P, iw, j, rm, rlo, R, r);
      lo0 = min(lo0, min(max(r[0], 0), P.count[0] - SH::L[0]));
      lo1 = min(lo1, min(max(r[1], 0), P.count[1] - SH::L[1]));
#pragma unroll
      for (int k = AMY_MAXI - 1; k >= 0; --k) {
        if (k < fd) {
          if (++iw.dig[k] < P.ucount[k]) break;
          iw.dig[k] = 0;
        }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo0 = min(lo0, __shfl_xor(lo0, off));
    lo1 = min(lo1, __shfl_xor(lo1, off));
  }
  if constexpr (CY > 1) {
    if (lane == 0) {
      wlo[0][w] = lo0;
      wlo[1][w] = lo1;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CY; ++q) {
      lo0 = min(lo0, wlo[0][q]);
      lo1 = min(lo1, wlo[1][q]);
    }
  }
  const int b0 = __builtin_amdgcn_readfirstlane(min(lo0, P.count[0] - BX::C[0]));
  const int b1 = __builtin_amdgcn_readfirstlane(min(lo1, P.count[1] - BX::C[1]));
  const VBuf<VI> vb(Vin, (uint32_t)P.n_x);
  {
    // rows (x, y) of the box, each the run of all heading cells; wave w
    // copies rows [w PER, (w + 1) PER) that lie in the box, in chunks of 7
    const uint32_t gl = ((uint32_t)b0 * (uint32_t)P.stride[0] + (uint32_t)b1 * (uint32_t)P.stride[1] +
                         (uint32_t)min(lane, nF - 1)) * (uint32_t)sizeof(VI);
    constexpr int CH = 7, PER = (BX::ROWS + CY - 1) / CY;
    constexpr bool EXACT = PER * CY == BX::ROWS && PER % CH == 0;
    const int qw = w * PER;
#pragma unroll
    for (int q0 = 0; q0 < PER; q0 += CH) {
      VI v[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        const int qq = EXACT ? qw + q0 + q : min(qw + q0 + q, BX::ROWS - 1);
        const int rx = qq / BX::C[1], ry = qq % BX::C[1];
        v[q] = vb.load(gl, ((uint32_t)rx * (uint32_t)P.stride[0] + (uint32_t)ry * (uint32_t)P.stride[1]) *
                               (uint32_t)sizeof(VI));
      }
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (EXACT || (q0 + q < PER && qw + q0 + q < BX::ROWS)) box[(qw + q0 + q) * 64 + lane] = v[q];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();
  double tmax = 0.0;
  do {  // the free lanes' rows; the others skip to the tail reduction
    if (!free) break;  // no barrier follows
    const VLds<VI, BX> vl{box};
    // the row tails' context entries of dimensions 0 and 1
    int64_t tb[2] = {0, 0};
    if constexpr (TAIL) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        int64_t cx = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < mt.cn[i]) {
            const int d = mt.ctx[i][k];
            cx += (int64_t)(d == 0 ? j[0] : d == 1 ? j[1] : j[2]) * mt.mult[i][k];
          }
        tb[i] = mt.off[i] + cx * mt.rc[i];
      }
    }
    int omin = nF;
    for (int f = 0; f < nf; ++f) omin = min(omin, min(max(j[F] + thr[f], 0), nF - LF));
    // A index of a fast input's first kept cell is gl + thr[f]; slots past
    // the heading count (t >= tv) and the LF slots before slot 0 read as
    // zero, so every kept-cell product needs no mask
    const int gl = j[F] - omin, tv = nF - omin;
#pragma unroll
    for (int k = 1; k <= LF; ++k) asl[-k * FIX_BLOCK] = AT(0);
    FixedRow<SH, MT> R;
    InputWalk iw;
    iw.reset();
    AT best = AT(-1);
    int arg = 0, u = 0;
    for (int sc = 0; sc < nslow; ++sc) {
      uint32_t base = (uint32_t)omin;
      int r[N];
      double2 ex, ey;
      if constexpr (TAIL) {
        // this slow combination's entries of dimensions 0 and 1, loaded now
        // and used after the contraction
        int64_t e0 = tb[0], e1 = tb[1];
#pragma unroll
        for (int k = 0; k < AMY_MAXI; ++k)
          if (k < fd) {
            e0 += (int64_t)iw.dig[k] * P.rmult[0][k];
            e1 += (int64_t)iw.dig[k] * P.rmult[1][k];
          }
        ex = mt.wg[e0];
        ey = mt.wg[e1];
      }
      rel_load<0, SH, MT>(P, iw, j, rm, rlo, R, r);
      rel_place<0, SH, MT>(P, r, t0, R, base);
      const int o0 = min(max(r[0], 0), P.count[0] - SH::L[0]) - b0;
      const int o1 = min(max(r[1], 0), P.count[1] - SH::L[1]) - b1;
      AT A[U];
      if (o0 >= 0 && o0 + SH::L[0] <= BX::C[0] && o1 >= 0 && o1 + SH::L[1] <= BX::C[1])
        contract_fac<SH, U, MT, AT, VLds<VI, BX>, COMP>(
            P, R, t0, vl, ((uint32_t)o0 * BX::S[0] + (uint32_t)o1 * BX::S[1] + (uint32_t)omin) * (uint32_t)sizeof(VI), A);
      else
        contract_fac<SH, U, MT, AT, VBuf<VI>, COMP>(P, R, t0, vb, base * (uint32_t)sizeof(VI), A);
#pragma unroll
      for (int t = 0; t < U; ++t) asl[t * FIX_BLOCK] = t < tv ? A[t] : AT(0);
      if constexpr (TAIL) {
        // the row's kept-window and grid masses, multiplied in dimension
        // order as k_tail_memo does, so the max is the same bits
        const double w01 = ex.x * ey.x, g01 = ex.y * ey.y;
        for (int f = 0; f < nf; ++f) {
          const double2 ef = fent[f * 64 + lane];
          tmax = fmax(tmax, g01 * ef.y - w01 * ef.x);
        }
      }
      for (int f = 0; f < nf; ++f, ++u) {
        // The window's origin is clamped to [0, nF - LF] over the fast
        // inputs (omin is the smallest clamped origin), so the kept cells of
        // an input lie in slots [g, g + LF) with g >= -LF after the clamp
        // below: slots before 0 are below the grid, slots at or past tv
        // beyond it.  g > U - LF happens only when omin = nF - LF, and then
        // every slot from LF = tv on is zero, so clamping g to U - LF reads
        // zeros as the unclamped window would have.  A zero term leaves the
        // sum's bits as they are.
        const int g = min(max(gl + thr[f], -LF), U - LF);
        const AT* ap = asl + g * FIX_BLOCK;
        AT q = AT(0);
#pragma unroll
        for (int k = 0; k < LF; ++k) q = fma_(AT(thm[f * LF + k]), ap[k * FIX_BLOCK], q);
        if (q > best) {
          best = q;
          arg = u;
        }
      }
#pragma unroll
      for (int k = AMY_MAXI - 1; k >= 0; --k) {
        if (k < fd) {
          if (++iw.dig[k] < P.ucount[k]) break;
          iw.dig[k] = 0;
        }
      }
    }
    Vout[s] = VO(best);
    if (pol) pol[s] = (int16_t)arg;
  } while (false);
  if constexpr (TAIL) wave_max_to(tmax, tailmax);
}

// ------------------------------------------------------------- launchers

template <int KIND, class SH>
struct FixedLaunch {
  static bool matches(const DevProblem& P) {
    if (P.kind != KIND || P.n != SH::N) return false;
    for (int i = 0; i < SH::N; ++i)
      if (P.L[i] != SH::L[i]) return false;
    return true;
  }
  // Every step (the tail step included) of a memoised solve runs the staged
  // box or plane sweep, which read their masses from the tables alone.
  static bool memo_complete(const DevProblem& P, bool f64) {
    if (!matches(P) || SH::LMAX > REL_SLOTS) return false;
    if constexpr (Planed<KIND, SH>::value) {
      using BX = PlaneBox<SH, 2>;
      // FP64 boxes only in the 8-wave form (147 KB of LDS)
      bool ok = (!f64 || P.count[4] == 8) && P.count[5] == 8 && P.count[6] == 8 && P.count[4] % 2 == 0;
      for (int d = 0; d < 5; ++d) ok = ok && P.count[d] >= BX::C[d];
      if (ok) return true;
    }
    if constexpr (Staged<KIND, SH>::value) {
      using BX = StageBox<SH, 1>;
      bool ok = true;
      for (int d = 0; d < SH::N; ++d) ok = ok && P.count[d] >= BX::C[d] && (d == 0 || P.count[d] % 4 == 0);
      return ok;
    }
    return false;
  }
  template <class MT, class AT, class VI, class VO, bool COMP, int T0>
  static void stage(const DevProblem& P, const void* Vin, void* Vout, const uint8_t* label, int16_t* pol,
                    const MT* rm, const double* wg, unsigned long long* tailmax, hipStream_t st) {
    if constexpr (Staged<KIND, SH>::value) {
      const dim3 gs((unsigned)(P.n_x / (STAGE_BLOCK * T0))), bs(STAGE_BLOCK * T0);
      const size_t slds = stage_lds_bytes<KIND, SH, MT, VI, T0>();
      if (tailmax)
        hipLaunchKernelGGL((k_sweep_stage<KIND, SH, MT, AT, VI, VO, COMP, true, T0>), gs, bs, slds, st, P,
                           (const VI*)Vin, (VO*)Vout, label, pol, rm, wg, tailmax);
      else
        hipLaunchKernelGGL((k_sweep_stage<KIND, SH, MT, AT, VI, VO, COMP, false, T0>), gs, bs, slds, st, P,
                           (const VI*)Vin, (VO*)Vout, label, pol, rm, wg, tailmax);
    }
  }
  template <class MT, class AT, class VI, class VO, bool COMP, int TW>
  static void plane(const DevProblem& P, const void* Vin, void* Vout, const uint8_t* label, int16_t* pol,
                    const MT* rm, const double* wg, unsigned long long* tailmax, hipStream_t st) {
    if constexpr (Planed<KIND, SH>::value) {
      using BX = PlaneBox<SH, TW>;
      const dim3 gs((unsigned)(P.n_x / (64 * TW))), bs(64 * TW);
      const size_t slds = ((BX::SIZE * sizeof(VI) + 15) & ~(size_t)15) +
                          (size_t)SH::BL * SH::LMAX * sizeof(MT) * PlaneLL<TW>::value;
      if (tailmax)
        hipLaunchKernelGGL((k_sweep_plane<KIND, SH, MT, AT, VI, VO, COMP, true, TW>), gs, bs, slds, st, P,
                           (const VI*)Vin, (VO*)Vout, label, pol, rm, wg, tailmax);
      else
        hipLaunchKernelGGL((k_sweep_plane<KIND, SH, MT, AT, VI, VO, COMP, false, TW>), gs, bs, slds, st, P,
                           (const VI*)Vin, (VO*)Vout, label, pol, rm, wg, tailmax);
    }
  }
  template <class MT, class AT, class VI, class VO, bool COMP>
  static void go(const DevProblem& P, const void* Vin, void* Vout, const uint8_t* label, int16_t* pol,
                 unsigned long long* tailmax, const void* tables, hipStream_t st) {
    const dim3 g((unsigned)((P.n_x + FIX_BLOCK - 1) / FIX_BLOCK)), b(FIX_BLOCK);
    if constexpr (SH::LMAX <= REL_SLOTS) {
      if constexpr (Planed<KIND, SH>::value) {
        using BX = PlaneBox<SH, 2>;
        bool ok = tables && P.tables == 2 && P.count[5] == 8 && P.count[6] == 8 && P.count[4] % 2 == 0 &&
                  (sizeof(VI) == 4 || P.count[4] == 8);
        for (int d = 0; d < 5; ++d) ok = ok && P.count[d] >= BX::C[d];
        if (ok) {
          const MT* rm = (const MT*)tables;
          const double* wg =
              (const double*)((const char*)tables + memo_wg_offset(P, amy_memo_rec(SH::LMAX), sizeof(MT)));
          // the whole 8-cell dimension 4 in one workgroup where the grid has
          // exactly that (its box, 72 KB in FP32, leaves room for two per CU)
          // (an FP64 box of the 2-wave form would be 90 KB for 2 waves; the
          // 8-wave one, 147 KB, holds one workgroup per CU)
          if (P.count[4] == 8) plane<MT, AT, VI, VO, COMP, 8>(P, Vin, Vout, label, pol, rm, wg, tailmax, st);
          else if constexpr (sizeof(VI) == 4) plane<MT, AT, VI, VO, COMP, 2>(P, Vin, Vout, label, pol, rm, wg, tailmax, st);
          return;
        }
      }
      if constexpr (Staged<KIND, SH>::value) {
        using BX = StageBox<SH, 1>;
        bool ok = tables && P.tables == 2;
        for (int d = 0; d < SH::N; ++d) ok = ok && P.count[d] >= BX::C[d] && (d == 0 || P.count[d] % 4 == 0);
        if (ok) {
          const MT* rm = (const MT*)tables;
          const double* wg =
              (const double*)((const char*)tables + memo_wg_offset(P, amy_memo_rec(SH::LMAX), sizeof(MT)));
          // two cells of dimension 0 per tile where the count is even, two
          // such boxes fit a CU's 160 KB of LDS (80 KB each: the FP64 3^5
          // box is 75 KB) and the box's rows of dimension 1 or 0 split
          // evenly between the two staging groups, else one
          constexpr bool two_ok = stage_lds_bytes<KIND, SH, MT, VI, 2>() <= 80 * 1024 &&
                                  (StageBox<SH, 2>::C[1] % 2 == 0 || StageBox<SH, 2>::C[0] % 2 == 0);
          if (two_ok && P.count[0] % 2 == 0 && P.count[0] >= StageBox<SH, 2>::C[0]) {
            stage<MT, AT, VI, VO, COMP, (two_ok ? 2 : 1)>(P, Vin, Vout, label, pol, rm, wg, tailmax, st);
            return;
          }
          stage<MT, AT, VI, VO, COMP, 1>(P, Vin, Vout, label, pol, rm, wg, tailmax, st);
          return;
        }
      }
      if (!tailmax && tables && P.tables == 2) {
      const MT* rm = (const MT*)tables;
      const size_t lds = (size_t)(SH::BL > 0 ? SH::BL : 1) * SH::LMAX * sizeof(MT) * FIX_BLOCK;
      hipLaunchKernelGGL((k_sweep_memo<KIND, SH, MT, AT, VI, VO, COMP>), g, b, lds, st, P, (const VI*)Vin, (VO*)Vout,
                         label, pol, rm);
      return;
      }
    }
    if (tailmax)
      hipLaunchKernelGGL((k_sweep_fixed<KIND, SH, MT, AT, VI, VO, COMP, true>), g, b, P.lds_bytes_tail, st, P,
                         (const VI*)Vin, (VO*)Vout, label, pol, tailmax);
    else
      hipLaunchKernelGGL((k_sweep_fixed<KIND, SH, MT, AT, VI, VO, COMP, false>), g, b, P.lds_bytes_fixed, st, P,
                         (const VI*)Vin, (VO*)Vout, label, pol, tailmax);
  }
  static hipError_t sweep(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout, const uint8_t* label,
                          int16_t* pol, unsigned long long* tailmax, const void* tables, hipStream_t st) {
    switch (sk) {
      case SWEEP_F64: go<double, double, double, double, false>(P, Vin, Vout, label, pol, tailmax, tables, st); break;
      case SWEEP_F32: go<float, float, float, float, true>(P, Vin, Vout, label, pol, tailmax, tables, st); break;
      case SWEEP_F32_LAST:
        go<float, double, float, double, false>(P, Vin, Vout, label, pol, tailmax, tables, st);
        break;
    }
    return hipGetLastError();
  }
  static hipError_t memo_build(const DevProblem& P, bool f64, void* tables, hipStream_t st) {
    if (SH::LMAX > REL_SLOTS) return hipErrorInvalidValue;  // the host never plans it
    const dim3 g((unsigned)((P.rel_entries + 63) / 64)), b(64);
    constexpr int REC = amy_memo_rec(SH::LMAX);
    double* wg = (double*)((char*)tables + memo_wg_offset(P, REC, f64 ? 8 : 4));
    if (P.noise != 0) {
      if (f64) hipLaunchKernelGGL((k_memo_build<KIND, SH::N, double, REC, true>), g, b, 0, st, P, (double*)tables, wg);
      else hipLaunchKernelGGL((k_memo_build<KIND, SH::N, float, REC, true>), g, b, 0, st, P, (float*)tables, wg);
    } else {
      if (f64) hipLaunchKernelGGL((k_memo_build<KIND, SH::N, double, REC, false>), g, b, 0, st, P, (double*)tables, wg);
      else hipLaunchKernelGGL((k_memo_build<KIND, SH::N, float, REC, false>), g, b, 0, st, P, (float*)tables, wg);
    }
    return hipGetLastError();
  }
};

// Factored launch of a shape (U: innermost cells reachable by the fast digit).
template <int KIND, class SH, int U>
struct FacLaunch {
  // dimension N-1 depends on the last input digit alone and its tables are
  // cached, no other dimension depends on that digit, and the fast digit's
  // windows span at most U innermost cells
  static bool feasible(const DevProblem& P) {
    if (!FixedLaunch<KIND, SH>::matches(P) || P.nocut) return false;
    const int F = SH::N - 1, fd = P.m - 1;
    if (P.rmult[F][fd] <= 0 || P.dep_mult[F][fd] <= 0) return false;
    for (int k = 0; k < fd; ++k)
      if (P.rmult[F][k] != 0) return false;
    for (int i = 0; i < F; ++i)
      if (P.rmult[i][fd] != 0) return false;
    if (P.ccount[F] <= 0 || P.ucount[fd] > 1024) return false;
    return span_bound(P) <= U;
  }
  // Window origins move by at most ceil(drift range / h) cells over the fast
  // digit, plus one for rounding at a cell boundary; the union adds L_F.
  static int span_bound(const DevProblem& P);
  // Cells per relative-box workgroup with these element types: the most
  // (4, 2 or 1 adjacent in y) that the y count divides, whose box fits the
  // grid and whose LDS (with the tail's entries when tail) stays within
  // 64 KB; 0 when none does.
  template <class MT, class AT, class VI>
  static int relbox_cy(const DevProblem& P, bool tail) {
    if constexpr (SH::N == 3 && RelDrift<KIND, SH::N>::ok) {
      if (P.rel_entries <= 0 || P.count[2] > 64) return 0;
      const int nf = P.ucount[P.m - 1];
      if (P.count[0] >= RelBox<SH, 4>::C[0] && P.count[1] >= RelBox<SH, 4>::C[1] && P.count[1] % 4 == 0 &&
          relbox_lds_bytes<SH, U, 4, MT, AT, VI>(nf, tail) <= 64 * 1024)
        return 4;
      if (P.count[0] >= RelBox<SH, 2>::C[0] && P.count[1] >= RelBox<SH, 2>::C[1] && P.count[1] % 2 == 0 &&
          relbox_lds_bytes<SH, U, 2, MT, AT, VI>(nf, tail) <= 64 * 1024)
        return 2;
      if (P.count[0] >= RelBox<SH, 1>::C[0] && P.count[1] >= RelBox<SH, 1>::C[1] &&
          relbox_lds_bytes<SH, U, 1, MT, AT, VI>(nf, tail) <= 64 * 1024)
        return 1;
    }
    return 0;
  }
  // The relative-box sweep can form the first step's row tails from the
  // memoised tables of T: the last dimension's context is its own cell
  // alone and some box of the plan's sweeps fits the LDS.
  static bool fuses_tail(const DevProblem& P, const DevProblem& T, bool f64) {
    const int F = SH::N - 1;
    if (T.tables != 2 || T.mctx_n[F] != 1 || T.mctx[F][0] != F) return false;
    for (int i = 0; i < F; ++i)
      if (T.mctx_n[i] < 1 || T.mctx_n[i] > 4) return false;
    if (f64) return relbox_cy<double, double, double>(P, true) > 0;
    return relbox_cy<float, float, float>(P, true) > 0 && relbox_cy<float, double, float>(P, true) > 0;
  }
  template <class MT, class AT, class VI, class VO, bool COMP, int CY, bool TAIL>
  static void relbox(const DevProblem& P, const void* Vin, void* Vout, const uint8_t* label, int16_t* pol,
                     const MT* rm, const int32_t* ro, const MemoTail& mt, unsigned long long* tailmax,
                     hipStream_t st) {
    const dim3 gb((unsigned)(P.n_x / P.count[2] / CY)), bb(64 * CY);
    const size_t lb = relbox_lds_bytes<SH, U, CY, MT, AT, VI>(P.ucount[P.m - 1], TAIL);
    hipLaunchKernelGGL((k_sweep_relbox<KIND, SH, U, MT, AT, VI, VO, COMP, CY, TAIL>), gb, bb, lb, st, P,
                       (const VI*)Vin, (VO*)Vout, label, pol, rm, ro, mt, tailmax);
  }
  // mt: the memoised tables for the row tails (with tailmax, when
  // fuses_tail holds), else nullptr
  template <class MT, class AT, class VI, class VO, bool COMP>
  static void go(const DevProblem& P, const void* Vin, void* Vout, const uint8_t* label, int16_t* pol,
                 unsigned long long* tailmax, const void* rel, hipStream_t st, const MemoTail* mt) {
    const dim3 g((unsigned)((P.n_x + FIX_BLOCK - 1) / FIX_BLOCK)), b(FIX_BLOCK);
    if constexpr (RelDrift<KIND, SH::N>::ok) {
      if (rel && P.rel_entries > 0) {
        const bool fuse = tailmax && mt && relbox_cy<MT, AT, VI>(P, true) > 0;
        const int cy = relbox_cy<MT, AT, VI>(P, fuse);
        if (tailmax && !fuse) {  // the first step: its row tails in a pass of their own
          const size_t tl = (size_t)(P.lds_bytes_tail - P.lds_tail_off);
          hipLaunchKernelGGL((k_tail_cached<KIND, SH::N>), g, b, tl, st, P, label, tailmax);
        }
        const MT* rm = (const MT*)rel;
        const int32_t* ro = (const int32_t*)((const char*)rel +
                                             (((uint64_t)P.rel_entries * REL_SLOTS * sizeof(MT) + 255) & ~255ull));
        const MemoTail m0 = fuse ? *mt : MemoTail{};
        switch (fuse ? -cy : cy) {
          case 4: relbox<MT, AT, VI, VO, COMP, 4, false>(P, Vin, Vout, label, pol, rm, ro, m0, nullptr, st); return;
          case 2: relbox<MT, AT, VI, VO, COMP, 2, false>(P, Vin, Vout, label, pol, rm, ro, m0, nullptr, st); return;
          case 1: relbox<MT, AT, VI, VO, COMP, 1, false>(P, Vin, Vout, label, pol, rm, ro, m0, nullptr, st); return;
          case -4: relbox<MT, AT, VI, VO, COMP, 4, true>(P, Vin, Vout, label, pol, rm, ro, m0, tailmax, st); return;
          case -2: relbox<MT, AT, VI, VO, COMP, 2, true>(P, Vin, Vout, label, pol, rm, ro, m0, tailmax, st); return;
          case -1: relbox<MT, AT, VI, VO, COMP, 1, true>(P, Vin, Vout, label, pol, rm, ro, m0, tailmax, st); return;
          default: break;
        }
        const int nf = P.ucount[P.m - 1];
        const size_t lds = (size_t)SH::L[0] * sizeof(MT) * FIX_BLOCK + (size_t)nf * SH::L[SH::N - 1] * sizeof(MT) +
                           (size_t)nf * 4;
        hipLaunchKernelGGL((k_sweep_rel<KIND, SH, U, MT, AT, VI, VO, COMP>), g, b, lds, st, P, (const VI*)Vin,
                           (VO*)Vout, label, pol, rm, ro);
        return;
      }
    }
    // the block's tables, then one slot of dimension 0's masses per lane
    const uint32_t t0 = (uint32_t)(((tailmax ? P.lds_bytes_tail : P.lds_bytes_fixed) + 15) & ~15);
    const size_t lds = t0 + (size_t)SH::L[0] * sizeof(MT) * FIX_BLOCK;
    if (tailmax)
      hipLaunchKernelGGL((k_sweep_fac<KIND, SH, U, MT, AT, VI, VO, COMP, true>), g, b, lds, st, P,
                         (const VI*)Vin, (VO*)Vout, label, pol, tailmax, t0);
    else
      hipLaunchKernelGGL((k_sweep_fac<KIND, SH, U, MT, AT, VI, VO, COMP, false>), g, b, lds, st, P,
                         (const VI*)Vin, (VO*)Vout, label, pol, tailmax, t0);
  }
  static hipError_t sweep(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout, const uint8_t* label,
                          int16_t* pol, unsigned long long* tailmax, const void* rel, hipStream_t st,
                          const MemoTail* mt) {
    switch (sk) {
      case SWEEP_F64: go<double, double, double, double, false>(P, Vin, Vout, label, pol, tailmax, rel, st, mt); break;
      case SWEEP_F32: go<float, float, float, float, true>(P, Vin, Vout, label, pol, tailmax, rel, st, mt); break;
      case SWEEP_F32_LAST:
        go<float, double, float, double, false>(P, Vin, Vout, label, pol, tailmax, rel, st, mt);
        break;
    }
    return hipGetLastError();
  }
  // shared relative tables of the family, if it has them
  static int rel_plan(DevProblem& P) {
    if constexpr (!RelDrift<KIND, SH::N>::ok) {
      return 0;
    } else {
      int off = 0;
      for (int i = 0; i < SH::N; ++i) {
        const int cx = RelDrift<KIND, SH::N>::ctx(i);
        P.rctx[i] = cx;
        P.rel_off[i] = off;
        off += (cx >= 0 ? P.count[cx] : 1) * P.rcount[i];
      }
      P.rel_entries = off;
      return off;
    }
  }
  static hipError_t rel_build(const DevProblem& P, bool f64, void* rel, hipStream_t st) {
    if constexpr (RelDrift<KIND, SH::N>::ok) {
      const dim3 g((unsigned)((P.rel_entries + 63) / 64)), b(64);
      const uint64_t msz = f64 ? 8 : 4;
      int32_t* ro = (int32_t*)((char*)rel + (((uint64_t)P.rel_entries * REL_SLOTS * msz + 255) & ~255ull));
      if (f64) hipLaunchKernelGGL((k_rel_build<KIND, SH::N, double>), g, b, 0, st, P, (double*)rel, ro);
      else hipLaunchKernelGGL((k_rel_build<KIND, SH::N, float>), g, b, 0, st, P, (float*)rel, ro);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
};

// Window shapes of the workload families (2-D linear, 3-D unicycle, 5-D
// room ring, 7-D vehicle).
// (first argument: the most gathers issued as one unrolled block)
using ShapeUnicycle = ShapeT<64, 5, 5, 2>;
using ShapeUnicycleWide = ShapeT<64, 6, 6, 3>;  // the same noise with the intersect window rule
using ShapeRoom5 = ShapeT<27, 3, 3, 3, 3, 3>;
using ShapeRoom5Narrow = ShapeT<16, 2, 2, 2, 2, 2>;  // windows of two cells (noise narrower than a cell)
using ShapeVehicle7 = ShapeT<27, 2, 2, 3, 3, 3, 3, 3>;
using ShapeLinear2 = ShapeT<28, 28, 28>;
#define AMY_FIXED_SHAPES(X)            \
  X(AMY_DYN_UNICYCLE_, ShapeUnicycle)  \
  X(AMY_DYN_UNICYCLE_, ShapeUnicycleWide) \
  X(AMY_DYN_ROOM_, ShapeRoom5)         \
  X(AMY_DYN_ROOM_, ShapeRoom5Narrow)   \
  X(AMY_DYN_VEHICLE7_, ShapeVehicle7)  \
  X(AMY_DYN_AFFINE_, ShapeLinear2)

// Unicycle: the heading moves by tau * omega, omega the last input.
static int unicycle_span(const DevProblem& P) {
  const int F = 2, fd = P.m - 1;
  const double range = fabs(P.params[0]) * (P.uhi[fd] - P.ulo[fd]);
  return (int)ceil(range * P.inv_h[F] - 1e-12) + 1 + P.L[F];
}
template <>
int FacLaunch<AMY_DYN_UNICYCLE_, ShapeUnicycle, 5>::span_bound(const DevProblem& P) {
  return unicycle_span(P);
}
template <>
int FacLaunch<AMY_DYN_UNICYCLE_, ShapeUnicycleWide, 6>::span_bound(const DevProblem& P) {
  return unicycle_span(P);
}

// (the centre rule's 5 x 5 x 2 windows; the intersect rule's 6 x 6 x 3)
#define AMY_FAC_SHAPES(X) X(AMY_DYN_UNICYCLE_, ShapeUnicycle, 5) X(AMY_DYN_UNICYCLE_, ShapeUnicycleWide, 6)

bool amy_fac_available(const DevProblem& P) {
  const uint64_t vbytes = (uint64_t)P.n_x * 8u;
  if (vbytes >= (1ull << 32)) return false;
#define X(K, SH, U) \
  if (FacLaunch<K, SH, U>::feasible(P)) return true;
  AMY_FAC_SHAPES(X)
#undef X
  return false;
}

bool amy_fac_fuses_tail(const DevProblem& P, const DevProblem& T, bool f64) {
#define X(K, SH, U) \
  if (FacLaunch<K, SH, U>::feasible(P)) return FacLaunch<K, SH, U>::fuses_tail(P, T, f64);
  AMY_FAC_SHAPES(X)
#undef X
  return false;
}

hipError_t amy_launch_sweep_fac(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                                const uint8_t* label, int16_t* pol, unsigned long long* tailmax, const void* rel,
                                hipStream_t st, const DevProblem* tail_dev, const void* tail_tab) {
  MemoTail mt{};
  const bool fused = tailmax && tail_dev && tail_tab;
  if (fused) {
    const bool f64 = (sk == SWEEP_F64);
    if (!amy_fac_fuses_tail(P, *tail_dev, f64)) return hipErrorInvalidValue;
    int lmax = 1;
    for (int i = 0; i < tail_dev->n; ++i) lmax = tail_dev->L[i] > lmax ? tail_dev->L[i] : lmax;
    mt.wg = (const double2*)((const char*)tail_tab + memo_wg_offset(*tail_dev, amy_memo_rec(lmax), f64 ? 8 : 4));
    for (int i = 0; i < 3; ++i) {
      mt.off[i] = tail_dev->rel_off[i];
      mt.rc[i] = tail_dev->rcount[i];
      mt.cn[i] = tail_dev->mctx_n[i];
      for (int k = 0; k < 4; ++k) {
        mt.ctx[i][k] = tail_dev->mctx[i][k];
        mt.mult[i][k] = tail_dev->mmult[i][k];
      }
    }
  }
#define X(K, SH, U)                            \
  if (FacLaunch<K, SH, U>::feasible(P)) \
    return FacLaunch<K, SH, U>::sweep(P, sk, Vin, Vout, label, pol, tailmax, rel, st, fused ? &mt : nullptr);
  AMY_FAC_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

int amy_rel_plan(DevProblem& P) {
#define X(K, SH, U) \
  if (FacLaunch<K, SH, U>::feasible(P)) return FacLaunch<K, SH, U>::rel_plan(P);
  AMY_FAC_SHAPES(X)
#undef X
  return 0;
}

hipError_t amy_launch_rel_build(const DevProblem& P, bool f64, void* rel, hipStream_t st) {
#define X(K, SH, U) \
  if (FacLaunch<K, SH, U>::feasible(P)) return FacLaunch<K, SH, U>::rel_build(P, f64, rel, st);
  AMY_FAC_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

bool amy_fixed_available(const DevProblem& P) {
  // buffer byte offsets are 32-bit
  const uint64_t vbytes = (uint64_t)P.n_x * 8u;
  if (vbytes >= (1ull << 32)) return false;
#define X(K, SH) \
  if (FixedLaunch<K, SH>::matches(P)) return true;
  AMY_FIXED_SHAPES(X)
#undef X
  return false;
}

bool amy_fixed_memo_complete(const DevProblem& P, bool f64) {
  if ((uint64_t)P.n_x * 8u >= (1ull << 32)) return false;
#define X(K, SH) \
  if (FixedLaunch<K, SH>::matches(P)) return FixedLaunch<K, SH>::memo_complete(P, f64);
  AMY_FIXED_SHAPES(X)
#undef X
  return false;
}

hipError_t amy_launch_sweep_fixed(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                                  const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                                  const void* tables, hipStream_t st) {
#define X(K, SH)                          \
  if (FixedLaunch<K, SH>::matches(P)) \
    return FixedLaunch<K, SH>::sweep(P, sk, Vin, Vout, label, pol, tailmax, tables, st);
  AMY_FIXED_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

size_t amy_tail_memo_lds(const DevProblem& P) {
  size_t ne = 0;
  for (int i = 0; i < P.n; ++i) ne += (size_t)P.rcount[i];
  return ne * 16 * TAIL_MEMO_BLOCK;
}

hipError_t amy_launch_tail_memo(const DevProblem& P, bool f64, const uint8_t* label, const void* tables,
                                unsigned long long* tailmax, hipStream_t st) {
  int lmax = 1;
  for (int i = 0; i < P.n; ++i) lmax = P.L[i] > lmax ? P.L[i] : lmax;
  const double* wg = (const double*)((const char*)tables + memo_wg_offset(P, amy_memo_rec(lmax), f64 ? 8 : 4));
  const dim3 g((unsigned)((P.n_x + TAIL_MEMO_BLOCK - 1) / TAIL_MEMO_BLOCK)), b(TAIL_MEMO_BLOCK);
  const size_t lds = amy_tail_memo_lds(P);
  switch (P.n) {
#define T(NN) \
  case NN: hipLaunchKernelGGL((k_tail_memo<NN>), g, b, lds, st, P, label, wg, tailmax); break;
    T(1) T(2) T(3) T(4) T(5) T(6) T(7) T(8)
#undef T
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t amy_launch_memo_build(const DevProblem& P, bool f64, void* tables, hipStream_t st) {
#define X(K, SH) \
  if (FixedLaunch<K, SH>::matches(P)) return FixedLaunch<K, SH>::memo_build(P, f64, tables, st);
  AMY_FIXED_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}
