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
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ VBuf(const VT* p, uint32_t n)
      : r(__builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(n * (uint32_t)sizeof(VT)), 0x00020000)) {}
  __device__ __forceinline__ VT load(uint32_t voff, uint32_t soff) const;
};
template <>
__device__ __forceinline__ float VBuf<float>::load(uint32_t voff, uint32_t soff) const {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double VBuf<double>::load(uint32_t voff, uint32_t soff) const {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
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
template <int D, class SH, class MT, class AT, class VT, bool COMP>
__device__ __forceinline__ AT contract_fixed(const DevProblem& P, const FixedRow<SH, MT>& R,
                                             const VBuf<VT>& vb, uint32_t voff, uint32_t soff);

template <int D, class SH, class MT, class AT, class VT, bool COMP>
__device__ __forceinline__ void contract_step(const DevProblem& P, const FixedRow<SH, MT>& R,
                                              const VBuf<VT>& vb, uint32_t voff, uint32_t soff, int k,
                                              AT& acc, AT& c) {
  AT inner;
  if constexpr (D == SH::N - 1) {
    inner = AT(vb.load(voff + (uint32_t)(k * sizeof(VT)), soff));
  } else {
    inner = contract_fixed<D + 1, SH, MT, AT, VT, COMP>(
        P, R, vb, voff, soff + (uint32_t)k * (uint32_t)P.stride[D] * (uint32_t)sizeof(VT));
  }
  // mass of slot k; in a loop level k is a uniform register, so pick it
  // with selects rather than an indexed (scratch) access
  MT mk;
  if constexpr (D < SH::BL) {
    mk = R.m[D][0];
#pragma unroll
    for (int j = 1; j < SH::L[D]; ++j) mk = (k == j) ? R.m[D][j] : mk;
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

template <int D, class SH, class MT, class AT, class VT, bool COMP>
__device__ __forceinline__ AT contract_fixed(const DevProblem& P, const FixedRow<SH, MT>& R,
                                             const VBuf<VT>& vb, uint32_t voff, uint32_t soff) {
  constexpr int L = SH::L[D];
  AT acc = AT(0), c = AT(0);
  if constexpr (D < SH::BL) {
#pragma clang loop unroll(disable)
    for (int k = 0; k < L; ++k) contract_step<D, SH, MT, AT, VT, COMP>(P, R, vb, voff, soff, k, acc, c);
  } else {
#pragma unroll
    for (int k = 0; k < L; ++k) contract_step<D, SH, MT, AT, VT, COMP>(P, R, vb, voff, soff, k, acc, c);
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
      build_cached<KIND, N, MT, TAIL, FIX_BLOCK>(P, st, x, S);
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
        const AT q = contract_fixed<0, SH, MT, AT, VI, COMP>(P, R, vb, base * (uint32_t)sizeof(VI), 0u);
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
    for (int off = 32; off > 0; off >>= 1) tmax = fmax(tmax, __shfl_xor(tmax, off));
    if ((threadIdx.x & 63) == 0 && tmax > 0.0)
      atomicMax(tailmax, (unsigned long long)__double_as_longlong(tmax));
  }
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
  template <class MT, class AT, class VI, class VO, bool COMP>
  static void go(const DevProblem& P, const void* Vin, void* Vout, const uint8_t* label, int16_t* pol,
                 unsigned long long* tailmax, hipStream_t st) {
    const dim3 g((unsigned)((P.n_x + FIX_BLOCK - 1) / FIX_BLOCK)), b(FIX_BLOCK);
    if (tailmax)
      hipLaunchKernelGGL((k_sweep_fixed<KIND, SH, MT, AT, VI, VO, COMP, true>), g, b, P.lds_bytes_tail, st, P,
                         (const VI*)Vin, (VO*)Vout, label, pol, tailmax);
    else
      hipLaunchKernelGGL((k_sweep_fixed<KIND, SH, MT, AT, VI, VO, COMP, false>), g, b, P.lds_bytes_fixed, st, P,
                         (const VI*)Vin, (VO*)Vout, label, pol, tailmax);
  }
  static hipError_t sweep(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout, const uint8_t* label,
                          int16_t* pol, unsigned long long* tailmax, hipStream_t st) {
    switch (sk) {
      case SWEEP_F64: go<double, double, double, double, false>(P, Vin, Vout, label, pol, tailmax, st); break;
      case SWEEP_F32: go<float, float, float, float, true>(P, Vin, Vout, label, pol, tailmax, st); break;
      case SWEEP_F32_LAST: go<float, double, float, double, false>(P, Vin, Vout, label, pol, tailmax, st); break;
    }
    return hipGetLastError();
  }
};

// Window shapes of the workload families (2-D linear, 3-D unicycle, 5-D
// room ring, 7-D vehicle).
// (first argument: the most gathers issued as one unrolled block)
using ShapeUnicycle = ShapeT<64, 5, 5, 2>;
using ShapeRoom5 = ShapeT<27, 3, 3, 3, 3, 3>;
using ShapeVehicle7 = ShapeT<27, 2, 2, 3, 3, 3, 3, 3>;
using ShapeLinear2 = ShapeT<28, 28, 28>;
#define AMY_FIXED_SHAPES(X)            \
  X(AMY_DYN_UNICYCLE_, ShapeUnicycle)  \
  X(AMY_DYN_ROOM_, ShapeRoom5)         \
  X(AMY_DYN_VEHICLE7_, ShapeVehicle7)  \
  X(AMY_DYN_AFFINE_, ShapeLinear2)

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

hipError_t amy_launch_sweep_fixed(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                                  const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                                  hipStream_t st) {
#define X(K, SH) \
  if (FixedLaunch<K, SH>::matches(P)) return FixedLaunch<K, SH>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
  AMY_FIXED_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}
