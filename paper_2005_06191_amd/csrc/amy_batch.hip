// amy_batch.hip -- many systems of uneven sizes in one launch.
//
// k_batch_init / k_batch_tail: labels and terminal values, then the FP64
// row-tail pass, over every system's 64-state tiles.
// k_batch_persistent: one cooperative launch runs every Bellman step of
// every system.  Systems are sorted by horizon (longest first), so the
// systems still active at global step s form a prefix; the work items of a
// phase are their tiles (64 states, or 64 / G states for the group
// variants).  Workgroups (one wave each) take items from atomic work queues
// -- one queue per XCD over a contiguous item range, stealing from the
// other XCDs' queues when their own is empty -- and a grid-wide barrier
// separates the phases (step 0 .. maxT-1).
// Every barrier wait is bounded: a wave that waits too long records an
// error and carries on, so the grid always drains.
//
// k_batch_step: one Bellman step for every system of a table (the serving
// loop's captured step); items are dealt to workgroups by a fixed stride.
//
// Each tile runs exactly the single-system kernels' per-state code
// (sweep_tile / stored_tile), so a system's result does not depend on what
// it is batched with.
#include <hip/hip_runtime.h>

#include "amy_generic.hpp"

#define BATCH_BLOCK 64

// The (dynamics, dimension) pairs a batched launch can hold, in two sets:
// the 2-D / 3-D set of the batch workload and every built-in family.  Each
// launch is instantiated for one set, so a batch of small systems does not
// carry the register budget of the 5-D and 7-D code.
#define AMY_BATCH_FAMILIES_SMALL(X)                                                              \
  X(AMY_DYN_AFFINE_, 1) X(AMY_DYN_AFFINE_, 2) X(AMY_DYN_AFFINE_, 3) X(AMY_DYN_AFFINE_, 4)         \
  X(AMY_DYN_UNICYCLE_, 3)
#define AMY_BATCH_FAMILIES(X)                                                                    \
  AMY_BATCH_FAMILIES_SMALL(X)                                                                    \
  X(AMY_DYN_ROOM_, 2) X(AMY_DYN_ROOM_, 3) X(AMY_DYN_ROOM_, 4) X(AMY_DYN_ROOM_, 5) X(AMY_DYN_VEHICLE7_, 7)

// Every per-state call below is inlined: the system descriptor is then read
// through a wave-uniform index, so its fields live in scalar registers (an
// out-of-line call would see them as per-lane values).
template <int KIND, int N, int G, class MT, class AT, class VI, class VO, bool COMP, bool TAIL>
__device__ __forceinline__ void call_variant(const DevProblem& P, uint32_t s, const VI* Vin, VO* Vout,
                                             const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                                             unsigned char* smem) {
  if constexpr (G == 1)
    sweep_tile<KIND, N, MT, AT, VI, VO, COMP, TAIL, false>(P, s, Vin, Vout, label, pol, tailmax, smem);
  else
    sweep_group<KIND, N, MT, AT, VI, VO, COMP, TAIL, G, false>(P, s, Vin, Vout, label, pol, tailmax, smem);
}

template <int KIND, int N, int G, bool F64>
__device__ __forceinline__ void run_otf_g(const BatchSys& B, uint32_t s, int t, unsigned char* smem) {
  const DevProblem& P = B.P;
  const int k = B.horizon - t;
  const bool last = (k == 1);
  int16_t* pol = B.pol ? B.pol + (int64_t)(k - 1) * P.n_x : nullptr;
  // the FP64 tail is a pass of its own (k_batch_tail / the server's start),
  // so the steps carry no tail code and keep their register budget low
  if constexpr (F64) {
    const double* Vin = (const double*)((t & 1) ? B.V1 : B.V0);
    double* Vo = last ? B.Vout : (double*)((t & 1) ? B.V0 : B.V1);
    call_variant<KIND, N, G, double, double, double, double, false, false>(P, s, Vin, Vo, B.label, pol, B.tailmax, smem);
  } else {
    const float* Vin = (const float*)((t & 1) ? B.V1 : B.V0);
    if (last)
      call_variant<KIND, N, G, float, double, float, double, false, false>(P, s, Vin, B.Vout, B.label, pol, B.tailmax, smem);
    else
      call_variant<KIND, N, G, float, float, float, float, true, false>(P, s, Vin, (float*)((t & 1) ? B.V0 : B.V1), B.label, pol, B.tailmax, smem);
  }
}

template <int KIND, int N, bool F64>
__device__ __forceinline__ void run_otf(const BatchSys& B, uint32_t tile, int t, unsigned char* smem) {
  // the host plans every batched system as LANES (1) or GROUP64 (64)
  if (B.P.grp_g == 64) run_otf_g<KIND, N, 64, F64>(B, tile, t, smem);
  else run_otf_g<KIND, N, 1, F64>(B, tile * BATCH_BLOCK + (threadIdx.x & 63), t, smem);
}

template <int N, bool F64>
__device__ __forceinline__ void run_stored(const BatchSys& B, uint32_t s, int t) {
  const DevProblem& P = B.P;
  const int k = B.horizon - t;
  const bool last = (k == 1);
  int16_t* pol = B.pol ? B.pol + (int64_t)(k - 1) * P.n_x : nullptr;
  if constexpr (F64) {
    stored_tile<N, double, double, double, double, false>(P, s, (const double*)B.T, B.org,
                                                          (const double*)((t & 1) ? B.V1 : B.V0),
                                                          last ? B.Vout : (double*)((t & 1) ? B.V0 : B.V1),
                                                          B.label, pol);
  } else if (last) {
    stored_tile<N, float, double, float, double, false>(P, s, (const float*)B.T, B.org,
                                                        (const float*)((t & 1) ? B.V1 : B.V0), B.Vout, B.label, pol);
  } else {
    stored_tile<N, float, float, float, float, true>(P, s, (const float*)B.T, B.org,
                                                     (const float*)((t & 1) ? B.V1 : B.V0),
                                                     (float*)((t & 1) ? B.V0 : B.V1), B.label, pol);
  }
}

// One tile of system B at its local step t (0 = the step k = T_d).  FS: the
// family set compiled in (0: 2-D / 3-D, 1: all); STORED: stored rows too.
template <bool F64, int FS, bool STORED>
__device__ __forceinline__ void run_tile(const BatchSys& B, uint32_t tile, int t, unsigned char* smem) {
  const uint32_t s = tile * BATCH_BLOCK + (threadIdx.x & 63);
  if constexpr (STORED) {
    if (B.mode == 1) {  // AMY_MODE_STORED: rows were built at admission
      switch (B.P.n) {
        case 1: run_stored<1, F64>(B, s, t); return;
        case 2: run_stored<2, F64>(B, s, t); return;
        case 3: run_stored<3, F64>(B, s, t); return;
        case 4: run_stored<4, F64>(B, s, t); return;
        case 5: run_stored<5, F64>(B, s, t); return;
        case 7: run_stored<7, F64>(B, s, t); return;
      }
      return;
    }
  }
#define X(K, N_) \
  case K * 16 + N_: run_otf<K, N_, F64>(B, tile, t, smem); return;
  if constexpr (FS == 0) {
    switch (B.P.kind * 16 + B.P.n) { AMY_BATCH_FAMILIES_SMALL(X) }
  } else {
    switch (B.P.kind * 16 + B.P.n) { AMY_BATCH_FAMILIES(X) }
  }
#undef X
}

bool amy_batch_supports(int kind, int n, int mode) {
  if (mode == 1) return n == 1 || n == 2 || n == 3 || n == 4 || n == 5 || n == 7;
#define X(K, N_) \
  if (kind == K && n == N_) return true;
  AMY_BATCH_FAMILIES(X)
#undef X
  return false;
}

int amy_batch_family_set(int kind, int n) {
#define X(K, N_) \
  if (kind == K && n == N_) return 0;
  AMY_BATCH_FAMILIES_SMALL(X)
#undef X
  return 1;
}

// FP64 row tails of one 64-state tile of system B, max into B.tailmax.
template <int FS>
__device__ __forceinline__ void tail_tile(const BatchSys& B, uint32_t tile) {
  const uint32_t s = tile * BATCH_BLOCK + (threadIdx.x & 63);
  double tmax = 0.0;
#define X(K, N_) \
  case K * 16 + N_: tmax = tail_state<K, N_, false>(B.P, s, B.label); break;
  if constexpr (FS == 0) {
    switch (B.P.kind * 16 + B.P.n) { AMY_BATCH_FAMILIES_SMALL(X) }
  } else {
    switch (B.P.kind * 16 + B.P.n) { AMY_BATCH_FAMILIES(X) }
  }
#undef X
  wave_max_to(tmax, B.tailmax);
}

template <bool F64>
__device__ __forceinline__ void init_tile(const BatchSys& B, uint32_t tile) {
  const uint32_t s = tile * BATCH_BLOCK + (threadIdx.x & 63);
  if (tile == 0 && threadIdx.x == 0 && B.tailmax) *B.tailmax = 0ull;
  if (s >= (uint32_t)B.P.n_x) return;
  double v;
  B.label[s] = init_state(B.P, s, v);
  if constexpr (F64) ((double*)B.V0)[s] = v;
  else ((float*)B.V0)[s] = (float)v;
  if (B.horizon == 0) B.Vout[s] = v;
}

// Item i of a phase -> (system, tile) through the tile prefix sums.
__device__ __forceinline__ int find_sys(const int32_t* __restrict__ tprefix, int nsys, uint32_t item) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((uint32_t)tprefix[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);  // item is wave-uniform, so is the system
}

// Grid-wide barrier over nblocks co-resident workgroups.  Arrival is an
// acquire-release add (publishes this workgroup's V writes); the waiters
// poll the generation with relaxed loads and a sleep between polls -- an
// acquire load per poll would invalidate the local caches every time, and
// thousands of polling waves would starve the working ones -- and take one
// acquire fence when it moves.  Bounded wait: on timeout the error flag is
// set and the wave carries on, so the grid always drains.
__device__ __forceinline__ void grid_barrier(BatchCtl* ctl, unsigned nblocks, unsigned& gen) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned a = __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (a == nblocks - 1) {
      __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&ctl->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(8);
        if (++spins > (1u << 24)) {
          atomicOr(&ctl->err, 1u);
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  ++gen;
  __syncthreads();
}

// Next chunk of items of a phase: this XCD's queue first, then the others'.
// Item range of XCD q: [q*n/8, (q+1)*n/8).  Returns false when all are done.
__device__ __forceinline__ bool grab(BatchCtl* ctl, int phase, uint32_t nitems, int chunk, bool xcd_order,
                                     int& q, uint32_t& first, uint32_t& last) {
  while (q < 8) {
    unsigned v = 0;
    const int qq = xcd_order ? ((int)(blockIdx.x & 7u) + q) & 7 : 0;
    const uint32_t lo = xcd_order ? (uint32_t)(((uint64_t)nitems * qq) / 8) : 0u;
    const uint32_t hi = xcd_order ? (uint32_t)(((uint64_t)nitems * (qq + 1)) / 8) : nitems;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(&ctl->ctr[phase * 8 + qq], (unsigned)chunk);
    v = __builtin_amdgcn_readfirstlane(v);  // wave-uniform from here on
    if (lo + v < hi) {
      first = lo + v;
      last = min(hi, first + (uint32_t)chunk);
      return true;
    }
    if (!xcd_order) return false;
    ++q;
  }
  return false;
}

template <bool F64, int FS>
__global__ void __launch_bounds__(BATCH_BLOCK) k_batch_persistent(const BatchSys* __restrict__ sys, int nsys,
                                                                  const int32_t* __restrict__ tprefix,
                                                                  const int32_t* __restrict__ active,
                                                                  int max_steps, BatchCtl* ctl, int chunk,
                                                                  int xcd_order) {
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned gen = 0;
  for (int phase = 0; phase < max_steps; ++phase) {
    const int nact = active[phase];
    const uint32_t nitems = (uint32_t)tprefix[nact];
    int q = 0;
    uint32_t first, last;
    while (grab(ctl, phase, nitems, chunk, xcd_order != 0, q, first, last)) {
      for (uint32_t it = first; it < last; ++it) {
        const int j = find_sys(tprefix, nact, it);
        run_tile<F64, FS, false>(sys[j], it - (uint32_t)tprefix[j], phase, smem);
      }
    }
    if (phase + 1 < max_steps) grid_barrier(ctl, gridDim.x, gen);
  }
}

// One step of every system of a table (the serving loop's captured step).
// meta[0] = number of systems, meta[1 ..] = their tile prefix sums;
// BatchSys::step_base holds each system's local step t for this launch.
// Both are read from device memory, so one captured launch serves any set
// of active systems.  Items are dealt by a fixed stride (no counters).
template <bool F64, int FS>
__global__ void __launch_bounds__(BATCH_BLOCK) k_batch_step(const BatchSys* __restrict__ sys,
                                                            const int32_t* __restrict__ meta) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nsys = meta[0];
  const int32_t* tprefix = meta + 1;
  const uint32_t nitems = (uint32_t)tprefix[nsys];
  for (uint32_t it = xcd_block(blockIdx.x, gridDim.x); it < nitems; it += gridDim.x) {
    const int j = find_sys(tprefix, nsys, it);
    const BatchSys& B = sys[j];
    if (B.step_base < 0 || B.step_base >= B.horizon) continue;
    run_tile<F64, FS, true>(B, it - (uint32_t)tprefix[j], B.step_base, smem);
  }
}

// Labels and terminal values of every system (64-state tiles, tp64 their
// prefix sums).
template <bool F64>
__global__ void __launch_bounds__(BATCH_BLOCK) k_batch_init(const BatchSys* __restrict__ sys, int nsys,
                                                            const int32_t* __restrict__ tp64) {
  const uint32_t nitems = (uint32_t)tp64[nsys];
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int j = find_sys(tp64, nsys, it);
    init_tile<F64>(sys[j], it - (uint32_t)tp64[j]);
  }
}

// FP64 tail pass of the systems that want it (after k_batch_init).
template <int FS>
__global__ void __launch_bounds__(BATCH_BLOCK) k_batch_tail(const BatchSys* __restrict__ sys, int nsys,
                                                            const int32_t* __restrict__ tp64) {
  const uint32_t nitems = (uint32_t)tp64[nsys];
  for (uint32_t it = xcd_block(blockIdx.x, gridDim.x); it < nitems; it += gridDim.x) {
    const int j = find_sys(tp64, nsys, it);
    if (sys[j].want_tail) tail_tile<FS>(sys[j], it - (uint32_t)tp64[j]);
  }
}

// After a persistent launch: if a grid-barrier wait gave up, every
// system's FP64 output becomes NaN, so a caller that does not read the
// control block (the asynchronous mode) still cannot take invalid values
// for results.  Block b handles systems b, b + gridDim.x, ...
__global__ void __launch_bounds__(256) k_batch_poison(const BatchSys* __restrict__ sys, int nsys,
                                                      const BatchCtl* __restrict__ ctl) {
  if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;
  const double nan = __builtin_nan("");
  for (int j = blockIdx.x; j < nsys; j += gridDim.x) {
    double* v = sys[j].Vout;
    const int64_t n = sys[j].P.n_x;
    for (int64_t s = threadIdx.x; s < n; s += blockDim.x) v[s] = nan;
  }
}

__global__ void k_fill_u32(unsigned* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ------------------------------------------------------------- launchers

const void* amy_batch_persistent_kernel(bool f64, int fs) {
  if (fs == 0) return f64 ? (const void*)&k_batch_persistent<true, 0> : (const void*)&k_batch_persistent<false, 0>;
  return f64 ? (const void*)&k_batch_persistent<true, 1> : (const void*)&k_batch_persistent<false, 1>;
}

hipError_t amy_launch_batch_persistent(bool f64, int fs, unsigned grid, size_t lds, const BatchSys* sys, int nsys,
                                       const int32_t* tprefix, const int32_t* active, int max_steps,
                                       BatchCtl* ctl, int chunk, int xcd_order, hipStream_t st) {
  void* args[] = {(void*)&sys, (void*)&nsys, (void*)&tprefix, (void*)&active, (void*)&max_steps,
                  (void*)&ctl, (void*)&chunk, (void*)&xcd_order};
  return hipLaunchCooperativeKernel(amy_batch_persistent_kernel(f64, fs), dim3(grid), dim3(BATCH_BLOCK), args,
                                    (unsigned)lds, st);
}

const void* amy_batch_step_kernel(bool f64, int fs) {
  if (fs == 0) return f64 ? (const void*)&k_batch_step<true, 0> : (const void*)&k_batch_step<false, 0>;
  return f64 ? (const void*)&k_batch_step<true, 1> : (const void*)&k_batch_step<false, 1>;
}

hipError_t amy_launch_batch_step(bool f64, int fs, unsigned grid, size_t lds, const BatchSys* sys,
                                 const int32_t* meta, hipStream_t st) {
  const dim3 g(grid), b(BATCH_BLOCK);
  if (fs == 0) {
    if (f64) hipLaunchKernelGGL((k_batch_step<true, 0>), g, b, lds, st, sys, meta);
    else hipLaunchKernelGGL((k_batch_step<false, 0>), g, b, lds, st, sys, meta);
  } else {
    if (f64) hipLaunchKernelGGL((k_batch_step<true, 1>), g, b, lds, st, sys, meta);
    else hipLaunchKernelGGL((k_batch_step<false, 1>), g, b, lds, st, sys, meta);
  }
  return hipGetLastError();
}

hipError_t amy_launch_batch_init(bool f64, const BatchSys* sys, int nsys, const int32_t* tprefix, unsigned grid,
                                 hipStream_t st) {
  if (f64) hipLaunchKernelGGL((k_batch_init<true>), dim3(grid), dim3(BATCH_BLOCK), 0, st, sys, nsys, tprefix);
  else hipLaunchKernelGGL((k_batch_init<false>), dim3(grid), dim3(BATCH_BLOCK), 0, st, sys, nsys, tprefix);
  return hipGetLastError();
}

hipError_t amy_launch_batch_tail(int fs, const BatchSys* sys, int nsys, const int32_t* tp64, unsigned grid,
                                 hipStream_t st) {
  if (fs == 0) hipLaunchKernelGGL((k_batch_tail<0>), dim3(grid), dim3(BATCH_BLOCK), 0, st, sys, nsys, tp64);
  else hipLaunchKernelGGL((k_batch_tail<1>), dim3(grid), dim3(BATCH_BLOCK), 0, st, sys, nsys, tp64);
  return hipGetLastError();
}

hipError_t amy_launch_batch_poison(const BatchSys* sys, int nsys, const BatchCtl* ctl, hipStream_t st) {
  const unsigned g = (unsigned)(nsys < 1024 ? nsys : 1024);
  hipLaunchKernelGGL(k_batch_poison, dim3(g > 0 ? g : 1), dim3(256), 0, st, sys, nsys, ctl);
  return hipGetLastError();
}

hipError_t amy_launch_fill_u32(unsigned* p, size_t n, hipStream_t st) {
  const unsigned g = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_fill_u32, dim3(g > 0 ? g : 1), dim3(256), 0, st, p, n);
  return hipGetLastError();
}
