// amy_static.hip -- amy_solve_static: the single-problem solve on a
// workspace that the library keeps in device memory of its own, for callers
// that cannot allocate (code under stream capture, tight serving loops).
//
// The workspace is the file-scope array `scratch` below (AMY_STATIC_BYTES,
// 256-byte aligned).  Host code never uses the array's name as an address:
// the first call on a device, with that device current, asks the runtime for
// the device address of that device's copy and keeps it; every launch takes
// that pointer, exactly as amy_solve takes the caller's workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/amytiss.h"
#include "amy_host.hpp"

static __device__ __align__(256) unsigned char scratch[AMY_STATIC_WORKSPACE_BYTES];

static const int MAX_DEVICES = 64;
static std::mutex g_mu;
static void* g_ptr[MAX_DEVICES];

// Device address of the current device's copy of `scratch` (looked up once
// per device).
static amy_status scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return amy_hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return amy_fail(AMY_E_UNSUPPORTED, "device ordinal %d >= %d", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return amy_hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p & 255)) return amy_fail(AMY_E_DEVICE, "static workspace address not 256-byte aligned");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return AMY_OK;
}

extern "C" amy_status amy_solve_static(const amy_problem* p, void* stream, double* V_out, int16_t* policy_out) {
  amy_status st = amy_validate(p);
  if (st != AMY_OK) return st;
  if (p->dyn.kind == AMY_DYN_USER) return amy_fail(AMY_E_INVALID, "dynamics given as text are solved with amy_solve_user");
  if (!V_out) return amy_fail(AMY_E_INVALID, "V_out is NULL");
  Plan pl;
  st = amy_resolve(p, AMY_STATIC_WORKSPACE_BYTES, &pl);
  if (st == AMY_E_NOMEM)
    return amy_fail(AMY_E_NOMEM, "problem needs a %llu B workspace; the static workspace holds %llu B",
                    (unsigned long long)pl.ws_bytes, (unsigned long long)AMY_STATIC_WORKSPACE_BYTES);
  if (st != AMY_OK) return st;
  if (pl.ws_bytes > AMY_STATIC_WORKSPACE_BYTES)
    return amy_fail(AMY_E_NOMEM, "problem needs a %llu B workspace; the static workspace holds %llu B",
                    (unsigned long long)pl.ws_bytes, (unsigned long long)AMY_STATIC_WORKSPACE_BYTES);
  void* ws = nullptr;
  if ((st = scratch_ptr(&ws)) != AMY_OK) return st;
  // every region a solve reads is written by its own kernels first (labels,
  // both V buffers, the per-solve tables; the tail slot is cleared by the
  // init kernel), so nothing left by an earlier call needs clearing here
  return amy_enqueue(pl, (hipStream_t)stream, ws, V_out, policy_out, p->horizon, false, nullptr);
}
