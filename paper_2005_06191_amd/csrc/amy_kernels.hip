// amy_kernels.hip -- dispatch of the generic-window kernels by dynamics
// family, and the family-independent kernels (init, copy, stored sweep).
#include "amy_generic.hpp"

#define DECL_FAMILY(name)                                                                                \
  hipError_t amy_gen_##name##_tail(const DevProblem&, const uint8_t*, unsigned long long*, hipStream_t); \
  hipError_t amy_gen_##name##_sweep(const DevProblem&, SweepKind, const void*, void*, const uint8_t*,   \
                                    int16_t*, unsigned long long*, hipStream_t);                         \
  hipError_t amy_gen_##name##_build(const DevProblem&, bool, const uint8_t*, void*, int32_t*,           \
                                    unsigned long long*, hipStream_t);                                   \
  hipError_t amy_gen_##name##_group(const DevProblem&, SweepKind, const void*, void*, const uint8_t*,   \
                                    int16_t*, unsigned long long*, hipStream_t);
DECL_FAMILY(affine)
DECL_FAMILY(room)
DECL_FAMILY(unicycle)
DECL_FAMILY(vehicle7)
DECL_FAMILY(robot)

#define AMY_DISPATCH(OP, ...)                                                \
  switch (P.kind) {                                                           \
    case AMY_DYN_AFFINE_: return amy_gen_affine_##OP(__VA_ARGS__);           \
    case AMY_DYN_ROOM_: return amy_gen_room_##OP(__VA_ARGS__);               \
    case AMY_DYN_UNICYCLE_: return amy_gen_unicycle_##OP(__VA_ARGS__);       \
    case AMY_DYN_VEHICLE7_: return amy_gen_vehicle7_##OP(__VA_ARGS__);       \
    case AMY_DYN_ROBOT_: return amy_gen_robot_##OP(__VA_ARGS__);             \
  }                                                                           \
  return hipErrorInvalidValue;

hipError_t amy_launch_init(const DevProblem& P, uint8_t* label, void* V0, bool v0_double, double* Vout,
                           unsigned long long* tailmax, hipStream_t st) {
  return amy_launch_init_impl(P, label, V0, v0_double, Vout, tailmax, st);
}

hipError_t amy_launch_copy_out(int64_t n, const void* src, bool src_double, double* dst, hipStream_t st) {
  return amy_launch_copy_out_impl(n, src, src_double, dst, st);
}

hipError_t amy_launch_tail(const DevProblem& P, const uint8_t* label, unsigned long long* tailmax,
                           hipStream_t st) {
  AMY_DISPATCH(tail, P, label, tailmax, st)
}

hipError_t amy_launch_sweep_otf(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                                const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                                hipStream_t st) {
  AMY_DISPATCH(sweep, P, sk, Vin, Vout, label, pol, tailmax, st)
}

hipError_t amy_launch_sweep_group(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                                  const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                                  hipStream_t st) {
  AMY_DISPATCH(group, P, sk, Vin, Vout, label, pol, tailmax, st)
}

hipError_t amy_launch_build(const DevProblem& P, bool f64, const uint8_t* label, void* T, int32_t* org,
                            unsigned long long* tailmax, hipStream_t st) {
  AMY_DISPATCH(build, P, f64, label, T, org, tailmax, st)
}

hipError_t amy_launch_sweep_stored(const DevProblem& P, SweepKind sk, const void* T, const int32_t* org,
                                   const void* Vin, void* Vout, const uint8_t* label, int16_t* pol,
                                   hipStream_t st) {
  switch (P.n) {
    case 1: return sweep_stored_n<1>(P, sk, T, org, Vin, Vout, label, pol, st);
    case 2: return sweep_stored_n<2>(P, sk, T, org, Vin, Vout, label, pol, st);
    case 3: return sweep_stored_n<3>(P, sk, T, org, Vin, Vout, label, pol, st);
    case 4: return sweep_stored_n<4>(P, sk, T, org, Vin, Vout, label, pol, st);
    case 5: return sweep_stored_n<5>(P, sk, T, org, Vin, Vout, label, pol, st);
    case 6: return sweep_stored_n<6>(P, sk, T, org, Vin, Vout, label, pol, st);
    case 7: return sweep_stored_n<7>(P, sk, T, org, Vin, Vout, label, pol, st);
    case 8: return sweep_stored_n<8>(P, sk, T, org, Vin, Vout, label, pol, st);
  }
  return hipErrorInvalidValue;
}
