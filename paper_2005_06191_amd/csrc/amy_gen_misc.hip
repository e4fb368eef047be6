// amy_gen_misc.hip -- generic-window kernels of the unicycle, 7-D vehicle and
// planar robot families.
#include "amy_generic.hpp"

hipError_t amy_gen_unicycle_tail(const DevProblem& P, const uint8_t* label, unsigned long long* tailmax,
                              hipStream_t st) {
  switch (P.n) {
    case 3: return Launch<AMY_DYN_UNICYCLE_, 3>::tail(P, label, tailmax, st);
  }
  return hipErrorInvalidValue;
}

hipError_t amy_gen_unicycle_sweep(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                               const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                               hipStream_t st) {
  switch (P.n) {
    case 3: return Launch<AMY_DYN_UNICYCLE_, 3>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
  }
  return hipErrorInvalidValue;
}

hipError_t amy_gen_unicycle_build(const DevProblem& P, bool f64, const uint8_t* label, void* T, int32_t* org,
                               unsigned long long* tailmax, hipStream_t st) {
  switch (P.n) {
    case 3: return Launch<AMY_DYN_UNICYCLE_, 3>::build(P, f64, label, T, org, tailmax, st);
  }
  return hipErrorInvalidValue;
}


hipError_t amy_gen_vehicle7_tail(const DevProblem& P, const uint8_t* label, unsigned long long* tailmax,
                              hipStream_t st) {
  switch (P.n) {
    case 7: return Launch<AMY_DYN_VEHICLE7_, 7>::tail(P, label, tailmax, st);
  }
  return hipErrorInvalidValue;
}

hipError_t amy_gen_vehicle7_sweep(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                               const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                               hipStream_t st) {
  switch (P.n) {
    case 7: return Launch<AMY_DYN_VEHICLE7_, 7>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
  }
  return hipErrorInvalidValue;
}

hipError_t amy_gen_vehicle7_build(const DevProblem& P, bool f64, const uint8_t* label, void* T, int32_t* org,
                               unsigned long long* tailmax, hipStream_t st) {
  switch (P.n) {
    case 7: return Launch<AMY_DYN_VEHICLE7_, 7>::build(P, f64, label, T, org, tailmax, st);
  }
  return hipErrorInvalidValue;
}

hipError_t amy_gen_unicycle_group(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                               const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                               hipStream_t st) {
  if (P.n == 3) return Launch<AMY_DYN_UNICYCLE_, 3>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
  return hipErrorInvalidValue;
}

hipError_t amy_gen_vehicle7_group(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                               const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                               hipStream_t st) {
  if (P.n == 7) return Launch<AMY_DYN_VEHICLE7_, 7>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
  return hipErrorInvalidValue;
}

hipError_t amy_gen_robot_tail(const DevProblem& P, const uint8_t* label, unsigned long long* tailmax, hipStream_t st) {
  if (P.n == 2) return Launch<AMY_DYN_ROBOT_, 2>::tail(P, label, tailmax, st);
  return hipErrorInvalidValue;
}

hipError_t amy_gen_robot_sweep(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout, const uint8_t* label,
                               int16_t* pol, unsigned long long* tailmax, hipStream_t st) {
  if (P.n == 2) return Launch<AMY_DYN_ROBOT_, 2>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
  return hipErrorInvalidValue;
}

hipError_t amy_gen_robot_build(const DevProblem& P, bool f64, const uint8_t* label, void* T, int32_t* org,
                               unsigned long long* tailmax, hipStream_t st) {
  if (P.n == 2) return Launch<AMY_DYN_ROBOT_, 2>::build(P, f64, label, T, org, tailmax, st);
  return hipErrorInvalidValue;
}

hipError_t amy_gen_robot_group(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout, const uint8_t* label,
                               int16_t* pol, unsigned long long* tailmax, hipStream_t st) {
  if (P.n == 2) return Launch<AMY_DYN_ROBOT_, 2>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
  return hipErrorInvalidValue;
}
