// amy_gen_affine.hip -- generic-window kernels of the affine dynamics family.
#include "amy_generic.hpp"

hipError_t amy_gen_affine_tail(const DevProblem& P, const uint8_t* label, unsigned long long* tailmax,
                              hipStream_t st) {
  switch (P.n) {
    case 1: return Launch<AMY_DYN_AFFINE_, 1>::tail(P, label, tailmax, st);
    case 2: return Launch<AMY_DYN_AFFINE_, 2>::tail(P, label, tailmax, st);
    case 3: return Launch<AMY_DYN_AFFINE_, 3>::tail(P, label, tailmax, st);
    case 4: return Launch<AMY_DYN_AFFINE_, 4>::tail(P, label, tailmax, st);
    case 5: return Launch<AMY_DYN_AFFINE_, 5>::tail(P, label, tailmax, st);
    case 6: return Launch<AMY_DYN_AFFINE_, 6>::tail(P, label, tailmax, st);
    case 7: return Launch<AMY_DYN_AFFINE_, 7>::tail(P, label, tailmax, st);
    case 8: return Launch<AMY_DYN_AFFINE_, 8>::tail(P, label, tailmax, st);
  }
  return hipErrorInvalidValue;
}

hipError_t amy_gen_affine_sweep(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                               const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                               hipStream_t st) {
  switch (P.n) {
    case 1: return Launch<AMY_DYN_AFFINE_, 1>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 2: return Launch<AMY_DYN_AFFINE_, 2>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 3: return Launch<AMY_DYN_AFFINE_, 3>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 4: return Launch<AMY_DYN_AFFINE_, 4>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 5: return Launch<AMY_DYN_AFFINE_, 5>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 6: return Launch<AMY_DYN_AFFINE_, 6>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 7: return Launch<AMY_DYN_AFFINE_, 7>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 8: return Launch<AMY_DYN_AFFINE_, 8>::sweep(P, sk, Vin, Vout, label, pol, tailmax, st);
  }
  return hipErrorInvalidValue;
}

hipError_t amy_gen_affine_build(const DevProblem& P, bool f64, const uint8_t* label, void* T, int32_t* org,
                               unsigned long long* tailmax, hipStream_t st) {
  switch (P.n) {
    case 1: return Launch<AMY_DYN_AFFINE_, 1>::build(P, f64, label, T, org, tailmax, st);
    case 2: return Launch<AMY_DYN_AFFINE_, 2>::build(P, f64, label, T, org, tailmax, st);
    case 3: return Launch<AMY_DYN_AFFINE_, 3>::build(P, f64, label, T, org, tailmax, st);
    case 4: return Launch<AMY_DYN_AFFINE_, 4>::build(P, f64, label, T, org, tailmax, st);
    case 5: return Launch<AMY_DYN_AFFINE_, 5>::build(P, f64, label, T, org, tailmax, st);
    case 6: return Launch<AMY_DYN_AFFINE_, 6>::build(P, f64, label, T, org, tailmax, st);
    case 7: return Launch<AMY_DYN_AFFINE_, 7>::build(P, f64, label, T, org, tailmax, st);
    case 8: return Launch<AMY_DYN_AFFINE_, 8>::build(P, f64, label, T, org, tailmax, st);
  }
  return hipErrorInvalidValue;
}

hipError_t amy_gen_affine_group(const DevProblem& P, SweepKind sk, const void* Vin, void* Vout,
                               const uint8_t* label, int16_t* pol, unsigned long long* tailmax,
                               hipStream_t st) {
  switch (P.n) {
    case 1: return Launch<AMY_DYN_AFFINE_, 1>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 2: return Launch<AMY_DYN_AFFINE_, 2>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 3: return Launch<AMY_DYN_AFFINE_, 3>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 4: return Launch<AMY_DYN_AFFINE_, 4>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 5: return Launch<AMY_DYN_AFFINE_, 5>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 6: return Launch<AMY_DYN_AFFINE_, 6>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 7: return Launch<AMY_DYN_AFFINE_, 7>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
    case 8: return Launch<AMY_DYN_AFFINE_, 8>::group(P, sk, Vin, Vout, label, pol, tailmax, st);
  }
  return hipErrorInvalidValue;
}
