// Step kernels of 5 to 8 lifted components per initialisation (Sec. 3.2: the lifted problem
// runs the same projected gradient step on l columns per initialisation and rounds on the
// sign of their sum). The kernel templates are those of kernels.hip; this translation unit
// instantiates only the wide component counts, plain and with momentum, so they compile in
// parallel with the others. Rows hold one gather slot per window (8 loads in flight per lane
// divided among the components), four values per lane, or one for one-element lanes.
#define DECO_KERNELS_ONLY_TU 1
#include "kernels.hip"

namespace deco {
namespace {

template <typename T, int VEC, bool MOM>
hipError_t wide_l(const StepArgs& a, int wmode, int grid, hipStream_t s) {
  switch (a.L) {
    case 5: return step_dispatch<T, VEC, 5, MOM>(a, wmode, grid, s);
    case 6: return step_dispatch<T, VEC, 6, MOM>(a, wmode, grid, s);
    case 7: return step_dispatch<T, VEC, 7, MOM>(a, wmode, grid, s);
    case 8: return step_dispatch<T, VEC, 8, MOM>(a, wmode, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <bool MOM>
hipError_t wide(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s) {
  const int wmode = step_weight_mode(a);
  if (dtype == 0) {
    if (vec == 4) return wide_l<float, 4, MOM>(a, wmode, grid, s);
    if (vec == 1) return wide_l<float, 1, MOM>(a, wmode, grid, s);
  } else {
    if (vec == 4) return wide_l<uint16_t, 4, MOM>(a, wmode, grid, s);
    if (vec == 1) return wide_l<uint16_t, 1, MOM>(a, wmode, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_step_wide(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s) {
  return a.vel != nullptr ? wide<true>(a, dtype, vec, grid, s) : wide<false>(a, dtype, vec, grid, s);
}

}  // namespace deco
