// Step kernels of 5 to 8 lifted components per initialisation with heavy-ball momentum
// (dispatch in step_wide.inc).
#define DECO_KERNELS_ONLY_TU 1
#include "kernels.hip"
#include "step_wide.inc"

namespace deco {

hipError_t launch_step_wide_momentum(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s) {
  return wide<true>(a, dtype, vec, grid, s);
}

}  // namespace deco
