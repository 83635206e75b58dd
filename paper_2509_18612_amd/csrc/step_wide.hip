// Plain step kernels of 5 to 8 lifted components per initialisation (dispatch in
// step_wide.inc); the momentum variants are instantiated in step_wide_momentum.hip.
#define DECO_KERNELS_ONLY_TU 1
#include "kernels.hip"
#include "step_wide.inc"

namespace deco {

hipError_t launch_step_wide(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s) {
  return a.vel != nullptr ? launch_step_wide_momentum(a, dtype, vec, grid, s) : wide<false>(a, dtype, vec, grid, s);
}

}  // namespace deco
