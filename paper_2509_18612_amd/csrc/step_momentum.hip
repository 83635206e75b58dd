// Step kernels with heavy-ball momentum (V' = mu V + G, X' = Proj(X + eta V'); the paper
// runs PGA with momentum, Sec. 4.2 and Sec. 5). The kernel templates are those of
// kernels.hip; this translation unit instantiates only their velocity variants and the
// launcher for them, so they compile in parallel with the plain ones.
#define DECO_KERNELS_ONLY_TU 1
#include "kernels.hip"

namespace deco {

hipError_t launch_step_momentum(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s) {
  return launch_step_impl<true>(a, dtype, vec, grid, s);
}

}  // namespace deco
