// step_f16su.hip -- instantiation unit of the fused step for one storage type
// (split so the variants compile in parallel).
#include "step_kernel.hpp"

namespace lbf {
hipError_t launch_step_f16su(int Q, int tile_rows, bool walls_y, bool ffield, const StepArgs& a,
                             hipStream_t s) {
  return launch_step_storage<kF16SU>(Q, tile_rows, walls_y, ffield, a, s);
}
}  // namespace lbf
