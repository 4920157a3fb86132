// adjoint_f32.hip -- instantiation unit of the adjoint step for F32 storage
// (split so the variants compile in parallel).
#include "adjoint_kernel.hpp"

namespace lbf {
hipError_t launch_adjoint_f32(int Q, int tile_rows, bool walls_y, bool ffield, const StepArgs& a,
                             hipStream_t s) {
  return launch_adjoint_type<float>(Q, tile_rows, walls_y, ffield, a, s);
}
}  // namespace lbf
