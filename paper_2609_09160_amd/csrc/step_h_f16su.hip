// step_h_f16su.hip -- instantiation unit of the D3Q27h step (the D3Q27 set
// with the complete Hermite basis) for one storage type.
#include "step_kernel.hpp"

namespace lbf {
hipError_t launch_step_h_f16su(int tile_rows, bool walls_y, bool ffield, const StepArgs& a,
                               hipStream_t s) {
  return launch_step_storage_full<kF16SU>(tile_rows, walls_y, ffield, a, s);
}
}  // namespace lbf
