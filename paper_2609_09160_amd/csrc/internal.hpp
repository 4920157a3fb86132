// internal.hpp -- declarations shared by the host runtime (lbfast.cpp) and
// the kernel launchers (*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbf {

// Arguments of one fused step launch (by value into the kernel).
struct StepArgs {
  const void* src;     // current moment buffer (10 planes)
  void* dst;           // next moment buffer (10 planes)
  const void* Ffield;  // 3 planes of the compute type, or nullptr (uniform F)
  int nx, ny, nz;
  int64_t N;           // plane stride = nx*ny*nz
  int tiles_x, tiles_y, zchunks, zchunk;
  double omega;
  double F[3];         // uniform force (used when Ffield == nullptr)
  float scale[10];     // 16-bit storage: value = scale * q
  float inv_scale[10];
};

// rows per tile supported by the step kernel
constexpr int kTileRowsSupported[] = {4, 6, 8, 14};

// Launch one fused step.  Returns hipErrorInvalidValue for an unsupported
// combination.  nblocks = tiles_x * tiles_y * zchunks.
hipError_t launch_step(int Q, int storage, int tile_rows, bool walls_y, const StepArgs& a,
                       hipStream_t stream);

// copy nplanes planes of n floats (n * 4 < 2^32) with the step's memory
// instruction forms
hipError_t launch_stream_probe(const void* src, void* dst, int64_t n, int nplanes,
                               hipStream_t stream);

// user array (F64 or F32, 10 planes) -> storage buffer
hipError_t launch_encode(int storage, int user_dtype, const void* user, void* buf, int64_t N,
                         int64_t plane_offset, int64_t nplanes, const float* inv_scale,
                         hipStream_t stream);
// storage buffer -> user array
hipError_t launch_decode(int storage, int user_dtype, const void* buf, void* user, int64_t N,
                         int64_t plane_offset, int64_t nplanes, const float* scale,
                         hipStream_t stream);
// per-plane max |v| of a user array (10 planes) into out_bits[10] (float bits,
// must be zeroed before)
hipError_t launch_maxabs(int user_dtype, const void* user, int64_t N, int64_t plane_offset,
                         int64_t nplanes, unsigned* out_bits, hipStream_t stream);
// FP64 sums [a0, a1x, a1y, a1z, 1/2 |a1|^2] of the state into out[5]
// (partials: kReduceBlocks*5 doubles of scratch)
constexpr int kReduceBlocks = 1024;
hipError_t launch_reduce(int storage, const void* buf, int64_t N, const float* scale,
                         double* partials, double* out, hipStream_t stream);

}  // namespace lbf
