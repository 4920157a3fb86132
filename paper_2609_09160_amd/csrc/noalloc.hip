// noalloc.hip -- the FP64 state reduction of lbfast_reduce without any device
// allocation, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops).  The per-block partial sums, which lbfast_reduce keeps
// in memory the library allocates at create, live here in a file-scope device
// array; every call on a device shares that device's copy.
#include <mutex>

#include "internal.hpp"
#include "lbfast.h"

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kScratchDoubles = static_cast<size_t>(lbf::kReduceBlocks) * 5;

// Per-block partials of the two-pass reduction (40 KiB per device).  In host
// code this name is only a stand-in for the symbol: the device address comes
// from hipGetSymbolAddress below, once per device.
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// device address of this device's scratch array (looked up on the first call
// made with `dev` current, then kept until the process ends)
hipError_t scratch_on(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

bool device_memory(const void* p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

int fail(int code, const char* msg) { return lbf::set_error(code, msg); }

}  // namespace

extern "C" int lbfast_reduce_noalloc(const void* state_dev, int storage, int64_t n_sites,
                                     const float scale[10], double* out_dev, void* stream) {
  lbf::clear_error();
  if (!state_dev || !out_dev) return fail(LBF_E_ARG, "state_dev and out_dev are required");
  if (storage != LBF_F64 && storage != LBF_F32 && storage != LBF_F16S && storage != LBF_BF16S &&
      storage != LBF_F16SU)
    return fail(LBF_E_ARG, "unknown storage");
  if (n_sites < 1 || static_cast<double>(n_sites) > 4.0e9)
    return fail(LBF_E_ARG, "n_sites must be in [1, 4e9] (the largest grid lbfast_create accepts)");
  const size_t eb = storage == LBF_F64 ? 8 : (storage == LBF_F32 ? 4 : 2);
  if (reinterpret_cast<uintptr_t>(state_dev) & (eb - 1))
    return fail(LBF_E_ARG, "state_dev is not aligned to its element size");
  if (reinterpret_cast<uintptr_t>(out_dev) & 7) return fail(LBF_E_ARG, "out_dev is misaligned");
  const bool s16 = storage == LBF_F16S || storage == LBF_BF16S || storage == LBF_F16SU;
  if (s16 && !scale) return fail(LBF_E_ARG, "16-bit storage needs its ten scales");
  if (!device_memory(state_dev) || !device_memory(out_dev))
    return fail(LBF_E_ARG, "state_dev and out_dev must be device memory");
  float sc[10];
  for (int k = 0; k < 10; ++k) sc[k] = (s16 && scale) ? scale[k] : 1.0f;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(LBF_E_DEVICE, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(LBF_E_UNSUPPORTED, "device index >= 64");
  double* partials = nullptr;
  e = scratch_on(dev, &partials);
  if (e != hipSuccess) return fail(LBF_E_DEVICE, hipGetErrorString(e));
  // every partial is written by the first pass: nothing needs clearing
  e = lbf::launch_reduce(storage, state_dev, n_sites, sc, partials, out_dev,
                         static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(LBF_E_DEVICE, hipGetErrorString(e));
  return LBF_OK;
}
