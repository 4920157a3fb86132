// aux.hip -- non-hot-path device work: conversion between user arrays and the
// storage format, per-plane max |v| for 16-bit scales, deterministic FP64
// reductions of the state (mass, momentum, kinetic energy), and the step
// dispatcher.
#include "internal.hpp"
#include "lattice.hpp"

namespace lbf {

hipError_t launch_step_f64(int, int, bool, bool, const StepArgs&, hipStream_t);
hipError_t launch_step_f32(int, int, bool, bool, const StepArgs&, hipStream_t);
hipError_t launch_step_f16s(int, int, bool, bool, const StepArgs&, hipStream_t);
hipError_t launch_step_bf16s(int, int, bool, bool, const StepArgs&, hipStream_t);

hipError_t launch_step(int Q, int storage, int tile_rows, bool walls_y, const StepArgs& a,
                       hipStream_t stream) {
  const bool ff = a.Ffield != nullptr;
  switch (storage) {
    case kF64: return launch_step_f64(Q, tile_rows, walls_y, ff, a, stream);
    case kF32: return launch_step_f32(Q, tile_rows, walls_y, ff, a, stream);
    case kF16S: return launch_step_f16s(Q, tile_rows, walls_y, ff, a, stream);
    case kBF16S: return launch_step_bf16s(Q, tile_rows, walls_y, ff, a, stream);
    default: return hipErrorInvalidValue;
  }
}

namespace {

constexpr int kThreads = 256;

// 10 scales passed by value
struct Scales {
  float v[10];
};

int grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return static_cast<int>(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

template <int ST, typename U>
__global__ void encode_kernel(const U* __restrict__ user, typename Storage<ST>::T* __restrict__ buf,
                              int64_t N, int64_t p0, Scales inv) {
  const int k = static_cast<int>(blockIdx.y);
  const int64_t base = (p0 + k) * N;
  const U* u = user + static_cast<int64_t>(k) * N;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    using C = typename Storage<ST>::C;
    const C v = static_cast<C>(u[i]);
    Storage<ST>::store(buf, base + i, v, inv.v[p0 + k]);
  }
}

template <int ST, typename U>
__global__ void decode_kernel(const typename Storage<ST>::T* __restrict__ buf, U* __restrict__ user,
                              int64_t N, int64_t p0, Scales s) {
  const int k = static_cast<int>(blockIdx.y);
  const int64_t base = (p0 + k) * N;
  U* u = user + static_cast<int64_t>(k) * N;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    u[i] = static_cast<U>(Storage<ST>::load(buf, base + i, s.v[p0 + k]));
  }
}

template <typename U>
__global__ void maxabs_kernel(const U* __restrict__ user, int64_t N, int64_t p0,
                              unsigned* __restrict__ out_bits) {
  const int k = static_cast<int>(blockIdx.y);
  const U* u = user + static_cast<int64_t>(k) * N;
  float m = 0.0f;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const float v = fabsf(static_cast<float>(u[i]));
    m = v > m ? v : m;  // NaN never wins; an all-NaN plane keeps scale 1
  }
  __shared__ float sh[kThreads];
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w)
      sh[threadIdx.x] = sh[threadIdx.x] > sh[threadIdx.x + w] ? sh[threadIdx.x] : sh[threadIdx.x + w];
    __syncthreads();
  }
  // non-negative float bits order like unsigned integers
  if (threadIdx.x == 0) atomicMax(out_bits + p0 + k, __float_as_uint(sh[0]));
}

template <int ST>
__global__ void reduce_partial_kernel(const typename Storage<ST>::T* __restrict__ buf, int64_t N,
                                      Scales s, double* __restrict__ partials) {
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double a0 = static_cast<double>(Storage<ST>::load(buf, i, s.v[0]));
    const double ux = static_cast<double>(Storage<ST>::load(buf, N + i, s.v[1]));
    const double uy = static_cast<double>(Storage<ST>::load(buf, 2 * N + i, s.v[2]));
    const double uz = static_cast<double>(Storage<ST>::load(buf, 3 * N + i, s.v[3]));
    acc[0] += a0;
    acc[1] += ux;
    acc[2] += uy;
    acc[3] += uz;
    acc[4] += 0.5 * (ux * ux + uy * uy + uz * uz);
  }
  __shared__ double sh[5][kThreads];
#pragma unroll
  for (int j = 0; j < 5; ++j) sh[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w)
#pragma unroll
      for (int j = 0; j < 5; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 5) partials[blockIdx.x * 5 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void reduce_final_kernel(const double* __restrict__ partials, int nparts,
                                    double* __restrict__ out) {
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int p = threadIdx.x; p < nparts; p += kThreads)
#pragma unroll
    for (int j = 0; j < 5; ++j) acc[j] += partials[p * 5 + j];
  __shared__ double sh[5][kThreads];
#pragma unroll
  for (int j = 0; j < 5; ++j) sh[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w)
#pragma unroll
      for (int j = 0; j < 5; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 5) out[threadIdx.x] = sh[threadIdx.x][0];
}

// plane-by-plane copy with the step's memory-instruction forms (dword buffer
// loads, non-temporal dword buffer stores, one element per lane)
__global__ void stream_probe_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                    int64_t n, int nplanes) {
  const uint32_t bytes = static_cast<uint32_t>(n * sizeof(float));
  for (int k = 0; k < nplanes; ++k) {
    const auto rs = plane_rsrc(src + k * n, bytes);
    const auto rd = plane_rsrc(dst + k * n, bytes);
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads) {
      const uint32_t off = static_cast<uint32_t>(i * sizeof(float));
      buf_store_nt<float>(buf_load<float>(rs, off), rd, off);
    }
  }
}

Scales to_scales(const float* p) {
  Scales s;
  for (int k = 0; k < 10; ++k) s.v[k] = p[k];
  return s;
}

template <int ST>
hipError_t encode_st(int user_dtype, const void* user, void* buf, int64_t N, int64_t p0,
                     int64_t np, const float* inv, hipStream_t st) {
  using T = typename Storage<ST>::T;
  const dim3 grid(grid_for(N), static_cast<unsigned>(np));
  if (user_dtype == kF64)
    hipLaunchKernelGGL((encode_kernel<ST, double>), grid, dim3(kThreads), 0, st,
                       static_cast<const double*>(user), static_cast<T*>(buf), N, p0, to_scales(inv));
  else
    hipLaunchKernelGGL((encode_kernel<ST, float>), grid, dim3(kThreads), 0, st,
                       static_cast<const float*>(user), static_cast<T*>(buf), N, p0, to_scales(inv));
  return hipGetLastError();
}

template <int ST>
hipError_t decode_st(int user_dtype, const void* buf, void* user, int64_t N, int64_t p0,
                     int64_t np, const float* scale, hipStream_t st) {
  using T = typename Storage<ST>::T;
  const dim3 grid(grid_for(N), static_cast<unsigned>(np));
  if (user_dtype == kF64)
    hipLaunchKernelGGL((decode_kernel<ST, double>), grid, dim3(kThreads), 0, st,
                       static_cast<const T*>(buf), static_cast<double*>(user), N, p0,
                       to_scales(scale));
  else
    hipLaunchKernelGGL((decode_kernel<ST, float>), grid, dim3(kThreads), 0, st,
                       static_cast<const T*>(buf), static_cast<float*>(user), N, p0,
                       to_scales(scale));
  return hipGetLastError();
}

template <int ST>
hipError_t reduce_st(const void* buf, int64_t N, const float* scale, double* partials, double* out,
                     hipStream_t st) {
  using T = typename Storage<ST>::T;
  hipLaunchKernelGGL((reduce_partial_kernel<ST>), dim3(kReduceBlocks), dim3(kThreads), 0, st,
                     static_cast<const T*>(buf), N, to_scales(scale), partials);
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kThreads), 0, st, partials, kReduceBlocks,
                     out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stream_probe(const void* src, void* dst, int64_t n, int nplanes,
                               hipStream_t s) {
  hipLaunchKernelGGL(stream_probe_kernel, dim3(8192), dim3(kThreads), 0, s,
                     static_cast<const float*>(src), static_cast<float*>(dst), n, nplanes);
  return hipGetLastError();
}

hipError_t launch_encode(int storage, int user_dtype, const void* user, void* buf, int64_t N,
                         int64_t p0, int64_t np, const float* inv_scale, hipStream_t s) {
  switch (storage) {
    case kF64: return encode_st<kF64>(user_dtype, user, buf, N, p0, np, inv_scale, s);
    case kF32: return encode_st<kF32>(user_dtype, user, buf, N, p0, np, inv_scale, s);
    case kF16S: return encode_st<kF16S>(user_dtype, user, buf, N, p0, np, inv_scale, s);
    case kBF16S: return encode_st<kBF16S>(user_dtype, user, buf, N, p0, np, inv_scale, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_decode(int storage, int user_dtype, const void* buf, void* user, int64_t N,
                         int64_t p0, int64_t np, const float* scale, hipStream_t s) {
  switch (storage) {
    case kF64: return decode_st<kF64>(user_dtype, buf, user, N, p0, np, scale, s);
    case kF32: return decode_st<kF32>(user_dtype, buf, user, N, p0, np, scale, s);
    case kF16S: return decode_st<kF16S>(user_dtype, buf, user, N, p0, np, scale, s);
    case kBF16S: return decode_st<kBF16S>(user_dtype, buf, user, N, p0, np, scale, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_maxabs(int user_dtype, const void* user, int64_t N, int64_t p0, int64_t np,
                         unsigned* out_bits, hipStream_t s) {
  const dim3 grid(grid_for(N), static_cast<unsigned>(np));
  if (user_dtype == kF64)
    hipLaunchKernelGGL(maxabs_kernel<double>, grid, dim3(kThreads), 0, s,
                       static_cast<const double*>(user), N, p0, out_bits);
  else
    hipLaunchKernelGGL(maxabs_kernel<float>, grid, dim3(kThreads), 0, s,
                       static_cast<const float*>(user), N, p0, out_bits);
  return hipGetLastError();
}

hipError_t launch_reduce(int storage, const void* buf, int64_t N, const float* scale,
                         double* partials, double* out, hipStream_t s) {
  switch (storage) {
    case kF64: return reduce_st<kF64>(buf, N, scale, partials, out, s);
    case kF32: return reduce_st<kF32>(buf, N, scale, partials, out, s);
    case kF16S: return reduce_st<kF16S>(buf, N, scale, partials, out, s);
    case kBF16S: return reduce_st<kBF16S>(buf, N, scale, partials, out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbf
