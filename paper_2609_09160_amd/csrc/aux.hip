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
hipError_t launch_step_f16su(int, int, bool, bool, const StepArgs&, hipStream_t);

hipError_t launch_step_h_f64(int, bool, bool, const StepArgs&, hipStream_t);
hipError_t launch_step_h_f32(int, bool, bool, const StepArgs&, hipStream_t);
hipError_t launch_step_h_f16s(int, bool, bool, const StepArgs&, hipStream_t);
hipError_t launch_step_h_bf16s(int, bool, bool, const StepArgs&, hipStream_t);
hipError_t launch_step_h_f16su(int, bool, bool, const StepArgs&, hipStream_t);

hipError_t launch_step(int Q, int storage, int tile_rows, bool walls_y, const StepArgs& a,
                       hipStream_t stream) {
  const bool ff = a.Ffield != nullptr;
  if (Q == kD3Q27H) {
    switch (storage) {
      case kF64: return launch_step_h_f64(tile_rows, walls_y, ff, a, stream);
      case kF32: return launch_step_h_f32(tile_rows, walls_y, ff, a, stream);
      case kF16S: return launch_step_h_f16s(tile_rows, walls_y, ff, a, stream);
      case kBF16S: return launch_step_h_bf16s(tile_rows, walls_y, ff, a, stream);
      case kF16SU: return launch_step_h_f16su(tile_rows, walls_y, ff, a, stream);
      default: return hipErrorInvalidValue;
    }
  }
  switch (storage) {
    case kF64: return launch_step_f64(Q, tile_rows, walls_y, ff, a, stream);
    case kF32: return launch_step_f32(Q, tile_rows, walls_y, ff, a, stream);
    case kF16S: return launch_step_f16s(Q, tile_rows, walls_y, ff, a, stream);
    case kBF16S: return launch_step_bf16s(Q, tile_rows, walls_y, ff, a, stream);
    case kF16SU: return launch_step_f16su(Q, tile_rows, walls_y, ff, a, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint_f64(int, int, bool, bool, const StepArgs&, hipStream_t);
hipError_t launch_adjoint_f32(int, int, bool, bool, const StepArgs&, hipStream_t);

hipError_t launch_adjoint(int Q, int storage, int tile_rows, bool walls_y, const StepArgs& a,
                          hipStream_t stream) {
  const bool ff = a.Ffield != nullptr;
  switch (storage) {
    case kF64: return launch_adjoint_f64(Q, tile_rows, walls_y, ff, a, stream);
    case kF32: return launch_adjoint_f32(Q, tile_rows, walls_y, ff, a, stream);
    default: return hipErrorInvalidValue;
  }
}

namespace {

constexpr int kThreads = 256;

__global__ void zero_kernel(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    p[i] = 0u;
}

// 10 scales passed by value
struct Scales {
  float v[10];
};

int grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return static_cast<int>(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

// velocity component c of site i as it reads back from storage: the user's
// value rounded to the storage format (deviation planes are relative to it)
template <int ST, typename U>
__device__ __forceinline__ float stored_u(const U* u, int64_t i, float inv, float s) {
  using S = Storage<ST>;
  if constexpr (S::kSplitU) {
    typename S::T hi, lo;
    S::split_unit(static_cast<float>(u[i]) * inv, hi, lo);
    return S::join(hi, lo, s);
  } else {
    return static_cast<float>(S::decode(S::encode(static_cast<typename S::C>(u[i]), inv), s));
  }
}

// user plane k (F64/F32) -> storage plane k; for deviation storage the planes
// k >= 4 hold a2 - u u with u rounded as stored (u0..u2: the user's u planes)
template <int ST, typename U>
__global__ void encode_kernel(const U* __restrict__ user, const U* __restrict__ u0,
                              const U* __restrict__ u1, const U* __restrict__ u2,
                              typename Storage<ST>::T* __restrict__ buf, int64_t N, int k,
                              Scales inv, Scales fwd) {
  using S = Storage<ST>;
  using C = typename S::C;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    C v = static_cast<C>(user[i]);
    if constexpr (S::kSplitU) {
      if (k >= 1 && k <= 3) {  // hi in plane k, lo in plane 9 + k
        typename S::T hi, lo;
        S::split_unit(v * inv.v[k], hi, lo);
        __builtin_nontemporal_store(hi, buf + plane_elem<S>(k, i, N));
        __builtin_nontemporal_store(lo, buf + plane_elem<S>(9 + k, i, N));
        continue;
      }
    }
    if constexpr (S::kNeq) {
      if (k >= 4) {
        const U* ua = a2_a(k) == 0 ? u0 : (a2_a(k) == 1 ? u1 : u2);
        const U* ub = a2_b(k) == 0 ? u0 : (a2_b(k) == 1 ? u1 : u2);
        v -= static_cast<C>(stored_u<ST>(ua, i, inv.v[1 + a2_a(k)], fwd.v[1 + a2_a(k)]) *
                            stored_u<ST>(ub, i, inv.v[1 + a2_b(k)], fwd.v[1 + a2_b(k)]));
      }
    }
    S::store(buf, plane_elem<S>(k, i, N), v, inv.v[k]);
  }
}

// storage plane k -> user plane k (total a2 for deviation storage)
template <int ST, typename U>
__global__ void decode_kernel(const typename Storage<ST>::T* __restrict__ buf, U* __restrict__ user,
                              int64_t N, int k, Scales s) {
  using S = Storage<ST>;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    // velocity component c as stored (hi + lo for the split form)
    auto vel = [&](int c) {
      if constexpr (S::kSplitU)
        return S::join(buf[plane_elem<S>(1 + c, i, N)], buf[plane_elem<S>(10 + c, i, N)],
                       s.v[1 + c]);
      else
        return S::load(buf, plane_elem<S>(1 + c, i, N), s.v[1 + c]);
    };
    auto v = (k >= 1 && k <= 3) ? vel(k - 1) : S::load(buf, plane_elem<S>(k, i, N), s.v[k]);
    if constexpr (S::kNeq) {
      if (k >= 4) v += vel(a2_a(k)) * vel(a2_b(k));
    }
    user[i] = static_cast<U>(v);
  }
}

// max |value stored in plane k| over a user plane (deviation for k >= 4 when
// `dev`), into out_bits[k] (float bits; must start at zero)
template <int ST, typename U>
__global__ void maxabs_kernel(const U* __restrict__ user, const U* __restrict__ u0,
                              const U* __restrict__ u1, const U* __restrict__ u2, int64_t N, int k,
                              int dev, Scales inv, Scales fwd, unsigned* __restrict__ out_bits) {
  float m = 0.0f;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    float v = static_cast<float>(user[i]);
    if (dev && k >= 4) {
      const U* ua = a2_a(k) == 0 ? u0 : (a2_a(k) == 1 ? u1 : u2);
      const U* ub = a2_b(k) == 0 ? u0 : (a2_b(k) == 1 ? u1 : u2);
      v = static_cast<float>(static_cast<double>(user[i]) -
                             static_cast<double>(stored_u<ST>(ua, i, inv.v[1 + a2_a(k)], fwd.v[1 + a2_a(k)])) *
                             stored_u<ST>(ub, i, inv.v[1 + a2_b(k)], fwd.v[1 + a2_b(k)]));
    }
    v = fabsf(v);
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
  if (threadIdx.x == 0) atomicMax(out_bits + k, __float_as_uint(sh[0]));
}

template <int ST>
__global__ void reduce_partial_kernel(const typename Storage<ST>::T* __restrict__ buf, int64_t N,
                                      Scales s, double* __restrict__ partials) {
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    using S = Storage<ST>;
    double u3[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if constexpr (S::kSplitU)
        u3[c] = static_cast<double>(S::join(buf[plane_elem<S>(1 + c, i, N)],
                                            buf[plane_elem<S>(10 + c, i, N)], s.v[1 + c]));
      else
        u3[c] = static_cast<double>(S::load(buf, plane_elem<S>(1 + c, i, N), s.v[1 + c]));
    }
    const double a0 = static_cast<double>(S::load(buf, plane_elem<S>(0, i, N), s.v[0]));
    const double ux = u3[0], uy = u3[1], uz = u3[2];
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

// One 16-byte access per lane and one per thread (a one-shot grid of
// 256-thread blocks), non-temporal stores: the fastest form of a copy
// measured on MI355X (6.2-6.3 TB/s; grid-stride forms reach 5.3), i.e. the
// ceiling of a single stream that reads and writes equal volumes.
typedef float F4 __attribute__((ext_vector_type(4)));
typedef float F2 __attribute__((ext_vector_type(2)));
__global__ void copy_wide_kernel(const F4* __restrict__ src, F4* __restrict__ dst, int64_t n4) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i < n4) __builtin_nontemporal_store(src[i], &dst[i]);
}

// The step's access pattern without halos or arithmetic: nplanes planes of n
// floats in structure of arrays, each thread reading 8 bytes (two consecutive
// floats) from every plane and then writing them, non-temporal stores.
template <int NPL>
__global__ void __launch_bounds__(kThreads) copy_planes_kernel(const float* __restrict__ src,
                                                               float* __restrict__ dst, int64_t n) {
  const int64_t i = (blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x) * 2;
  if (i >= n) return;
  F2 v[NPL];
#pragma unroll
  for (int k = 0; k < NPL; ++k) v[k] = *reinterpret_cast<const F2*>(src + k * n + i);
#pragma unroll
  for (int k = 0; k < NPL; ++k)
    __builtin_nontemporal_store(v[k], reinterpret_cast<F2*>(dst + k * n + i));
}

// The step's marching order without halos or arithmetic, for the layouts of
// a state: a workgroup of 8 waves owns a 128 x 8 column tile (two sites per
// lane, one row per wave) and a chunk of z-planes, and reads plane z + 1
// while it writes plane z (non-temporal stores).  Layout L: 0 = ten FP32
// planes apart, 1 = ten 16-bit planes apart, 2 = 16-bit planes in pairs (a
// 32-bit word per site), 3 = 16-bit planes in two groups of four and a pair
// (the library's 16-bit layout: a 64-bit, a 64-bit and a 32-bit word per
// site).  zm_bytes(L, g) is the bytes per site of stream g.
constexpr int kZmRows = 8;
constexpr int zm_streams(int L) { return L <= 1 ? 10 : (L == 2 ? 5 : 3); }
constexpr int zm_bytes(int L, int g) { return L == 0 ? 4 : (L == 1 ? 2 : (L == 2 ? 4 : (g < 2 ? 8 : 4))); }
constexpr int zm_prefix(int L, int g) { return g == 0 ? 0 : zm_prefix(L, g - 1) + zm_bytes(L, g - 1); }
template <int W> struct ZmVec;
template <> struct ZmVec<4> { using V = unsigned; };
template <> struct ZmVec<8> { using V = unsigned __attribute__((ext_vector_type(2))); };
template <> struct ZmVec<16> { using V = unsigned __attribute__((ext_vector_type(4))); };

template <int L>
__global__ void __launch_bounds__(64 * kZmRows) zmarch_copy_kernel(const char* __restrict__ src,
                                                                   char* __restrict__ dst, int nx,
                                                                   int ny, int nz, int zchunk) {
  constexpr int G = zm_streams(L);
  constexpr int WORDS = 2 * zm_prefix(L, G) / 4;  // 32-bit words a lane moves per plane
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tiles_x = nx / 128, tiles_y = ny / kZmRows;
  int b = static_cast<int>(blockIdx.x);
  const int tx = b % tiles_x;
  b /= tiles_x;
  const int ty = b % tiles_y;
  const int zc = b / tiles_y;
  const int64_t N = static_cast<int64_t>(nx) * ny * nz, P = static_cast<int64_t>(nx) * ny;
  const int64_t row = static_cast<int64_t>(ty * kZmRows + w) * nx + tx * 128 + 2 * lane;
  const int z0 = zc * zchunk, z1 = min(z0 + zchunk, nz);
  unsigned cur[WORDS], nxt[WORDS];
  auto load = [&](int z, unsigned (&r)[WORDS]) __attribute__((always_inline)) {
    const int64_t site = z * P + row;
    static_for<G>([&](auto I) {
      constexpr int g = decltype(I)::value, B = zm_bytes(L, g), O = 2 * zm_prefix(L, g) / 4;
      using V = typename ZmVec<2 * B>::V;
      const V v = *reinterpret_cast<const V*>(src + zm_prefix(L, g) * N + site * B);
      __builtin_memcpy(&r[O], &v, 2 * B);
    });
  };
  load(z0, cur);
  for (int z = z0; z < z1; ++z) {
    load(min(z + 1, z1 - 1), nxt);
    const int64_t site = z * P + row;
    static_for<G>([&](auto I) {
      constexpr int g = decltype(I)::value, B = zm_bytes(L, g), O = 2 * zm_prefix(L, g) / 4;
      using V = typename ZmVec<2 * B>::V;
      V v;
      __builtin_memcpy(&v, &cur[O], 2 * B);
      __builtin_nontemporal_store(v, reinterpret_cast<V*>(dst + zm_prefix(L, g) * N + site * B));
    });
#pragma unroll
    for (int k = 0; k < WORDS; ++k) cur[k] = nxt[k];
  }
}

Scales to_scales(const float* p) {
  Scales s;
  for (int k = 0; k < 10; ++k) s.v[k] = p[k];
  return s;
}

template <int ST>
hipError_t encode_st(int user_dtype, const void* plane, const void* const u[3], void* buf,
                     int64_t N, int k, const float* inv, const float* fwd, hipStream_t st) {
  using T = typename Storage<ST>::T;
  const dim3 grid(grid_for(N));
  if (user_dtype == kF64)
    hipLaunchKernelGGL((encode_kernel<ST, double>), grid, dim3(kThreads), 0, st,
                       static_cast<const double*>(plane), static_cast<const double*>(u[0]),
                       static_cast<const double*>(u[1]), static_cast<const double*>(u[2]),
                       static_cast<T*>(buf), N, k, to_scales(inv), to_scales(fwd));
  else
    hipLaunchKernelGGL((encode_kernel<ST, float>), grid, dim3(kThreads), 0, st,
                       static_cast<const float*>(plane), static_cast<const float*>(u[0]),
                       static_cast<const float*>(u[1]), static_cast<const float*>(u[2]),
                       static_cast<T*>(buf), N, k, to_scales(inv), to_scales(fwd));
  return hipGetLastError();
}

template <int ST>
hipError_t decode_st(int user_dtype, const void* buf, void* plane, int64_t N, int k,
                     const float* scale, hipStream_t st) {
  using T = typename Storage<ST>::T;
  const dim3 grid(grid_for(N));
  if (user_dtype == kF64)
    hipLaunchKernelGGL((decode_kernel<ST, double>), grid, dim3(kThreads), 0, st,
                       static_cast<const T*>(buf), static_cast<double*>(plane), N, k,
                       to_scales(scale));
  else
    hipLaunchKernelGGL((decode_kernel<ST, float>), grid, dim3(kThreads), 0, st,
                       static_cast<const T*>(buf), static_cast<float*>(plane), N, k,
                       to_scales(scale));
  return hipGetLastError();
}

template <int ST>
hipError_t maxabs_st(int user_dtype, const void* plane, const void* const u[3], int64_t N, int k,
                     const float* inv, const float* fwd, unsigned* out_bits, hipStream_t st) {
  const dim3 grid(grid_for(N));
  // The scale of every plane follows the magnitude of the total value: the
  // deviation a2 - u u of a state at equilibrium is ~0, and a scale sized on it
  // would overflow once the flow builds its non-equilibrium stress; smaller
  // deviations stay in the normal range of the 16-bit format.
  const int dev = 0;
  if (user_dtype == kF64)
    hipLaunchKernelGGL((maxabs_kernel<ST, double>), grid, dim3(kThreads), 0, st,
                       static_cast<const double*>(plane), static_cast<const double*>(u[0]),
                       static_cast<const double*>(u[1]), static_cast<const double*>(u[2]), N, k,
                       dev, to_scales(inv), to_scales(fwd), out_bits);
  else
    hipLaunchKernelGGL((maxabs_kernel<ST, float>), grid, dim3(kThreads), 0, st,
                       static_cast<const float*>(plane), static_cast<const float*>(u[0]),
                       static_cast<const float*>(u[1]), static_cast<const float*>(u[2]), N, k,
                       dev, to_scales(inv), to_scales(fwd), out_bits);
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

hipError_t launch_zero(void* p, int64_t nbytes, hipStream_t stream) {
  if (nbytes % 4 != 0) return hipErrorInvalidValue;
  const int64_t n = nbytes / 4;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(kThreads), 0, stream,
                     static_cast<uint32_t*>(p), n);
  return hipGetLastError();
}

hipError_t launch_stream_probe(const void* src, void* dst, int64_t n, int nplanes,
                               hipStream_t s) {
  hipLaunchKernelGGL(stream_probe_kernel, dim3(8192), dim3(kThreads), 0, s,
                     static_cast<const float*>(src), static_cast<float*>(dst), n, nplanes);
  return hipGetLastError();
}

hipError_t launch_copy_probe(const void* src, void* dst, int64_t n4, hipStream_t s) {
  const int64_t blocks = (n4 + kThreads - 1) / kThreads;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_wide_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, s,
                     static_cast<const F4*>(src), static_cast<F4*>(dst), n4);
  return hipGetLastError();
}

hipError_t launch_zmarch_probe(const void* src, void* dst, int nx, int ny, int nz, int layout,
                               int zchunk, hipStream_t s) {
  if (nx < 128 || nx % 128 || ny < kZmRows || ny % kZmRows || nz < 1 || zchunk < 1 ||
      layout < 0 || layout > 3)
    return hipErrorInvalidValue;
  const int64_t blocks =
      static_cast<int64_t>(nx / 128) * (ny / kZmRows) * ((nz + zchunk - 1) / zchunk);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(blocks)), block(64 * kZmRows);
  const char* a = static_cast<const char*>(src);
  char* b = static_cast<char*>(dst);
  switch (layout) {
    case 0: hipLaunchKernelGGL(zmarch_copy_kernel<0>, grid, block, 0, s, a, b, nx, ny, nz, zchunk); break;
    case 1: hipLaunchKernelGGL(zmarch_copy_kernel<1>, grid, block, 0, s, a, b, nx, ny, nz, zchunk); break;
    case 2: hipLaunchKernelGGL(zmarch_copy_kernel<2>, grid, block, 0, s, a, b, nx, ny, nz, zchunk); break;
    default: hipLaunchKernelGGL(zmarch_copy_kernel<3>, grid, block, 0, s, a, b, nx, ny, nz, zchunk); break;
  }
  return hipGetLastError();
}

hipError_t launch_planes_probe(const void* src, void* dst, int64_t n, int nplanes, hipStream_t s) {
  const int64_t blocks = (n / 2 + kThreads - 1) / kThreads;
  if (blocks > 0x7fffffff || nplanes < 1 || nplanes > 10 || n % 2) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(blocks));
  const float* a = static_cast<const float*>(src);
  float* b = static_cast<float*>(dst);
  auto go = [&](auto NPL) {
    hipLaunchKernelGGL(copy_planes_kernel<decltype(NPL)::value>, grid, dim3(kThreads), 0, s, a, b,
                       n);
  };
  switch (nplanes) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 5: go(std::integral_constant<int, 5>{}); break;
    case 6: go(std::integral_constant<int, 6>{}); break;
    case 7: go(std::integral_constant<int, 7>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 9: go(std::integral_constant<int, 9>{}); break;
    default: go(std::integral_constant<int, 10>{}); break;
  }
  return hipGetLastError();
}

hipError_t launch_encode(int storage, int user_dtype, const void* plane, const void* const u[3],
                         void* buf, int64_t N, int k, const float* inv_scale, const float* scale,
                         hipStream_t s) {
  switch (storage) {
    case kF64: return encode_st<kF64>(user_dtype, plane, u, buf, N, k, inv_scale, scale, s);
    case kF32: return encode_st<kF32>(user_dtype, plane, u, buf, N, k, inv_scale, scale, s);
    case kF16S: return encode_st<kF16S>(user_dtype, plane, u, buf, N, k, inv_scale, scale, s);
    case kBF16S: return encode_st<kBF16S>(user_dtype, plane, u, buf, N, k, inv_scale, scale, s);
    case kF16SU: return encode_st<kF16SU>(user_dtype, plane, u, buf, N, k, inv_scale, scale, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_decode(int storage, int user_dtype, const void* buf, void* plane, int64_t N,
                         int k, const float* scale, hipStream_t s) {
  switch (storage) {
    case kF64: return decode_st<kF64>(user_dtype, buf, plane, N, k, scale, s);
    case kF32: return decode_st<kF32>(user_dtype, buf, plane, N, k, scale, s);
    case kF16S: return decode_st<kF16S>(user_dtype, buf, plane, N, k, scale, s);
    case kBF16S: return decode_st<kBF16S>(user_dtype, buf, plane, N, k, scale, s);
    case kF16SU: return decode_st<kF16SU>(user_dtype, buf, plane, N, k, scale, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_maxabs(int storage, int user_dtype, const void* plane, const void* const u[3],
                         int64_t N, int k, const float* inv_scale, const float* scale,
                         unsigned* out_bits, hipStream_t s) {
  switch (storage) {
    case kF64: return maxabs_st<kF64>(user_dtype, plane, u, N, k, inv_scale, scale, out_bits, s);
    case kF32: return maxabs_st<kF32>(user_dtype, plane, u, N, k, inv_scale, scale, out_bits, s);
    case kF16S: return maxabs_st<kF16S>(user_dtype, plane, u, N, k, inv_scale, scale, out_bits, s);
    case kBF16S:
      return maxabs_st<kBF16S>(user_dtype, plane, u, N, k, inv_scale, scale, out_bits, s);
    case kF16SU:
      return maxabs_st<kF16SU>(user_dtype, plane, u, N, k, inv_scale, scale, out_bits, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce(int storage, const void* buf, int64_t N, const float* scale,
                         double* partials, double* out, hipStream_t s) {
  switch (storage) {
    case kF64: return reduce_st<kF64>(buf, N, scale, partials, out, s);
    case kF32: return reduce_st<kF32>(buf, N, scale, partials, out, s);
    case kF16S: return reduce_st<kF16S>(buf, N, scale, partials, out, s);
    case kBF16S: return reduce_st<kBF16S>(buf, N, scale, partials, out, s);
    case kF16SU: return reduce_st<kF16SU>(buf, N, scale, partials, out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbf
