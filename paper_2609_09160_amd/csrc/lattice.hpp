// lattice.hpp -- compile-time velocity sets, storage codecs and small
// device helpers for the fused moment-space LBM step (gfx950).
//
// Velocity sets: D3Q19 and D3Q27, both truncated at second order (paper,
// end of section 2).  The direction order is this library's own and is chosen
// for the z-marching kernel: directions that move in the x-y plane
// (c_x != 0 or c_y != 0) come first, so that their index is also their LDS
// staging slot; the three "column" directions (0,0,0), (0,0,+1), (0,0,-1)
// come last and never leave the thread that owns the (x, y) column.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace lbf {

// directions with c_x != 0 or c_y != 0: 16 of D3Q19, then the 8 corners of D3Q27
constexpr int kMove[24][3] = {
    {+1, 0, 0},  {-1, 0, 0},  {0, +1, 0},  {0, -1, 0},     // faces in x, y
    {+1, +1, 0}, {-1, -1, 0}, {+1, -1, 0}, {-1, +1, 0},    // xy edges
    {+1, 0, +1}, {-1, 0, -1}, {+1, 0, -1}, {-1, 0, +1},    // xz edges
    {0, +1, +1}, {0, -1, -1}, {0, +1, -1}, {0, -1, +1},    // yz edges
    {+1, +1, +1}, {-1, -1, -1}, {+1, +1, -1}, {-1, -1, +1},  // corners
    {+1, -1, +1}, {-1, +1, -1}, {-1, +1, +1}, {+1, -1, -1}};

template <int Q>
struct Lat {
  static_assert(Q == 19 || Q == 27, "D3Q19 or D3Q27");
  static constexpr int NP = (Q == 19) ? 16 : 24;  // in-plane-moving directions
  static constexpr int kRest = NP, kUp = NP + 1, kDown = NP + 2;
  static constexpr int c(int i, int a) {
    return i < NP ? kMove[i][a] : (a < 2 ? 0 : (i == kUp ? 1 : (i == kDown ? -1 : 0)));
  }
  static constexpr int cx(int i) { return c(i, 0); }
  static constexpr int cy(int i) { return c(i, 1); }
  static constexpr int cz(int i) { return c(i, 2); }
  static constexpr int c2(int i) { return cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i); }
  // weights by |c|^2 (standard tables; cs^2 = 1/3)
  static constexpr double w(int i) {
    return Q == 19 ? (c2(i) == 0 ? 1.0 / 3.0 : c2(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0)
                   : (c2(i) == 0 ? 8.0 / 27.0
                                 : c2(i) == 1 ? 2.0 / 27.0 : c2(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0);
  }
  // Common denominator of the weights: w_i = k_i / D with k_i a power of two
  // (or 3 for the D3Q19 rest weight), so that multiplying by k_i is exact or
  // unbiased and 1/D is applied once per projected moment.  Rounded weights
  // (e.g. fl(1/18)) would otherwise scale the projected velocity by the same
  // (1 + eps) every step, a drift that accumulates linearly in time.
  static constexpr int D = (Q == 19) ? 9 : 27;
  static constexpr double k(int i) { return w(i) * D; }
  static constexpr int opp(int i) {
    for (int j = 0; j < Q; ++j)
      if (cx(j) == -cx(i) && cy(j) == -cy(i) && cz(j) == -cz(i)) return j;
    return -1;
  }
  // rank of direction i among the directions with c_y == s (wall bookkeeping)
  static constexpr int rank_y(int i, int s) {
    int r = 0;
    for (int j = 0; j < i; ++j) r += (cy(j) == s);
    return r;
  }
  static constexpr int NB = (Q == 19) ? 5 : 9;  // directions with c_y == +1 (or -1)
  // index of the direction with velocity (x, y, z), or -1
  static constexpr int index(int x, int y, int z) {
    for (int j = 0; j < Q; ++j)
      if (cx(j) == x && cy(j) == y && cz(j) == z) return j;
    return -1;
  }
};

// compile-time loop: f(std::integral_constant<int, i>) for i = 0..N-1
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// x / d for a compile-time d: FP32 uses a hi + lo split of 1/d so the result
// is the nearly correctly rounded quotient (no systematic bias); FP64 uses
// the rounded reciprocal (bias ~1e-16 per use).
template <int d, typename C>
__device__ __forceinline__ C div_by(C x) {
  if constexpr (std::is_same_v<C, float>) {
    constexpr double r = 1.0 / d;
    constexpr float hi = static_cast<float>(r);
    constexpr float lo = static_cast<float>(r - static_cast<double>(hi));
    return __builtin_fmaf(x, hi, x * lo);
  } else {
    return x * (1.0 / d);
  }
}

// storage codecs: element type in HBM (T) and compute type (C)
enum { kF64 = 0, kF32 = 1, kF16S = 2, kBF16S = 3, kF16SU = 4 };

// lattice code of the D3Q27 set with the complete Hermite basis (the public
// LBF_D3Q27H); the two truncated sets go by their velocity counts, 19 and 27
constexpr int kD3Q27H = 270;

// Plane accesses go through buffer resources: one scalar descriptor per
// x-y plane (base, byte size) plus a 32-bit per-lane byte offset.  Each access
// is a single instruction with no per-lane address arithmetic, and the
// hardware range check against the plane size turns any out-of-range offset
// into a zero load / dropped store instead of a fault.
constexpr int kBufWord3 = 0x00020000;  // gfx9 family: 32-bit data format, raw access
// Cache policies of the plane accesses: non-temporal stores (2) and default
// loads (0).  Measured on MI355X at 512^3 FP32: plain stores 3.5% slower,
// non-temporal loads 34% slower (the halo re-reads then miss the caches).
constexpr int kNonTemporal = 2;
constexpr int kLoadCpol = 0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0),
                                           static_cast<int>(bytes), kBufWord3);
}

template <typename V>
__device__ __forceinline__ V buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(V) == 2) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, kLoadCpol));
  } else if constexpr (sizeof(V) == 4) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kLoadCpol));
  } else {
    static_assert(sizeof(V) == 8, "2, 4 or 8 bytes");
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kLoadCpol));
  }
}

// one value with the default cache policy (data read again soon)
template <typename V>
__device__ __forceinline__ void buf_store(V v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(V) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
  } else {
    static_assert(sizeof(V) == 8, "4 or 8 bytes");
    using U2 = unsigned int __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, off, 0, 0);
  }
}

template <typename V>
__device__ __forceinline__ void buf_store_nt(V v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(V) == 2) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, off, 0,
                                          kNonTemporal);
  } else if constexpr (sizeof(V) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0,
                                          kNonTemporal);
  } else {
    static_assert(sizeof(V) == 8, "2, 4 or 8 bytes");
    using U2 = unsigned int __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, off, 0, kNonTemporal);
  }
}

// S consecutive values (S = 1, 2, or 3 for 4-byte elements) at byte offset
// off, one load instruction.
// The builtin's result is bit-cast as a whole to a vector of the element type
// before its elements are taken: taking elements of the builtin's own
// integer-vector result directly was compiled (ROCm 7.2) into a load of the
// first dword only, with that dword reused for every element.
template <typename V, int S>
__device__ __forceinline__ void buf_load_n(__amdgpu_buffer_rsrc_t r, uint32_t off, V (&out)[S]) {
  if constexpr (S == 1) {
    out[0] = buf_load<V>(r, off);
  } else if constexpr (S == 3) {
    static_assert(sizeof(V) == 4, "three values per lane: 4-byte elements");
    using V3 = V __attribute__((ext_vector_type(3)));
    const V3 w = __builtin_bit_cast(V3, __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, kLoadCpol));
    out[0] = w.x;
    out[1] = w.y;
    out[2] = w.z;
  } else {
    static_assert(S == 2, "1, 2 or 3 values per lane");
    using V2 = V __attribute__((ext_vector_type(2)));
    V2 w;
    if constexpr (sizeof(V) == 2) {
      w = __builtin_bit_cast(V2, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kLoadCpol));
    } else if constexpr (sizeof(V) == 4) {
      w = __builtin_bit_cast(V2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kLoadCpol));
    } else {
      static_assert(sizeof(V) == 8, "2, 4 or 8 bytes");
      w = __builtin_bit_cast(V2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kLoadCpol));
    }
    out[0] = w.x;
    out[1] = w.y;
  }
}

// S consecutive values stored with one non-temporal store instruction
template <typename V, int S>
__device__ __forceinline__ void buf_store_nt_n(const V (&v)[S], __amdgpu_buffer_rsrc_t r,
                                               uint32_t off) {
  if constexpr (S == 1) {
    buf_store_nt<V>(v[0], r, off);
  } else if constexpr (S == 3) {
    static_assert(sizeof(V) == 4, "three values per lane: 4-byte elements");
    using U3 = unsigned int __attribute__((ext_vector_type(3)));
    const U3 w = {__builtin_bit_cast(unsigned, v[0]), __builtin_bit_cast(unsigned, v[1]),
                  __builtin_bit_cast(unsigned, v[2])};
    __builtin_amdgcn_raw_buffer_store_b96(w, r, off, 0, kNonTemporal);
  } else {
    static_assert(S == 2, "1, 2 or 3 values per lane");
    using V2 = V __attribute__((ext_vector_type(2)));
    const V2 w = {v[0], v[1]};
    if constexpr (sizeof(V) == 2) {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, w), r, off, 0,
                                            kNonTemporal);
    } else if constexpr (sizeof(V) == 4) {
      using U2 = unsigned int __attribute__((ext_vector_type(2)));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, w), r, off, 0, kNonTemporal);
    } else {
      static_assert(sizeof(V) == 8, "2, 4 or 8 bytes");
      using U4 = unsigned int __attribute__((ext_vector_type(4)));
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, w), r, off, 0, kNonTemporal);
    }
  }
}

template <int ST>
struct Storage;
// kNeq: the second-order planes hold the deviation a2 - u u (the
// non-equilibrium stress, small) instead of the total a2 (about u u plus a much
// smaller deviation), so 16-bit rounding does not wipe out the viscous stress.
// The u used is the stored (rounded) velocity, so decoding is exact up to the
// rounding of the deviation itself.
template <>
struct Storage<kF64> {
  using T = double;
  using C = double;
  static constexpr bool kNeq = false;
  static constexpr int kPlanes = 10;
  static constexpr bool kSplitU = false;
  static constexpr bool kGrouped = false;
  static __device__ __forceinline__ C load(const T* p, int64_t i, float) { return p[i]; }
  static __device__ __forceinline__ C decode(T q, float) { return q; }
  static __device__ __forceinline__ T encode(C v, float) { return v; }
  static __device__ __forceinline__ void store(T* p, int64_t i, C v, float) {
    __builtin_nontemporal_store(v, p + i);
  }
};
template <>
struct Storage<kF32> {
  using T = float;
  using C = float;
  static constexpr bool kNeq = false;
  static constexpr int kPlanes = 10;
  static constexpr bool kSplitU = false;
  static constexpr bool kGrouped = false;
  static __device__ __forceinline__ C load(const T* p, int64_t i, float) { return p[i]; }
  static __device__ __forceinline__ C decode(T q, float) { return q; }
  static __device__ __forceinline__ T encode(C v, float) { return v; }
  static __device__ __forceinline__ void store(T* p, int64_t i, C v, float) {
    __builtin_nontemporal_store(v, p + i);
  }
};

// IEEE binary16, value = s * q; conversion rounds to nearest even
__device__ __forceinline__ uint16_t f32_to_f16_bits(float v) {
  return __builtin_bit_cast(uint16_t, static_cast<_Float16>(v));
}
__device__ __forceinline__ float f16_bits_to_f32(uint16_t q) {
  return static_cast<float>(__builtin_bit_cast(_Float16, q));
}
// bfloat16 (upper half of binary32), round to nearest even; NaN stays NaN.
// gfx950 converts in hardware (one instruction); checked bit for bit against
// the integer rounding (add 0x7fff plus the kept part's lowest bit, keep the
// upper half) on 2^24 values, including every exact tie and the special
// values.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float v) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v));
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t q) {
  return __uint_as_float(static_cast<uint32_t>(q) << 16);
}

// 32-bit integer hash "lowbias32" (C. Wellons, "Prospecting for hash
// functions", 2018): xor-shift / multiply rounds with his published
// constants; a counter-based source of uniform bits for stochastic rounding.
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// Stochastic rounding of binary32 x to a format that keeps its top 32 - DROP
// bits: r (8 uniform bits) is added at the top of the dropped bits and the
// result truncated toward zero, so x rounds away from zero with probability
// (dropped part) / 2^DROP, up to 2^-8 of a unit in the last kept place: an
// unbiased rounding, which lets increments smaller than half a unit in the
// last place accumulate instead of being rounded away at every step.
template <int DROP>
__device__ __forceinline__ float round_stochastic(float x, uint32_t r) {
  uint32_t b = __float_as_uint(x);
  b += r << (DROP - 8);
  b &= ~((1u << DROP) - 1u);
  return __uint_as_float(b);
}

template <>
struct Storage<kF16S> {
  using T = uint16_t;
  using C = float;
  static constexpr bool kNeq = true;
  static constexpr int kPlanes = 10;
  static constexpr bool kSplitU = false;
  static constexpr bool kGrouped = true;
  static __device__ __forceinline__ C load(const T* p, int64_t i, float s) {
    return f16_bits_to_f32(p[i]) * s;
  }
  // q s as one mixed-precision multiply-add (the binary16 operand converted on
  // the fly; exact, s being a power of two; +0 for a zero product)
  static __device__ __forceinline__ C decode(T q, float s) {
    return __builtin_fmaf(f16_bits_to_f32(q), s, 0.0f);
  }
  static __device__ __forceinline__ T encode(C v, float inv_s) { return f32_to_f16_bits(v * inv_s); }
  // a value already in storage units, rounded to nearest or stochastically
  // (10 stored significand bits: 13 of binary32's are dropped; the truncated
  // value converts exactly in the normal range, below it the conversion
  // rounds to nearest)
  static __device__ __forceinline__ T encode_unit(C v) { return f32_to_f16_bits(v); }
  static __device__ __forceinline__ T encode_unit_sr(C v, uint32_t r) {
    return f32_to_f16_bits(round_stochastic<13>(v, r));
  }
  static __device__ __forceinline__ void store(T* p, int64_t i, C v, float inv_s) {
    __builtin_nontemporal_store(f32_to_f16_bits(v * inv_s), p + i);
  }
};
template <>
struct Storage<kBF16S> {
  using T = uint16_t;
  using C = float;
  static constexpr bool kNeq = true;
  static constexpr int kPlanes = 10;
  static constexpr bool kSplitU = false;
  static constexpr bool kGrouped = true;
  static __device__ __forceinline__ C load(const T* p, int64_t i, float s) {
    return bf16_bits_to_f32(p[i]) * s;
  }
  static __device__ __forceinline__ C decode(T q, float s) { return bf16_bits_to_f32(q) * s; }
  static __device__ __forceinline__ T encode(C v, float inv_s) { return f32_to_bf16_bits(v * inv_s); }
  // a value already in storage units, rounded to nearest or stochastically
  // (the stochastic form keeps the upper half of binary32)
  static __device__ __forceinline__ T encode_unit(C v) { return f32_to_bf16_bits(v); }
  static __device__ __forceinline__ T encode_unit_sr(C v, uint32_t r) {
    return static_cast<T>(__float_as_uint(round_stochastic<16>(v, r)) >> 16);
  }
  static __device__ __forceinline__ void store(T* p, int64_t i, C v, float inv_s) {
    __builtin_nontemporal_store(f32_to_bf16_bits(v * inv_s), p + i);
  }
};

// FP16-scaled storage with the velocity split over two binary16 words: p*
// and the six a2 - u u planes as in Storage<kF16S>, and each velocity
// component u = s (hi + 2^-11 lo), hi its rounding to binary16 and lo the
// rounding of the remainder, in three more planes (10..12).  The pair keeps
// 22 significant bits of u, where the error of 16-bit storage comes from
// almost entirely, for 13 x 2 bytes per site instead of 10 x 2.
constexpr float kSplitLo = 1.0f / 2048.0f;  // scale of lo relative to hi
template <>
struct Storage<kF16SU> : Storage<kF16S> {
  static constexpr int kPlanes = 13;
  static constexpr bool kSplitU = true;
  // value units (v / s) -> hi, lo; rounded to nearest even, the remainder
  // un - hi is exact in binary32
  static __device__ __forceinline__ void split_unit(C un, T& hi, T& lo) {
    hi = f32_to_f16_bits(un);
    lo = f32_to_f16_bits((un - f16_bits_to_f32(hi)) * 2048.0f);
  }
  // s (hi + 2^-11 lo), two exact products and one exact sum in the normal range
  static __device__ __forceinline__ C join(T hi, T lo, float s) {
    return decode(hi, s) + decode(lo, s * kSplitLo);
  }
};

// Element index of moment plane k at site i, in a state of N sites.  With
// kGrouped (16-bit storage) the planes go in groups of four, 4j .. 4j + 3,
// interleaved site by site in the space of the four planes: one 64-bit word
// holds the four values of a site, plane 4j in its lowest 16 bits.  Two
// planes left over form a pair the same way (one 32-bit word per site); a
// last odd plane stays on its own.  A wave then reads a few wide streams
// instead of many narrow ones.  Measured at 512^3 on MI355X: copies of ten
// 16-bit planes in the step's marching order moved 4.5-4.7 TB/s with the
// planes apart, 5.1-5.2 in pairs and 5.1-5.6 in groups of four and a pair;
// the D3Q19 FP16 step ran at 105-112, 114-116 and 120-124 GLUPS.
template <typename S>
__host__ __device__ constexpr int64_t plane_elem(int k, int64_t i, int64_t N) {
  if constexpr (S::kGrouped) {
    constexpr int q4 = S::kPlanes & ~3;       // planes in groups of four
    constexpr int q2 = q4 + (S::kPlanes & 2);  // then a pair, if two are left
    if (k < q4) return static_cast<int64_t>(k & ~3) * N + 4 * i + (k & 3);
    if (k < q2) return static_cast<int64_t>(q4) * N + 2 * i + (k & 1);
  }
  return static_cast<int64_t>(k) * N + i;
}

// index pairs (a, b) of the second-order planes 4..9: xx, yy, zz, xy, xz, yz
__host__ __device__ constexpr int a2_a(int k) { return k <= 6 ? k - 4 : (k == 9 ? 1 : 0); }
__host__ __device__ constexpr int a2_b(int k) { return k <= 6 ? k - 4 : (k == 7 ? 1 : 2); }

// periodic index for v in [-n, 2n)
__device__ __forceinline__ int wrap(int v, int n) {
  v = v < 0 ? v + n : v;
  return v >= n ? v - n : v;
}
// periodic index for any v
__device__ __forceinline__ int pmod(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

}  // namespace lbf
