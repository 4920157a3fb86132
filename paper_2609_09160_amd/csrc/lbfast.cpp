// lbfast.cpp -- host runtime behind the C ABI of include/lbfast.h: argument
// validation, buffer ownership, flip/flop bookkeeping (the paper's two
// ten-field arrays, section 3), launch shape, conversions and reductions.
#include "lbfast.h"
#include "lbfast_measure.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "internal.hpp"

namespace lbf {
// measurement utilities, aux.hip
hipError_t launch_copy_probe(const void* src, void* dst, int64_t n4, hipStream_t s);
hipError_t launch_planes_probe(const void* src, void* dst, int64_t n, int nplanes, hipStream_t s);
hipError_t launch_zmarch_probe(const void* src, void* dst, int nx, int ny, int nz, int layout,
                               int zchunk, hipStream_t s);
}  // namespace lbf

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

// error reporting for entry points defined in other translation units
namespace lbf {
void clear_error() { g_err.clear(); }
int set_error(int code, const char* msg) {
  g_err = msg;
  return code;
}
}  // namespace lbf

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fail(LBF_E_DEVICE, "%s: %s (%d)", what, hipGetErrorString(e), static_cast<int>(e));
}

size_t elem_bytes(int storage) {
  switch (storage) {
    case LBF_F64: return 8;
    case LBF_F32: return 4;
    case LBF_F16S:
    case LBF_BF16S:
    case LBF_F16SU: return 2;
    default: return 0;
  }
}

// planes of one state buffer: the ten moments, plus the three low velocity
// words of the split form
size_t state_planes(int storage) { return storage == LBF_F16SU ? 13 : 10; }

bool is_16bit(int storage) {
  return storage == LBF_F16S || storage == LBF_BF16S || storage == LBF_F16SU;
}

bool is_pow2_float(float s) {
  if (!(s > 0.0f) || !std::isfinite(s)) return false;
  int e;
  return std::frexp(s, &e) == 0.5f;
}

int validate(const lbfast_params* p) {
  if (!p) return fail(LBF_E_ARG, "params is NULL");
  if (p->struct_size != sizeof(lbfast_params))
    return fail(LBF_E_ARG, "params.struct_size = %u, expected %zu", p->struct_size,
                sizeof(lbfast_params));
  if (p->lattice != LBF_D3Q19 && p->lattice != LBF_D3Q27 && p->lattice != LBF_D3Q27H)
    return fail(LBF_E_ARG, "lattice must be LBF_D3Q19, LBF_D3Q27 or LBF_D3Q27H (got %d)",
                p->lattice);
  if (elem_bytes(p->storage) == 0) return fail(LBF_E_ARG, "unknown storage %d", p->storage);
  const int64_t n[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1) return fail(LBF_E_ARG, "grid extent %d is %lld (must be >= 1)", a,
                              static_cast<long long>(n[a]));
    if (n[a] > (1 << 30)) return fail(LBF_E_ARG, "grid extent %d too large", a);
    if (p->bc[a] != LBF_PERIODIC && p->bc[a] != LBF_WALLS)
      return fail(LBF_E_ARG, "bc[%d] = %d is not LBF_PERIODIC/LBF_WALLS", a, p->bc[a]);
  }
  if (p->bc[0] == LBF_WALLS || p->bc[2] == LBF_WALLS)
    return fail(LBF_E_UNSUPPORTED, "walls are supported on the y axis only");
  if (p->bc[1] == LBF_WALLS && p->ny < 2)
    return fail(LBF_E_ARG, "a walled axis needs at least 2 sites (ny = %lld)",
                static_cast<long long>(p->ny));
  const double N = static_cast<double>(p->nx) * static_cast<double>(p->ny) * static_cast<double>(p->nz);
  if (N > 4.0e9) return fail(LBF_E_ARG, "grid has %.3g sites (limit 4e9)", N);
  // in-plane byte offsets are 32-bit in the kernels (8-byte elements worst case)
  if (static_cast<double>(p->nx) * static_cast<double>(p->ny) * 8.0 >= 4294967296.0)
    return fail(LBF_E_ARG, "nx*ny too large (an x-y plane of 8-byte values must fit in 4 GiB)");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau))
    return fail(LBF_E_ARG, "tau must be a finite value > 1/2 (got %g)", p->tau);
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->force[a])) return fail(LBF_E_ARG, "force[%d] is not finite", a);
  const bool s16 = is_16bit(p->storage);
  for (int k = 0; k < 10; ++k) {
    if (p->scale[k] == 0.0f) continue;
    if (!s16) return fail(LBF_E_ARG, "scale[] is only meaningful for 16-bit storage");
    if (!is_pow2_float(p->scale[k]))
      return fail(LBF_E_ARG, "scale[%d] = %g is not a positive power of two", k, p->scale[k]);
  }
  for (int k = 0; k < 7; ++k)
    if (p->reserved[k] != 0) return fail(LBF_E_ARG, "reserved[%d] must be zero", k);
  if (p->rounding != LBF_ROUND_AUTO && p->rounding != LBF_ROUND_NEAREST &&
      p->rounding != LBF_ROUND_STOCHASTIC)
    return fail(LBF_E_ARG, "rounding must be LBF_ROUND_AUTO, _NEAREST or _STOCHASTIC");
  if (p->rounding == LBF_ROUND_STOCHASTIC && !s16)
    return fail(LBF_E_ARG, "stochastic rounding applies to 16-bit storage only");
  if (p->storage == LBF_F16SU && p->rounding == LBF_ROUND_STOCHASTIC)
    return fail(LBF_E_ARG, "LBF_F16SU rounds to nearest (its velocity keeps 22 bits)");
  return LBF_OK;
}

}  // namespace

struct lbfast_ctx {
  lbfast_params p;
  int device = 0;
  hipStream_t stream = nullptr;
  void* buf[2] = {nullptr, nullptr};
  bool owned = false;
  int cur = 0;
  const void* Ffield = nullptr;
  float scale[10];
  float inv_scale[10];
  bool scales_fixed = false;
  int tile_rows = 8;
  int z_chunk = 0;
  int lane_sites = 1;
  bool two_phase = false;
  lbfast_phase_params pp;
  void* phi[2] = {nullptr, nullptr};  // phase field, two time levels
  void* Fph[2] = {nullptr, nullptr};  // force of the two time levels (3 planes)
  int pcur = 0;
  double* d_partials = nullptr;  // kReduceBlocks*5 + 5 doubles
  unsigned* d_maxbits = nullptr; // 10
  int64_t N = 0;
  uint64_t steps_done = 0;       // steps since create: seeds the stochastic rounding
  int adj_sites = 0, adj_rows = 0;  // adjoint launch shape (0: automatic)
  int block_order = 0;              // 0 automatic, 1 hardware order, 2 per-XCD ranges
};

namespace {

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// LDS of one step workgroup: staged populations x (rows + 2) x (64 S + 2)
// columns, plus the x-halo column buffer
// LDS of one step workgroup; the two-component step stages phi(t+1) in one
// more slot for its stencils
size_t lds_bytes(int Q, int storage, int tile_rows, int lane_sites, bool stencil = false) {
  const size_t np = ((Q == LBF_D3Q19) ? 16 : 24) + (stencil ? 1 : 0);
  const size_t c = (storage == LBF_F64) ? 8 : 4;
  return c * np * static_cast<size_t>(tile_rows + 2) * static_cast<size_t>(64 * lane_sites + 4);
}
constexpr size_t kLdsLimit = 160 * 1024;

// default launch shape (measured on MI355X at 512^3): two x-sites per lane
// where nx allows it (even, at least one 128-wide tile), 8-row tiles (FP64:
// 4 rows with two sites per lane, 6 with one) or the tallest that fits the
// LDS; z-chunks only when the column tiles alone give too few workgroups.
// D3Q27h in FP64 keeps one site per lane: two spill registers there.
void default_launch(lbfast_ctx* h) {
  // two sites per lane unless 128-wide tiles would leave more of the last
  // tile empty than 64-wide ones; else three (FP32, second-order sets) where
  // 192-wide tiles leave no more empty than 64-wide ones (measured at 192^3:
  // 143 us against 178 us per step with a force field, 6-row tiles)
  const int64_t nx = h->p.nx;
  const int64_t waste1 = ceil_div(nx, 64) * 64 - nx;
  const int64_t waste2 = ceil_div(nx, 128) * 128 - nx;
  const int64_t waste3 = ceil_div(nx, 192) * 192 - nx;
  const bool three_ok = h->p.storage == LBF_F32 && h->p.lattice != LBF_D3Q27H && nx % 3 == 0 &&
                        nx >= 192 && !h->two_phase;
  if (nx % 2 == 0 && nx >= 128 && waste2 <= waste1)
    h->lane_sites = 2;
  else if (three_ok && waste3 <= waste1)
    h->lane_sites = 3;
  else
    h->lane_sites = 1;
  // D3Q27h spills registers with two sites per lane in FP64.  The 16-bit forms
  // keep two since their planes are grouped (measured at 512^3, one / two
  // sites: FP16 65.9 / 68.0 GLUPS, split FP16 61.0 / 67.1, BF16 70.0 / 70.2)
  if (h->p.lattice == LBF_D3Q27H && h->p.storage == LBF_F64) h->lane_sites = 1;
  h->tile_rows = 4;
  const bool f64 = h->p.storage == LBF_F64;
  const int first = f64 ? (h->lane_sites == 2 ? 4 : 6) : (h->lane_sites == 3 ? 6 : 8);
  for (int ty : {first, 6, 4})
    if (lds_bytes(h->p.lattice, h->p.storage, ty, h->lane_sites) <= kLdsLimit) {
      h->tile_rows = ty;
      break;
    }
  h->z_chunk = 0;
}

int resolve_zchunk(const lbfast_ctx* h, int lane_sites, int tile_rows, int* tiles_x, int* tiles_y,
                   int* zchunks, int* zchunk) {
  *tiles_x = static_cast<int>(ceil_div(h->p.nx, 64 * lane_sites));
  *tiles_y = static_cast<int>(ceil_div(h->p.ny, tile_rows));
  const int64_t cols = static_cast<int64_t>(*tiles_x) * *tiles_y;
  int64_t zc = h->z_chunk;
  if (zc <= 0) {
    // at most ~512 workgroups (~1024 for FP64 with two sites per lane, whose
    // 4-row tiles are short) in chunks of >= 64 planes; measured on MI355X,
    // shorter chunks or more workgroups cost 10-20% (256^3: 4 chunks of 64
    // planes 61 GLUPS, 8 of 32 planes 52; 512^3: 2 chunks 65, 4 chunks 52).
    // Grids too small for that many long chunks take enough workgroups
    // first, in chunks of >= 8 planes.
    const int64_t target = (h->p.storage == LBF_F64 && lane_sites == 2) ? 1024 : 512;
    const int64_t by_blocks = std::max<int64_t>(1, target / cols);
    const int64_t long_chunks = std::max<int64_t>(1, h->p.nz / 64);
    int64_t nchunks;
    if (cols * long_chunks >= 128) {
      nchunks = std::min(by_blocks, long_chunks);
    } else {
      const int64_t want = ceil_div(target, cols);
      const int64_t maxc = h->p.nz >= 8 ? h->p.nz / 8 : 1;
      nchunks = want < 1 ? 1 : (want > maxc ? maxc : want);
    }
    zc = ceil_div(h->p.nz, nchunks);
  }
  if (zc > h->p.nz) zc = h->p.nz;
  *zchunk = static_cast<int>(zc);
  *zchunks = static_cast<int>(ceil_div(h->p.nz, zc));
  if (static_cast<int64_t>(*zchunks) * cols > 0x7fffffff) return fail(LBF_E_ARG, "grid too large");
  return LBF_OK;
}

int check_handle(lbfast_t h) {
  if (!h) return fail(LBF_E_ARG, "handle is NULL");
  return LBF_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int now;
    if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
  }
};

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

// launch geometry, relaxation, force and scales of the handle's step
int step_args(const lbfast_ctx* h, lbf::StepArgs* a) {
  *a = lbf::StepArgs{};
  a->nx = static_cast<int>(h->p.nx);
  a->ny = static_cast<int>(h->p.ny);
  a->nz = static_cast<int>(h->p.nz);
  a->N = h->N;
  a->lane_sites = h->lane_sites;
  if (int rc = resolve_zchunk(h, h->lane_sites, h->tile_rows, &a->tiles_x, &a->tiles_y,
                              &a->zchunks, &a->zchunk))
    return rc;
  a->omega = 1.0 / h->p.tau;
  for (int k = 0; k < 3; ++k) a->F[k] = h->Ffield ? 0.0 : h->p.force[k];
  for (int k = 0; k < 10; ++k) {
    a->scale[k] = h->scale[k];
    a->inv_scale[k] = h->inv_scale[k];
  }
  {
    const double inv_d = 1.0 / ((h->p.lattice == LBF_D3Q19) ? 9.0 : 27.0);
    const float hi = static_cast<float>(inv_d);
    const float lo = static_cast<float>(inv_d - static_cast<double>(hi));
    for (int k = 0; k < 4; ++k) {
      a->enc_hi[k] = hi * h->inv_scale[k];
      a->enc_lo[k] = lo * h->inv_scale[k];
    }
  }
  a->Ffield = h->Ffield;
  // Block order, measured at 512^3 on one box with the two orders built as
  // separate libraries and run interleaved: contiguous tile ranges per XCD
  // are faster for FP64 (21% for D3Q19, 6% for D3Q27h) and for FP32 D3Q27
  // (3%), the hardware order for 16-bit storage (2-5%); D3Q19 FP32 and its
  // adjoint are equal within 1% and keep the hardware order.
  a->xcd_remap = h->block_order == 2 ||
                 (h->block_order == 0 &&
                  (h->p.storage == LBF_F64 || (h->p.storage == LBF_F32 && h->p.lattice != LBF_D3Q19)));
  a->stochastic = h->p.rounding == LBF_ROUND_STOCHASTIC ||
                  (h->p.rounding == LBF_ROUND_AUTO && h->p.storage == LBF_BF16S);
  if (h->two_phase) {
    // the phases' relaxation times replace params.tau
    a->omega = 1.0 / h->pp.tau_l;
    a->rho_l = h->pp.rho_l;
    a->rho_h = h->pp.rho_h;
    a->nu_l = (h->pp.tau_l - 0.5) / 3.0;
    a->nu_h = (h->pp.tau_h - 0.5) / 3.0;
  }
  return LBF_OK;
}

// seed of the stochastic rounding of step t (16-bit storage): the step
// counter through SplitMix64's output mix (Steele, Lea and Flood, 2014), so
// that every step draws fresh bits per site
uint32_t step_seed(uint64_t t) {
  uint64_t x = t + 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return static_cast<uint32_t>(x ^ (x >> 31));
}

int launch_forward(const lbfast_ctx* h, const lbf::StepArgs& a) {
  hipError_t e = lbf::launch_step(h->p.lattice, h->p.storage, h->tile_rows,
                                  h->p.bc[1] == LBF_WALLS, a, h->stream);
  if (e != hipSuccess) return hip_fail(e, "step launch");
  return LBF_OK;
}

size_t compute_bytes(const lbfast_ctx* h) { return h->p.storage == LBF_F64 ? 8 : 4; }

// phase-field launch arguments for the current time level
lbf::PhaseArgs phase_args(const lbfast_ctx* h) {
  lbf::PhaseArgs a{};
  a.phi = h->phi[h->pcur];
  a.phi_out = h->phi[h->pcur ^ 1];
  a.state = h->buf[h->cur];
  a.F = h->Fph[h->pcur ^ 1];
  a.nx = static_cast<int>(h->p.nx);
  a.ny = static_cast<int>(h->p.ny);
  a.nz = static_cast<int>(h->p.nz);
  a.N = h->N;
  a.D = h->pp.diffusivity;
  a.lambda = 4.0 * h->pp.diffusivity / h->pp.width;
  a.beta = 12.0 * h->pp.sigma / h->pp.width;
  a.kappa = 1.5 * h->pp.sigma * h->pp.width;
  a.eps = 1e-12;  // n = grad(phi) / (|grad(phi)| + eps)
  for (int k = 0; k < 3; ++k) a.Fb[k] = h->p.force[k];  // body acceleration
  for (int k = 0; k < 10; ++k) a.scale[k] = h->scale[k];
  a.walls_y = h->p.bc[1] == LBF_WALLS;
  a.contrast = h->pp.rho_l != h->pp.rho_h;
  a.rho_l = h->pp.rho_l;
  a.rho_h = h->pp.rho_h;
  a.nu_l = (h->pp.tau_l - 0.5) / 3.0;
  a.nu_h = (h->pp.tau_h - 0.5) / 3.0;
  return a;
}

// phases of unequal density or viscosity, or a density other than 1: the
// step reads the phase field for a density and relaxation rate per site
bool variable_properties(const lbfast_ctx* h) {
  return h->pp.rho_l != 1.0 || h->pp.rho_h != 1.0 || h->pp.tau_l != h->pp.tau_h;
}

int check_adjoint_args(const lbfast_ctx* h, int64_t nsteps, int64_t every) {
  if (h->two_phase)
    return fail(LBF_E_UNSUPPORTED, "the adjoint does not cover the two-component variant");
  if (h->p.storage != LBF_F64 && h->p.storage != LBF_F32)
    return fail(LBF_E_UNSUPPORTED, "the adjoint supports F64 and F32 storage only");
  if (h->p.lattice == LBF_D3Q27H)
    return fail(LBF_E_UNSUPPORTED, "the adjoint covers the second-order sets D3Q19 and D3Q27");
  if (nsteps < 0) return fail(LBF_E_ARG, "nsteps must be >= 0");
  if (every < 1) return fail(LBF_E_ARG, "every must be >= 1");
  return LBF_OK;
}

}  // namespace

extern "C" {

int lbfast_abi_version(void) { return LBFAST_ABI_VERSION; }

size_t lbfast_buffer_bytes(const lbfast_params* p) {
  if (validate(p) != LBF_OK) return 0;
  return static_cast<size_t>(p->nx) * static_cast<size_t>(p->ny) * static_cast<size_t>(p->nz) *
         state_planes(p->storage) * elem_bytes(p->storage);
}

const char* lbfast_last_error(void) { return g_err.c_str(); }

int lbfast_stream_probe(const void* src, void* dst, int64_t n, int nplanes, void* stream) {
  g_err.clear();
  if (!src || !dst) return fail(LBF_E_ARG, "null buffer");
  if (n < 1 || static_cast<double>(n) * 4.0 >= 4294967296.0)
    return fail(LBF_E_ARG, "n must be in [1, 2^30)");
  if (nplanes < 1) return fail(LBF_E_ARG, "nplanes must be >= 1");
  hipError_t e = lbf::launch_stream_probe(src, dst, n, nplanes, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "stream probe");
  return LBF_OK;
}

int lbfast_copy_probe(const void* src, void* dst, int64_t n4, void* stream) {
  g_err.clear();
  if (!src || !dst) return fail(LBF_E_ARG, "null buffer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
    return fail(LBF_E_ARG, "buffers must be 16-byte aligned");
  if (n4 < 1) return fail(LBF_E_ARG, "n4 must be >= 1");
  hipError_t e = lbf::launch_copy_probe(src, dst, n4, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "copy probe");
  return LBF_OK;
}

int lbfast_planes_probe(const void* src, void* dst, int64_t n, int nplanes, void* stream) {
  g_err.clear();
  if (!src || !dst) return fail(LBF_E_ARG, "null buffer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 7)
    return fail(LBF_E_ARG, "buffers must be 8-byte aligned");
  if (n < 2 || n % 2) return fail(LBF_E_ARG, "n must be even and >= 2");
  if (nplanes < 1 || nplanes > 10) return fail(LBF_E_ARG, "nplanes must be in [1, 10]");
  hipError_t e = lbf::launch_planes_probe(src, dst, n, nplanes, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "planes probe");
  return LBF_OK;
}

int lbfast_zmarch_probe(const void* src, void* dst, int nx, int ny, int nz, int layout,
                        int zchunk, void* stream) {
  g_err.clear();
  if (!src || !dst) return fail(LBF_E_ARG, "null buffer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
    return fail(LBF_E_ARG, "buffers must be 16-byte aligned");
  if (nx < 128 || nx % 128) return fail(LBF_E_ARG, "nx must be a positive multiple of 128");
  if (ny < 8 || ny % 8) return fail(LBF_E_ARG, "ny must be a positive multiple of 8");
  if (nz < 1 || zchunk < 1) return fail(LBF_E_ARG, "nz and zchunk must be >= 1");
  if (layout < 0 || layout > 3) return fail(LBF_E_ARG, "layout must be in [0, 3]");
  if (static_cast<int64_t>(nx / 128) * (ny / 8) * ((nz + zchunk - 1) / zchunk) > 0x7fffffff)
    return fail(LBF_E_ARG, "grid too large");
  hipError_t e = lbf::launch_zmarch_probe(src, dst, nx, ny, nz, layout, zchunk,
                                          static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "z-march probe");
  return LBF_OK;
}

int lbfast_create(const lbfast_params* p, void* stream, void* buf0, void* buf1, lbfast_t* out) {
  g_err.clear();
  if (!out) return fail(LBF_E_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc != LBF_OK) return rc;
  if ((buf0 == nullptr) != (buf1 == nullptr))
    return fail(LBF_E_ARG, "pass both buffers or neither");
  if (buf0 && buf0 == buf1) return fail(LBF_E_ARG, "buf0 and buf1 must differ");
  if ((buf0 && (reinterpret_cast<uintptr_t>(buf0) & 255)) ||
      (buf1 && (reinterpret_cast<uintptr_t>(buf1) & 255)))
    return fail(LBF_E_ARG, "buffers must be 256-byte aligned");

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");

  lbfast_ctx* h = new (std::nothrow) lbfast_ctx();
  if (!h) return fail(LBF_E_NOMEM, "host allocation failed");
  h->p = *p;
  h->device = dev;
  h->stream = static_cast<hipStream_t>(stream);
  h->N = p->nx * p->ny * p->nz;
  const size_t bytes = lbfast_buffer_bytes(p);
  for (int k = 0; k < 10; ++k) {
    h->scale[k] = (p->scale[k] != 0.0f) ? p->scale[k] : 1.0f;
    h->inv_scale[k] = 1.0f / h->scale[k];
  }
  const bool s16 = is_16bit(p->storage);
  h->scales_fixed = !s16;
  if (s16) {
    bool all = true;
    for (int k = 0; k < 10; ++k) all = all && p->scale[k] != 0.0f;
    h->scales_fixed = all;
  }
  default_launch(h);

  if (buf0) {
    h->buf[0] = buf0;
    h->buf[1] = buf1;
    h->owned = false;
  } else {
    h->owned = true;
    for (int i = 0; i < 2; ++i) {
      e = hipMalloc(&h->buf[i], bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        if (h->buf[0]) (void)hipFree(h->buf[0]);
        delete h;
        return fail(LBF_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
      }
    }
  }
  e = hipMalloc(reinterpret_cast<void**>(&h->d_partials),
                (lbf::kReduceBlocks * 5 + 5) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->d_maxbits), 16 * sizeof(unsigned));
  if (e == hipSuccess) e = hipMemsetAsync(h->buf[0], 0, bytes, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->buf[1], 0, bytes, h->stream);
  if (e != hipSuccess) {
    int r = hip_fail(e, "create");
    lbfast_destroy(h);
    return r;
  }
  *out = h;
  return LBF_OK;
}

int lbfast_destroy(lbfast_t h) {
  if (!h) return LBF_OK;
  DeviceGuard g(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  if (h->owned) {
    if (h->buf[0]) (void)hipFree(h->buf[0]);
    if (h->buf[1]) (void)hipFree(h->buf[1]);
  }
  for (void* p : {h->phi[0], h->phi[1], h->Fph[0], h->Fph[1]})
    if (p) (void)hipFree(p);
  if (h->d_partials) (void)hipFree(h->d_partials);
  if (h->d_maxbits) (void)hipFree(h->d_maxbits);
  delete h;
  return LBF_OK;
}

int lbfast_set_moments(lbfast_t h, const void* m, int dtype, int on_device) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (!m) return fail(LBF_E_ARG, "moment array is NULL");
  if (dtype != LBF_F64 && dtype != LBF_F32) return fail(LBF_E_ARG, "dtype must be F64 or F32");
  if (on_device != 0 && on_device != 1) return fail(LBF_E_ARG, "on_device must be 0 or 1");
  DeviceGuard g(h->device);
  const size_t ub = (dtype == LBF_F64) ? 8 : 4;
  const int64_t N = h->N;
  const size_t pbytes = static_cast<size_t>(N) * ub;
  hipError_t e = hipSuccess;
  // Device input is read in place.  Host input goes through a device staging
  // area: the three velocity planes (kept for the whole call, the deviation
  // storage of the second-order planes needs them) and one plane at a time.
  char* staging = nullptr;
  if (!on_device) {
    e = hipMalloc(reinterpret_cast<void**>(&staging), 4 * pbytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(LBF_E_NOMEM, "staging allocation failed");
    }
    e = hipMemcpyAsync(staging, static_cast<const char*>(m) + pbytes, 3 * pbytes,
                       hipMemcpyHostToDevice, h->stream);
  }
  const void* u[3];
  for (int c = 0; c < 3; ++c)
    u[c] = on_device ? static_cast<const char*>(m) + (1 + c) * pbytes
                     : static_cast<const void*>(staging + c * pbytes);
  // device pointer of user plane k (host planes are copied in first)
  auto plane = [&](int k, hipError_t& err) -> const void* {
    if (on_device) return static_cast<const char*>(m) + k * pbytes;
    if (k >= 1 && k <= 3) return staging + (k - 1) * pbytes;
    char* p = staging + 3 * pbytes;
    err = hipMemcpyAsync(p, static_cast<const char*>(m) + k * pbytes, pbytes,
                         hipMemcpyHostToDevice, h->stream);
    return p;
  };
  // automatic 16-bit scales: the power of two placing the magnitude M of the
  // plane's group just below 2^10, which leaves a factor 64 of growth before
  // FP16 overflows (65504); FP16 keeps its relative precision down to 2^-14.
  // M is max|u| for the velocity planes, max(|a2|, max|u|^2) for the
  // second-order planes and max(|p*|, 3 max|u|^2) for p*: a plane that starts
  // at zero (p* of a solenoidal field, u_z of a planar flow) takes its group's
  // magnitude instead of a scale of 1, which would put its later values in
  // FP16's subnormal range.
  if (!h->scales_fixed) {
    float mx[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
      const int k0 = pass == 0 ? 0 : 4, k1 = pass == 0 ? 4 : 10;
      e = hipMemsetAsync(h->d_maxbits, 0, 16 * sizeof(unsigned), h->stream);
      for (int k = k0; k < k1 && e == hipSuccess; ++k) {
        const void* src = plane(k, e);
        if (e == hipSuccess)
          e = lbf::launch_maxabs(h->p.storage, dtype, src, u, N, k, h->inv_scale, h->scale,
                                 h->d_maxbits, h->stream);
        // the single plane slot of the staging area is reused: wait before the next copy
        if (e == hipSuccess && !on_device) e = hipStreamSynchronize(h->stream);
      }
      unsigned bits[16];
      if (e == hipSuccess)
        e = hipMemcpyAsync(bits, h->d_maxbits, sizeof bits, hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) break;
      for (int k = k0; k < k1; ++k) {
        std::memcpy(&mx[k], &bits[k], sizeof(float));
        if (!std::isfinite(mx[k])) mx[k] = 0.0f;
      }
    }
    if (e == hipSuccess) {
      const float um = std::max(mx[1], std::max(mx[2], mx[3]));
      float am = um * um;
      for (int k = 4; k < 10; ++k) am = std::max(am, mx[k]);
      const float pm = std::max(mx[0], 3.0f * um * um);
      for (int k = 0; k < 10; ++k) {
        if (h->p.scale[k] != 0.0f) continue;
        const float M = k == 0 ? pm : (k < 4 ? um : am);
        float sc = 1.0f;
        if (M > 0.0f) {
          int ex;
          std::frexp(M, &ex);              // M in [2^(ex-1), 2^ex)
          sc = std::ldexp(1.0f, ex - 10);  // M / sc < 2^10
        }
        h->scale[k] = sc;
        h->inv_scale[k] = 1.0f / sc;
      }
      h->scales_fixed = true;
    }
  }
  void* dst = h->buf[h->cur];
  for (int k = 0; k < 10 && e == hipSuccess; ++k) {
    const void* src = plane(k, e);
    if (e == hipSuccess)
      e = lbf::launch_encode(h->p.storage, dtype, src, u, dst, N, k, h->inv_scale, h->scale,
                             h->stream);
    if (e == hipSuccess && !on_device) e = hipStreamSynchronize(h->stream);
  }
  if (staging) {
    hipError_t e2 = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = e2;
    (void)hipFree(staging);
  }
  if (e != hipSuccess) return hip_fail(e, "set_moments");
  return LBF_OK;
}

int lbfast_get_moments(lbfast_t h, void* m, int dtype, int on_device) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (!m) return fail(LBF_E_ARG, "moment array is NULL");
  if (dtype != LBF_F64 && dtype != LBF_F32) return fail(LBF_E_ARG, "dtype must be F64 or F32");
  if (on_device != 0 && on_device != 1) return fail(LBF_E_ARG, "on_device must be 0 or 1");
  DeviceGuard g(h->device);
  const size_t ub = (dtype == LBF_F64) ? 8 : 4;
  const int64_t N = h->N;
  const size_t pbytes = static_cast<size_t>(N) * ub;
  const void* src = h->buf[h->cur];
  hipError_t e = hipSuccess;
  void* staging = nullptr;
  if (!on_device) {
    e = hipMalloc(&staging, pbytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(LBF_E_NOMEM, "staging allocation failed");
    }
  }
  for (int k = 0; k < 10 && e == hipSuccess; ++k) {
    void* dst = on_device ? static_cast<void*>(static_cast<char*>(m) + k * pbytes) : staging;
    e = lbf::launch_decode(h->p.storage, dtype, src, dst, N, k, h->scale, h->stream);
    if (e == hipSuccess && !on_device)
      e = hipMemcpyAsync(static_cast<char*>(m) + k * pbytes, staging, pbytes,
                         hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && !on_device) e = hipStreamSynchronize(h->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (staging) (void)hipFree(staging);
  if (e != hipSuccess) return hip_fail(e, "get_moments");
  return LBF_OK;
}

int lbfast_set_force_field(lbfast_t h, const void* F_dev, int dtype) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (h->two_phase)
    return fail(LBF_E_STATE, "the two-component variant computes its own force field");
  if (!F_dev) {
    h->Ffield = nullptr;
    return LBF_OK;
  }
  const int want = (h->p.storage == LBF_F64) ? LBF_F64 : LBF_F32;
  if (dtype != want)
    return fail(LBF_E_ARG, "force field dtype must be the compute type (%s)",
                want == LBF_F64 ? "F64" : "F32");
  if (reinterpret_cast<uintptr_t>(F_dev) & (dtype == LBF_F64 ? 7 : 3))
    return fail(LBF_E_ARG, "force field is misaligned");
  if (!is_device_ptr(F_dev)) return fail(LBF_E_ARG, "force field must be device memory");
  h->Ffield = F_dev;
  return LBF_OK;
}

int lbfast_set_launch(lbfast_t h, int tile_rows, int z_chunk) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (tile_rows != 0) {
    bool ok = false;
    for (int t : lbf::kTileRowsSupported) ok = ok || t == tile_rows;
    if (!ok) return fail(LBF_E_ARG, "tile_rows %d not supported (4, 6, 8 or 14)", tile_rows);
    if (h->lane_sites >= 2 && tile_rows > 8)
      return fail(LBF_E_UNSUPPORTED, "two or three x-sites per lane support tiles of at most 8 rows");
    if (h->p.lattice == LBF_D3Q27H && tile_rows > 8)
      return fail(LBF_E_UNSUPPORTED, "D3Q27h supports tiles of at most 8 rows");
    const size_t lb = lds_bytes(h->p.lattice, h->p.storage, tile_rows, h->lane_sites, h->two_phase);
    if (lb > kLdsLimit)
      return fail(LBF_E_UNSUPPORTED, "tile_rows %d needs %zu bytes of LDS (limit 160 KiB)",
                  tile_rows, lb);
  }
  if (z_chunk < 0) return fail(LBF_E_ARG, "z_chunk must be >= 0");
  if (tile_rows) h->tile_rows = tile_rows;
  if (z_chunk) h->z_chunk = z_chunk;
  return LBF_OK;
}

int lbfast_set_block_order(lbfast_t h, int order) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (order < 0 || order > 2) return fail(LBF_E_ARG, "order must be 0, 1 or 2");
  h->block_order = order;
  return LBF_OK;
}

int lbfast_set_lane_sites(lbfast_t h, int sites) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (sites != 1 && sites != 2 && sites != 3) return fail(LBF_E_ARG, "sites must be 1, 2 or 3");
  if (sites == 2 && h->p.nx % 2 != 0)
    return fail(LBF_E_UNSUPPORTED, "two x-sites per lane need an even nx");
  if (sites == 3 && (h->p.nx % 3 != 0 || h->p.storage != LBF_F32 ||
                     h->p.lattice == LBF_D3Q27H || h->two_phase))
    return fail(LBF_E_UNSUPPORTED,
                "three x-sites per lane need nx divisible by 3, F32 storage, a second-order "
                "set and one component");
  // keep the tile height if it fits, else the tallest one (of 8, 6, 4) that does
  int ty = h->tile_rows;
  if ((sites >= 2 && ty > 8) ||
      lds_bytes(h->p.lattice, h->p.storage, ty, sites, h->two_phase) > kLdsLimit) {
    ty = 0;
    for (int t : {8, 6, 4})
      if (lds_bytes(h->p.lattice, h->p.storage, t, sites, h->two_phase) <= kLdsLimit) {
        ty = t;
        break;
      }
    if (ty == 0) return fail(LBF_E_UNSUPPORTED, "no tile height fits %d sites per lane", sites);
  }
  h->lane_sites = sites;
  h->tile_rows = ty;
  return LBF_OK;
}

int lbfast_set_adjoint_launch(lbfast_t h, int sites, int tile_rows) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (sites < 0 || sites > 3) return fail(LBF_E_ARG, "sites must be 0, 1, 2 or 3");
  if (tile_rows != 0 && tile_rows != 4 && tile_rows != 6 && tile_rows != 8 && tile_rows != 14)
    return fail(LBF_E_ARG, "tile_rows must be 0, 4, 6, 8 or 14");
  const int S = sites ? sites : 1;
  const int ty = tile_rows ? tile_rows : (h->p.storage == LBF_F64 ? 6 : 8);
  if (S > 1) {
    if (h->p.storage != LBF_F32)
      return fail(LBF_E_UNSUPPORTED, "two or three sites per lane: F32 storage only");
    if ((S == 2 && h->p.nx % 2 != 0) || (S == 3 && h->p.nx % 3 != 0))
      return fail(LBF_E_UNSUPPORTED, "nx must be divisible by the sites per lane");
    if (ty > 6 || (h->p.lattice == LBF_D3Q27 && ty != 4) ||
        (h->p.lattice == LBF_D3Q19 && ty != 4 && ty != 6))
      return fail(LBF_E_UNSUPPORTED,
                  "two or three sites per lane: 4- or 6-row tiles (D3Q27: 4 rows)");
  }
  h->adj_sites = sites;
  h->adj_rows = tile_rows;
  return LBF_OK;
}

int lbfast_step(lbfast_t h, int64_t n) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (n < 0) return fail(LBF_E_ARG, "n must be >= 0");
  if (n == 0) return LBF_OK;
  if (!h->scales_fixed) return fail(LBF_E_STATE, "16-bit scales not set: call set_moments first");
  DeviceGuard g(h->device);
  lbf::StepArgs a;
  if (int rc = step_args(h, &a)) return rc;
  for (int64_t s = 0; s < n; ++s) {
    a.src = h->buf[h->cur];
    a.dst = h->buf[h->cur ^ 1];
    a.sr_seed = step_seed(h->steps_done++);
    if (h->two_phase) {
      // phi(t+1) first: the step computes F(t+1) from it for the correction
      lbf::PhaseArgs pa = phase_args(h);
      hipError_t e = lbf::launch_phase_step(h->p.storage, pa, h->stream);
      if (e != hipSuccess) return hip_fail(e, "phase-field launch");
      a.Ffield = h->Fph[h->pcur];
      a.Fout = h->Fph[h->pcur ^ 1];
      a.phi_dst = h->phi[h->pcur ^ 1];
      a.beta = pa.beta;
      a.kappa = pa.kappa;
      for (int k = 0; k < 3; ++k) a.Fb[k] = pa.Fb[k];
      a.contrast = pa.contrast;
      if (variable_properties(h)) a.phi_src = h->phi[h->pcur];
    }
    if (int rc = launch_forward(h, a)) return rc;
    h->cur ^= 1;
    if (h->two_phase) h->pcur ^= 1;
  }
  return LBF_OK;
}

int lbfast_enable_two_phase(lbfast_t h, const lbfast_phase_params* pp) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (!pp) return fail(LBF_E_ARG, "phase params is NULL");
  if (pp->struct_size != sizeof(lbfast_phase_params))
    return fail(LBF_E_ARG, "phase params struct_size = %u, expected %zu", pp->struct_size,
                sizeof(lbfast_phase_params));
  if (pp->reserved0 != 0) return fail(LBF_E_ARG, "reserved0 must be zero");
  if (!std::isfinite(pp->sigma) || pp->sigma < 0) return fail(LBF_E_ARG, "sigma must be >= 0");
  if (!std::isfinite(pp->width) || !(pp->width > 0)) return fail(LBF_E_ARG, "width must be > 0");
  if (!std::isfinite(pp->diffusivity) || pp->diffusivity < 0)
    return fail(LBF_E_ARG, "diffusivity must be >= 0");
  if (!std::isfinite(pp->rho_l) || !std::isfinite(pp->rho_h) || !(pp->rho_l > 0) ||
      !(pp->rho_h > 0))
    return fail(LBF_E_ARG, "phase densities must be finite and > 0");
  if (!std::isfinite(pp->tau_l) || !std::isfinite(pp->tau_h) || !(pp->tau_l > 0.5) ||
      !(pp->tau_h > 0.5))
    return fail(LBF_E_ARG, "phase relaxation times must be finite and > 1/2");
  if (h->p.bc[0] != LBF_PERIODIC || h->p.bc[2] != LBF_PERIODIC)
    return fail(LBF_E_UNSUPPORTED, "walls are supported on the y axis only");
  if (h->p.storage == LBF_F16SU)
    return fail(LBF_E_UNSUPPORTED, "the two-component variant does not cover LBF_F16SU storage");
  if (h->Ffield) return fail(LBF_E_STATE, "a per-site force field is set");
  if (h->two_phase) return fail(LBF_E_STATE, "two-component variant already enabled");
  DeviceGuard g(h->device);
  const size_t c = compute_bytes(h);
  const size_t pb = static_cast<size_t>(h->N) * c;
  hipError_t e = hipSuccess;
  void** slots[4] = {&h->phi[0], &h->phi[1], &h->Fph[0], &h->Fph[1]};
  const size_t sizes[4] = {pb, pb, 3 * pb, 3 * pb};
  for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipMalloc(slots[i], sizes[i]);
  for (int i = 0; i < 4 && e == hipSuccess; ++i)
    e = lbf::launch_zero(*slots[i], static_cast<int64_t>(sizes[i]), h->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    for (int i = 0; i < 4; ++i)
      if (*slots[i]) {
        (void)hipFree(*slots[i]);
        *slots[i] = nullptr;
      }
    return fail(LBF_E_NOMEM, "two-component buffers: %s", hipGetErrorString(e));
  }
  h->pp = *pp;
  h->two_phase = true;
  h->pcur = 0;
  // The two-component step has one- and two-site forms of at most 8 rows,
  // with one more LDS slot (phi(t+1)) than the one-component step.  With
  // variable density or viscosity, one site per lane: the two-site form
  // spills registers there (measured at 256^3 FP32: 0.80 ms against 0.57).
  const bool one_site = h->lane_sites == 3 || (h->lane_sites == 2 && variable_properties(h));
  const bool reshape = one_site || h->tile_rows > 8 ||
                       lds_bytes(h->p.lattice, h->p.storage, h->tile_rows, h->lane_sites,
                                 true) > kLdsLimit;
  if (one_site) h->lane_sites = 1;
  if (reshape) {
    h->tile_rows = 4;
    for (int ty : {8, 6})
      if (lds_bytes(h->p.lattice, h->p.storage, ty, h->lane_sites, true) <= kLdsLimit) {
        h->tile_rows = ty;
        break;
      }
  }
  // F(0) of phi = 0: the body force alone
  lbf::PhaseArgs pa = phase_args(h);
  pa.phi_out = h->phi[0];
  pa.F = h->Fph[0];
  e = lbf::launch_capillary_force(h->p.storage, pa, h->stream);
  if (e != hipSuccess) return hip_fail(e, "capillary force");
  return LBF_OK;
}

int lbfast_set_phase(lbfast_t h, const void* phi, int dtype, int on_device) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (!h->two_phase) return fail(LBF_E_STATE, "two-component variant not enabled");
  if (!phi) return fail(LBF_E_ARG, "phi is NULL");
  if (dtype != LBF_F64 && dtype != LBF_F32) return fail(LBF_E_ARG, "dtype must be F64 or F32");
  if (on_device != 0 && on_device != 1) return fail(LBF_E_ARG, "on_device must be 0 or 1");
  DeviceGuard g(h->device);
  const size_t ub = (dtype == LBF_F64) ? 8 : 4;
  const size_t bytes = static_cast<size_t>(h->N) * ub;
  const void* src = phi;
  void* staging = nullptr;
  hipError_t e = hipSuccess;
  if (!on_device) {
    e = hipMalloc(&staging, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(LBF_E_NOMEM, "staging allocation failed");
    }
    e = hipMemcpyAsync(staging, phi, bytes, hipMemcpyHostToDevice, h->stream);
    src = staging;
  }
  if (e == hipSuccess)
    e = lbf::launch_convert(h->p.storage, dtype, src, 0, h->phi[h->pcur], h->N, h->stream);
  if (e == hipSuccess) {
    lbf::PhaseArgs pa = phase_args(h);
    pa.phi_out = h->phi[h->pcur];
    pa.F = h->Fph[h->pcur];
    e = lbf::launch_capillary_force(h->p.storage, pa, h->stream);
  }
  if (staging) {
    hipError_t e2 = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = e2;
    (void)hipFree(staging);
  }
  if (e != hipSuccess) return hip_fail(e, "set_phase");
  return LBF_OK;
}

int lbfast_get_phase(lbfast_t h, void* phi, int dtype, int on_device) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (!h->two_phase) return fail(LBF_E_STATE, "two-component variant not enabled");
  if (!phi) return fail(LBF_E_ARG, "phi is NULL");
  if (dtype != LBF_F64 && dtype != LBF_F32) return fail(LBF_E_ARG, "dtype must be F64 or F32");
  if (on_device != 0 && on_device != 1) return fail(LBF_E_ARG, "on_device must be 0 or 1");
  DeviceGuard g(h->device);
  const size_t ub = (dtype == LBF_F64) ? 8 : 4;
  const size_t bytes = static_cast<size_t>(h->N) * ub;
  void* dst = phi;
  void* staging = nullptr;
  hipError_t e = hipSuccess;
  if (!on_device) {
    e = hipMalloc(&staging, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(LBF_E_NOMEM, "staging allocation failed");
    }
    dst = staging;
  }
  e = lbf::launch_convert(h->p.storage, dtype, h->phi[h->pcur], 1, dst, h->N, h->stream);
  if (e == hipSuccess && staging)
    e = hipMemcpyAsync(phi, staging, bytes, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (staging) (void)hipFree(staging);
  if (e != hipSuccess) return hip_fail(e, "get_phase");
  return LBF_OK;
}

int lbfast_forward_checkpointed(lbfast_t h, int64_t nsteps, int64_t every, void* ckpt_dev) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (int rc = check_adjoint_args(h, nsteps, every)) return rc;
  if (nsteps > 0 && !ckpt_dev) return fail(LBF_E_ARG, "ckpt_dev is NULL");
  if (reinterpret_cast<uintptr_t>(ckpt_dev) & 255)
    return fail(LBF_E_ARG, "ckpt_dev must be 256-byte aligned");
  DeviceGuard g(h->device);
  const size_t bytes = lbfast_buffer_bytes(&h->p);
  lbf::StepArgs a;
  if (int rc = step_args(h, &a)) return rc;
  char* ck = static_cast<char*>(ckpt_dev);
  if (every == 1 && nsteps > 0) {
    // every state is kept: each step writes straight into the next slot, and
    // only the last one (the final state, which has no slot) into the buffer
    hipError_t e = hipMemcpyAsync(ck, h->buf[h->cur], bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
    for (int64_t t = 0; t < nsteps; ++t) {
      a.src = ck + t * bytes;
      a.dst = (t + 1 < nsteps) ? static_cast<void*>(ck + (t + 1) * bytes) : h->buf[h->cur ^ 1];
      if (int rc = launch_forward(h, a)) return rc;
    }
    h->cur ^= 1;
    return LBF_OK;
  }
  for (int64_t t = 0; t < nsteps; ++t) {
    if (t % every == 0) {
      hipError_t e = hipMemcpyAsync(ck + (t / every) * bytes, h->buf[h->cur], bytes,
                                    hipMemcpyDeviceToDevice, h->stream);
      if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
    }
    a.src = h->buf[h->cur];
    a.dst = h->buf[h->cur ^ 1];
    if (int rc = launch_forward(h, a)) return rc;
    h->cur ^= 1;
  }
  return LBF_OK;
}

size_t lbfast_adjoint_work_bytes(lbfast_t h, int64_t every) {
  if (!h || every < 1) return 0;
  return static_cast<size_t>(every + 2) * lbfast_buffer_bytes(&h->p);
}

int lbfast_adjoint(lbfast_t h, int64_t nsteps, int64_t every, const void* ckpt_dev,
                   const void* lambda_T_dev, void* gF_dev, void* lambda0_dev, void* work_dev) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (int rc = check_adjoint_args(h, nsteps, every)) return rc;
  if (!lambda_T_dev || !gF_dev) return fail(LBF_E_ARG, "lambda_T_dev and gF_dev are required");
  if (nsteps > 0 && (!ckpt_dev || !work_dev))
    return fail(LBF_E_ARG, "ckpt_dev and work_dev are required for nsteps > 0");
  const size_t ce = (h->p.storage == LBF_F64) ? 8 : 4;
  for (const void* p : {ckpt_dev, static_cast<const void*>(work_dev)})
    if (reinterpret_cast<uintptr_t>(p) & 255)
      return fail(LBF_E_ARG, "ckpt_dev and work_dev must be 256-byte aligned");
  for (const void* p : {lambda_T_dev, static_cast<const void*>(gF_dev),
                        static_cast<const void*>(lambda0_dev)})
    if (reinterpret_cast<uintptr_t>(p) & (ce - 1))
      return fail(LBF_E_ARG, "adjoint arrays must be aligned to the compute type");
  DeviceGuard g(h->device);
  const size_t bytes = lbfast_buffer_bytes(&h->p);
  const int64_t N = h->N;
  hipError_t e = lbf::launch_zero(gF_dev, 3 * N * static_cast<int64_t>(ce), h->stream);
  if (e != hipSuccess) return hip_fail(e, "zero dJ/dF");
  if (nsteps == 0) {
    if (lambda0_dev) {
      e = hipMemcpyAsync(lambda0_dev, lambda_T_dev, bytes, hipMemcpyDeviceToDevice, h->stream);
      if (e != hipSuccess) return hip_fail(e, "adjoint copy");
    }
    return LBF_OK;
  }
  char* work = static_cast<char*>(work_dev);
  // work: recomputed states 1..every of a segment, then two adjoint buffers
  void* lam[2] = {work + every * bytes, work + (every + 1) * bytes};
  e = hipMemcpyAsync(lam[0], lambda_T_dev, bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint copy");
  int cur = 0;
  lbf::StepArgs fa, aa;
  if (int rc = step_args(h, &fa)) return rc;
  aa = fa;
  aa.gF = gF_dev;
  // The adjoint step reads 22 values per destination site: by default one
  // site per lane and 8-row tiles (FP64: 6); lbfast_set_adjoint_launch may
  // choose two or three sites per lane with 4- or 6-row tiles (FP32)
  aa.lane_sites = h->adj_sites ? h->adj_sites : 1;
  const int adj_rows = h->adj_rows ? h->adj_rows : ((h->p.storage == LBF_F64) ? 6 : 8);
  if (int rc = resolve_zchunk(h, aa.lane_sites, adj_rows, &aa.tiles_x, &aa.tiles_y, &aa.zchunks,
                              &aa.zchunk))
    return rc;
  const int64_t nseg = (nsteps + every - 1) / every;
  const bool walls_y = h->p.bc[1] == LBF_WALLS;
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t len = std::min(every, nsteps - seg * every);
    char* ck = static_cast<char*>(const_cast<void*>(ckpt_dev));
    // a segment's end state is the next checkpoint, except for the last
    // segment, whose end (the final state) is recomputed; with every == 1
    // only that one state is recomputed at all
    const bool end_stored = seg + 1 < nseg;
    auto state = [&](int64_t j) -> void* {  // state at t = seg*every + j
      if (j == 0) return ck + seg * bytes;
      if (j == len && end_stored) return ck + (seg + 1) * bytes;
      return work + (j - 1) * bytes;
    };
    for (int64_t j = 0; j < (end_stored ? len - 1 : len); ++j) {  // recompute the segment
      fa.src = state(j);
      fa.dst = state(j + 1);
      if (int rc = launch_forward(h, fa)) return rc;
    }
    for (int64_t j = len - 1; j >= 0; --j) {  // sweep it backwards
      aa.src = lam[cur];
      aa.dst = lam[cur ^ 1];
      aa.state_old = state(j);
      aa.state_new = state(j + 1);
      e = lbf::launch_adjoint(h->p.lattice, h->p.storage, adj_rows, walls_y, aa, h->stream);
      if (e != hipSuccess) return hip_fail(e, "adjoint launch");
      cur ^= 1;
    }
  }
  if (lambda0_dev) {
    e = hipMemcpyAsync(lambda0_dev, lam[cur], bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint copy");
  }
  return LBF_OK;
}

int lbfast_sync(lbfast_t h) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  DeviceGuard g(h->device);
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "sync");
  return LBF_OK;
}

int lbfast_reduce(lbfast_t h, double out[5]) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (!out) return fail(LBF_E_ARG, "out is NULL");
  DeviceGuard g(h->device);
  double* d_out = h->d_partials + lbf::kReduceBlocks * 5;
  hipError_t e = lbf::launch_reduce(h->p.storage, h->buf[h->cur], h->N, h->scale, h->d_partials,
                                    d_out, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, d_out, 5 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "reduce");
  for (int k = 0; k < 5; ++k)
    if (!std::isfinite(out[k])) return fail(LBF_E_NONFINITE, "non-finite sum %d in the state", k);
  return LBF_OK;
}

int lbfast_state_ptr(lbfast_t h, void** dev_ptr) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (!dev_ptr) return fail(LBF_E_ARG, "dev_ptr is NULL");
  *dev_ptr = h->buf[h->cur];
  return LBF_OK;
}

int lbfast_get_scales(lbfast_t h, float out[10]) {
  g_err.clear();
  if (int rc = check_handle(h)) return rc;
  if (!out) return fail(LBF_E_ARG, "out is NULL");
  for (int k = 0; k < 10; ++k) out[k] = h->scale[k];
  return LBF_OK;
}

}  // extern "C"
