// internal.hpp -- declarations shared by the host runtime (lbfast.cpp) and
// the kernel launchers (*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbf {

// the calling thread's message for lbfast_last_error (lbfast.cpp)
void clear_error();
int set_error(int code, const char* msg);

// Arguments of one fused step launch (by value into the kernel).
struct StepArgs {
  const void* src;     // current moment buffer (10 planes)
  void* dst;           // next moment buffer (10 planes)
  const void* Ffield;  // 3 planes of the compute type, or nullptr (uniform F)
  // Two-component flow (else nullptr): Ffield holds F(t); the step computes
  // F(t+1) from phi(t+1) (phi_dst, N values of the compute type) at each
  // destination, uses it in the correction and writes it to Fout (3 planes).
  // F = mu grad(phi) + rho(phi) Fb, mu = 4 beta phi (phi - 1)(phi - 1/2) -
  // kappa lap(phi); with `contrast` also the pressure and viscous terms.
  void* Fout;
  const void* phi_dst;
  double beta, kappa, Fb[3];
  int contrast;
  // variable density and viscosity (else nullptr): phi(t) at the sources;
  // rho = rho_l + phi (rho_h - rho_l), likewise nu
  const void* phi_src;
  double rho_l, rho_h, nu_l, nu_h;
  int nx, ny, nz;
  int64_t N;           // plane stride = nx*ny*nz
  int tiles_x, tiles_y, zchunks, zchunk;
  int lane_sites;      // consecutive x-sites per lane: 1, 2 or 3 (tile width 64, 128, 192)
  int xcd_remap;       // give each XCD a contiguous range of tiles (else hardware order)
  double omega;
  double F[3];         // uniform force (used when Ffield == nullptr)
  float scale[10];     // 16-bit storage: value = scale * q
  float inv_scale[10];
  // 16-bit storage: inv_scale[k] / D (D the velocity set's weight
  // denominator) for p* and u as a hi + lo pair, hi = fl(1/D) inv_scale[k],
  // lo = fl(1/D - fl(1/D)) inv_scale[k] (exact: the scales are powers of two)
  float enc_hi[4], enc_lo[4];
  uint32_t sr_seed;    // 16-bit storage: seed of this step's stochastic rounding
  int stochastic;      // 16-bit storage: round p* and u stochastically
  // adjoint step only (src/dst then hold the adjoint variables at t+1 / t)
  const void* state_old;  // moments at t (10 planes; the velocity planes are read)
  const void* state_new;  // moments at t+1
  void* gF;               // 3 planes, dJ/dF accumulated in place
};

// rows per tile supported by the step kernel
constexpr int kTileRowsSupported[] = {4, 6, 8, 14};

// Launch one fused step.  Returns hipErrorInvalidValue for an unsupported
// combination.  nblocks = tiles_x * tiles_y * zchunks.
hipError_t launch_step(int Q, int storage, int tile_rows, bool walls_y, const StepArgs& a,
                       hipStream_t stream);

// One step of the discrete adjoint (FP64 or FP32 storage only).
hipError_t launch_adjoint(int Q, int storage, int tile_rows, bool walls_y, const StepArgs& a,
                          hipStream_t stream);

// Two-component variant: arguments of the phase-field kernels (compute type
// C = double for FP64 storage, float otherwise).
struct PhaseArgs {
  const void* phi;    // phi(t), N values of C
  void* phi_out;      // phi(t+1)
  const void* state;  // moment buffer at t (its velocity planes are read)
  void* F;            // receives F(t+1): 3 planes of C
  int nx, ny, nz;
  int64_t N;
  double D, lambda, beta, kappa, eps;
  double Fb[3];       // body acceleration g: the force adds rho(phi) g
  float scale[10];    // storage scales (16-bit storage)
  int walls_y;        // halfway walls in y: mirror images for the stencils
  int contrast;       // add the pressure and viscous force terms
  double rho_l, rho_h, nu_l, nu_h;
};
// phi_out = FTCS step of the Allen-Cahn equation from phi and the state's u
hipError_t launch_phase_step(int storage, const PhaseArgs& a, hipStream_t stream);
// F = mu(phi_out) grad(phi_out) + Fb
hipError_t launch_capillary_force(int storage, const PhaseArgs& a, hipStream_t stream);
// n values between a user array (F64 or F32) and the compute type of the storage:
// dst_is_user = 0 converts user -> compute type, 1 compute type -> user
hipError_t launch_convert(int storage, int user_dtype, const void* src, int dst_is_user,
                          void* dst, int64_t n, hipStream_t stream);

// zero nbytes bytes (a multiple of 4) with a kernel, so that graph capture
// records no memset node
hipError_t launch_zero(void* p, int64_t nbytes, hipStream_t stream);

// copy nplanes planes of n floats (n * 4 < 2^32) with the step's memory
// instruction forms
hipError_t launch_stream_probe(const void* src, void* dst, int64_t n, int nplanes,
                               hipStream_t stream);

// Conversions between user planes (F64 or F32, N values each) and plane k of
// a storage buffer.  u[0..2] are the user's velocity planes (the deviation
// storage of the second-order planes needs them); scale/inv_scale: the 10
// per-plane storage scales.
hipError_t launch_encode(int storage, int user_dtype, const void* plane, const void* const u[3],
                         void* buf, int64_t N, int k, const float* inv_scale, const float* scale,
                         hipStream_t stream);
hipError_t launch_decode(int storage, int user_dtype, const void* buf, void* plane, int64_t N,
                         int k, const float* scale, hipStream_t stream);
// max |stored value| of user plane k into out_bits[k] (float bits, zeroed before)
hipError_t launch_maxabs(int storage, int user_dtype, const void* plane, const void* const u[3],
                         int64_t N, int k, const float* inv_scale, const float* scale,
                         unsigned* out_bits, hipStream_t stream);
// FP64 sums [a0, a1x, a1y, a1z, 1/2 |a1|^2] of the state into out[5]
// (partials: kReduceBlocks*5 doubles of scratch)
constexpr int kReduceBlocks = 1024;
hipError_t launch_reduce(int storage, const void* buf, int64_t N, const float* scale,
                         double* partials, double* out, hipStream_t stream);

}  // namespace lbf
