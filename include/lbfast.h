/*
 * lbfast.h -- C ABI of the moment-represented ("lightweight") regularized
 * lattice Boltzmann step for AMD Instinct MI355X (gfx950).
 *
 * Method (Lauricella et al., "LBFAST: a lightweight moment-represented
 * lattice Boltzmann solver", arXiv 2609.09160):
 *   - every lattice site stores only the ten second-order Hermite
 *     coefficients a0 = p*, a1 = u (3), a2 (6, symmetric) (section 3,
 *     "Implementation", description of the two ten-field flip/flop arrays);
 *   - one fused step rebuilds the post-collision populations of the
 *     neighbours from their moments (Eqs. (4a,b), (6)), pulls them (Eq. (3))
 *     and projects them back onto the Hermite basis (Eqs. (5), (7));
 *   - the force-consistent correction of Eq. (8) with the Guo source of
 *     Eq. (9) closes the step.
 *
 * Conventions shared by every entry point
 *   - N = nx*ny*nz sites; site index s = x + nx*(y + ny*z) (x fastest).
 *   - A "moment array" is 10 planes of N values (structure of arrays), plane
 *     order m = [a0, a1x, a1y, a1z, a2xx, a2yy, a2zz, a2xy, a2xz, a2yz].
 *     a0 is the rescaled pressure p* = p/(rho cs^2), a1 the velocity and a2
 *     the total second-order Hermite coefficient (equilibrium u u plus the
 *     non-equilibrium part), exactly as defined under Eq. (6).  rho is the
 *     phase density, identically 1 for one component.
 *   - Lattice speed of sound cs^2 = 1/3, omega = 1/tau, nu = cs^2 (tau - 1/2).
 *   - A force array is 3 planes of N values (Fx, Fy, Fz), force per unit
 *     volume as in Eq. (9).
 *   - Every call returns an int status (LBF_OK or a negative LBF_E_* code);
 *     no C++ exception crosses this boundary.  On failure the call has no
 *     effect on the handle's state, and lbfast_last_error() returns a
 *     message for the calling thread.
 *   - Arguments are validated on the host before any device work.
 *   - A handle is bound to one HIP device (the current device at create) and
 *     one HIP stream; work is enqueued asynchronously on that stream.  A
 *     handle is not thread-safe.  Device faults surface at the next
 *     synchronising call (get_*, reduce, sync) as LBF_E_DEVICE.
 *   - Host arrays are copied in/out and never retained.  Device arrays passed
 *     as "borrowed" must stay alive (and unmodified by others while a call
 *     that reads them is in flight) until the handle is destroyed or the
 *     array is replaced.
 */
#ifndef LBFAST_H_
#define LBFAST_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBFAST_ABI_VERSION 1

typedef struct lbfast_ctx* lbfast_t; /* opaque handle */

/* status codes */
enum {
  LBF_OK = 0,
  LBF_E_ARG = -1,         /* invalid argument (bad size, null pointer, tau<=1/2 ...) */
  LBF_E_UNSUPPORTED = -2, /* valid request that this build does not implement */
  LBF_E_NOMEM = -3,       /* device or host allocation failed */
  LBF_E_DEVICE = -4,      /* HIP runtime error or kernel fault */
  LBF_E_NONFINITE = -5,   /* a reduction found NaN/Inf in the state */
  LBF_E_STATE = -6        /* call not valid in the handle's current state */
};

/* velocity sets (section 2, the paragraph after Eq. (9)).  LBF_D3Q19 and
 * LBF_D3Q27: Hermite series truncated at second order.  LBF_D3Q27H: the D3Q27
 * set with the series over its complete Hermite basis (orders up to 6), the
 * coefficients of order >= 3 rebuilt every step from u and a2 - u u by the
 * recursive closures the paper cites (Shan et al. for the equilibrium,
 * Malaspinas for the non-equilibrium part); the stored fields, the projection
 * and the correction are those of the other sets.  Its value is a code, not
 * a velocity count.  The adjoint covers LBF_D3Q19 and LBF_D3Q27 only. */
enum { LBF_D3Q19 = 19, LBF_D3Q27 = 27, LBF_D3Q27H = 270 };

/* element types: storage of the moment planes, and dtype of user arrays.
 * F16S/BF16S = 16-bit storage of v/s_m with a power-of-two scale s_m per
 * moment plane, arithmetic in FP32 (only valid as `storage`).  In 16-bit
 * storage the second-order planes hold the deviation a2 - u u (u as stored),
 * p* and u are deviations already; the ABI always exchanges the total a2.
 * lbfast_set_moments rounds to nearest even; the step rounds as
 * lbfast_params.rounding says.
 * F16SU = F16S with each velocity component split over two binary16 words,
 * u = s_u (hi + 2^-11 lo), hi the rounding of u/s_u and lo that of the
 * remainder (both to nearest even): 22 significant bits for u, which carries
 * almost all of the 16-bit storage error of a slowly evolving flow.  A state
 * then holds 13 planes of N binary16 words: the ten moment planes (planes
 * 1..3 the hi words), then the lo words of u_x, u_y, u_z.  All three
 * velocity sets, one component, rounding to nearest only.
 * Layout of a 16-bit state (what lbfast_state_ptr points to): planes 4j ..
 * 4j + 3 share the 8 N bytes at offset 8 j N, interleaved by site: the 64-bit
 * word at offset 8 (j N + i) holds the four values of site i, plane 4j in its
 * lowest 16 bits.  Two planes left over (8 and 9 of F16S and BF16S) share the
 * 4 N bytes after the groups the same way, one 32-bit word per site, the lower
 * plane in its low half; a last single plane (12 of F16SU) is N plain
 * binary16 words at offset 2 (12 N).  FP32 and FP64 states are plane after
 * plane: plane k of site i at element k N + i. */
enum { LBF_F64 = 0, LBF_F32 = 1, LBF_F16S = 2, LBF_BF16S = 3, LBF_F16SU = 4 };

/* boundary per axis: periodic, or stationary halfway bounce-back walls at
 * both ends (walls at -1/2 and n-1/2; every layer is fluid).  Walls are
 * supported on the y axis only. */
enum { LBF_PERIODIC = 0, LBF_WALLS = 1 };

typedef struct lbfast_params {
  uint32_t struct_size; /* = sizeof(lbfast_params) */
  int32_t lattice;      /* LBF_D3Q19, LBF_D3Q27 or LBF_D3Q27H */
  int32_t storage;      /* LBF_F64, LBF_F32, LBF_F16S, LBF_BF16S, LBF_F16SU */
  int32_t bc[3];        /* per axis x, y, z: LBF_PERIODIC or LBF_WALLS */
  int64_t nx, ny, nz;   /* grid, each >= 1 (>= 2 on a walled axis) */
  double tau;           /* relaxation time, > 1/2 */
  double force[3];      /* uniform body force per unit volume (rho = 1);
                           ignored while a force field is set */
  float scale[10];      /* 16-bit storage only: power-of-two scale per moment
                           plane; 0 = choose at the first set_moments as the
                           power of two that maps M just below 2^10, with M
                           max|u| over the three velocity planes for each of
                           them, max(|a2|, max|u|^2) over the six second-order
                           planes for each of them, and max(|p*|, 3 max|u|^2)
                           for p* (so that a plane that starts at zero, like
                           p* of a solenoidal field, still gets a scale of its
                           group's magnitude).  The scales then stay fixed:
                           FP16 storage overflows once a plane grows beyond
                           64 times its magnitude at that set_moments (a
                           channel driven from noise or from rest, a flow
                           spun up by a force), which lbfast_reduce reports
                           as LBF_E_NONFINITE; pass scales sized for the
                           largest expected values in such runs, and for a
                           state at rest, which has no magnitude to go by */
  int32_t rounding;     /* 16-bit storage only: how the step rounds p* and u,
                           LBF_ROUND_AUTO (0: to nearest for F16S, stochastic
                           for BF16S, whose 8-bit significand drops nearly
                           every per-step change of a slowly evolving flow),
                           LBF_ROUND_NEAREST (1, to nearest even) or
                           LBF_ROUND_STOCHASTIC (2: uniform bits from a hash
                           of the site index and a seed drawn from the step
                           count since create, so that changes below half a
                           unit in the last place survive on average instead
                           of being dropped at every step: slowly evolving
                           flows do not stall, at the price of rounding noise);
                           a2 - u u always rounds to nearest.  Runs are
                           reproducible bit for bit from the same create; a
                           restart into a new handle draws other bits */
  int32_t reserved[7];  /* must be zero */
} lbfast_params;

enum { LBF_ROUND_AUTO = 0, LBF_ROUND_NEAREST = 1, LBF_ROUND_STOCHASTIC = 2 };

/* ABI version of the loaded library (LBFAST_ABI_VERSION at build time). */
int lbfast_abi_version(void);

/* Bytes of one moment buffer (10 planes x N x element size), 0 on invalid
 * params.  The memory model of section 3: M = N * n_fields * b. */
size_t lbfast_buffer_bytes(const lbfast_params* p);

/* Create a solver for the problem the paper states in section 2: a lattice
 * of nx x ny x nz sites, a velocity set, the relaxation time of the
 * collision (Eq. (3), nu = cs^2 (tau - 1/2)) and a body force (Eq. (9)),
 * with the two ten-field flip/flop state buffers of section 3
 * ("Implementation").  `stream` is a hipStream_t (NULL = legacy default stream).
 * buf0/buf1: two device buffers of lbfast_buffer_bytes(p) bytes, 256-byte
 * aligned, borrowed (caller frees after destroy); pass both NULL to have the
 * library allocate and own them.  The state is zero (rest) after create. */
int lbfast_create(const lbfast_params* p, void* stream, void* buf0, void* buf1,
                  lbfast_t* out);
int lbfast_destroy(lbfast_t h);

/* Copy a moment array (10 x N, dtype LBF_F64 or LBF_F32, physical values):
 * the Hermite coefficients p*, u, a2 of Eq. (6) that section 3 stores per
 * site, as reported after the correction of Eq. (8), into / out of the
 * current state.  on_device: 1 = device pointer, 0 = host.
 * set converts to the storage type (round to nearest even); get converts
 * from it.  get synchronises the stream. */
int lbfast_set_moments(lbfast_t h, const void* m, int dtype, int on_device);
int lbfast_get_moments(lbfast_t h, void* m, int dtype, int on_device);

/* Per-site body force (3 x N device array, borrowed, static in time), the
 * F^b term of the force split in section 2.  dtype must be the compute
 * type: LBF_F64 for F64 storage, LBF_F32 otherwise.  NULL reverts to the
 * uniform params.force. */
int lbfast_set_force_field(lbfast_t h, const void* F_dev, int dtype);

/* Advance n >= 0 fused steps (Eq. (7) then Eq. (8)), asynchronously. */
int lbfast_step(lbfast_t h, int64_t n);

/* Wait for the handle's stream; reports device errors. */
int lbfast_sync(lbfast_t h);

/* Deterministic FP64 sums over the current state (synchronising):
 * out = [sum a0, sum a1x, sum a1y, sum a1z, 1/2 sum |a1|^2]: the totals the
 * step conserves (the zeroth and first Hermite coefficients, Eqs. (5) and
 * (8): sum p* exactly, sum u up to the applied force) and the kinetic energy
 * whose decay the Taylor-Green validation of section 4 fits.
 * Returns LBF_E_NONFINITE (out still written) if any sum is NaN/Inf. */
int lbfast_reduce(lbfast_t h, double out[5]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sums of
 * lbfast_reduce over any moment array, with no handle and no allocation.
 *   state_dev  10 x n_sites values in the storage format and layout of
 *              `storage` (LBF_F64, LBF_F32, LBF_F16S, LBF_BF16S; 13 x n_sites
 *              for LBF_F16SU), device memory, e.g. lbfast_state_ptr() or a
 *              checkpoint slot; read only;
 *   scale      the ten 16-bit storage scales (lbfast_get_scales), host array;
 *              required for 16-bit storage, ignored (may be NULL) otherwise;
 *   out_dev    5 doubles of device memory, receives
 *              [sum a0, sum a1x, sum a1y, sum a1z, 1/2 sum |a1|^2];
 *   stream     hipStream_t of the current device (NULL = legacy stream).
 * Asynchronous: the result is in out_dev once the stream reaches it; no
 * synchronisation and no non-finite check (the caller inspects out_dev).
 * The per-block partial sums live in a fixed 40 KiB device array of the
 * library, one per GPU, held until the process ends; calls that overlap on one
 * GPU (different streams or threads) race on it and must be serialised by the
 * caller.  n_sites above 4e9 (the largest grid lbfast_create accepts) is
 * rejected with LBF_E_ARG, as are NULL, misaligned or host pointers. */
int lbfast_reduce_noalloc(const void* state_dev, int storage, int64_t n_sites,
                          const float scale[10], double* out_dev, void* stream);

/* Device pointer to the buffer holding the current state (flips every
 * step), for zero-copy reads; valid until the next step/destroy. */
int lbfast_state_ptr(lbfast_t h, void** dev_ptr);

/* The 16-bit storage scales in use (10 floats); 1.0 for FP32/FP64. */
int lbfast_get_scales(lbfast_t h, float out[10]);

/* Launch shape: rows per tile (4, 6, 8 or 14 -- at most 8 with two sites
 * per lane or with LBF_D3Q27H; LBF_E_UNSUPPORTED if the tile's LDS would
 * exceed 160 KiB) and z-planes per workgroup (>= 1); 0 keeps
 * the current value.  The default z-planes per workgroup follow the grid: at
 * most ~512 workgroups (~1024 for F64 with two sites per lane) in chunks of
 * >= 64 planes, or, where that leaves fewer than 128 workgroups, enough
 * workgroups in chunks of >= 8 planes; a z_chunk set here replaces that rule.
 * Every shape computes the same formulas per site; the
 * tile heights are separately compiled, so results may differ between shapes
 * in the last bits (floating-point contraction), while one shape is bitwise
 * reproducible from run to run. */
int lbfast_set_launch(lbfast_t h, int tile_rows, int z_chunk);

/* Consecutive x-sites per lane: 1 (64-wide tiles), 2 (128-wide tiles, one
 * 2-wide load or store per moment plane; needs an even nx and tiles of at
 * most 8 rows) or 3 (192-wide tiles, 3-wide accesses; F32 storage, LBF_D3Q19
 * or LBF_D3Q27, one component, nx divisible by 3, tiles of at most 8 rows;
 * enabling the two-component variant returns to one site per lane, as it
 * does from two with variable density or viscosity).  The default is 2 where
 * nx is even and at least 128 and the 128-wide tiles leave no more of the
 * last tile empty than 64-wide ones, else 3 where nx is divisible by 3 and
 * at least 192 and 192-wide tiles leave no more empty (F32, LBF_D3Q19 or
 * LBF_D3Q27), else 1; always 1 for LBF_D3Q27H with F64 storage, where two
 * sites spill registers.  If the
 * current tile height does not fit the 160 KiB of LDS with the new setting,
 * the tallest of 8, 6 and 4 rows that does is taken.  Same formulas per site;
 * results may differ between settings in the last bits. */
int lbfast_set_lane_sites(lbfast_t h, int sites);

/* Order in which the workgroups of the marching kernels (step, checkpointed
 * forward pass, adjoint) are handed to the GPU's 8 XCDs (each with its own
 * L2), for the calls that follow: 0 = automatic (contiguous
 * tile ranges per XCD for F64 storage and for F32 with LBF_D3Q27 and
 * LBF_D3Q27H, the hardware's order otherwise, as measured at 512^3),
 * 1 = the hardware's order (consecutive workgroups on the XCDs in turn),
 * 2 = a contiguous range of tiles per XCD.  A launch choice only: every
 * order computes bitwise the same results.  LBF_E_ARG for other values. */
int lbfast_set_block_order(lbfast_t h, int order);

/* Two-component variant (section 2): a phase field phi in [0, 1] (1: heavy
 * phase) transported by the conservative Allen-Cahn equation, Eq. (2),
 * advanced by forward-time centred-space differences with the D3Q27-weighted
 * derivative stencils of section 2.  Density and viscosity are blended
 * linearly in phi, rho = rho_l + phi (rho_h - rho_l), nu = nu_l + phi
 * (nu_h - nu_l), nu_k = (tau_k - 1/2)/3, so the relaxation rate is per site
 * (params.tau is not used in this mode).  The force is
 *   F = mu grad(phi) + rho g - p* cs^2 grad(rho)
 *       - (nu omega / cs^2)(a2 - u u) . grad(rho),
 * mu = 4 beta phi (phi - 1)(phi - 1/2) - kappa lap(phi), beta = 12 sigma/W,
 * kappa = 3 sigma W / 2, g = params.force read as a body acceleration (the
 * same as a force per unit volume where rho = 1); the last two terms vanish
 * at equal densities.  Walls: y only, with mirror images for the phase-field
 * stencils.  No per-site force field in this mode.  Each lbfast_step then
 * performs, in order: phi(t+1) from phi(t) and u(t); the fused step with
 * F(t)/rho(t) and omega(t) at the sources and F(t+1)/rho(t+1) in the
 * correction of Eq. (8), where each destination computes F(t+1) itself from
 * phi(t+1) (its pressure and viscous terms from p*, u, a2 of the site at t)
 * and keeps it as the next step's F(t).  FTCS is stable for diffusivity < ~0.34 with these
 * stencils (not checked). */
typedef struct lbfast_phase_params {
  uint32_t struct_size; /* = sizeof(lbfast_phase_params) */
  int32_t reserved0;    /* must be zero */
  double sigma;         /* surface tension, >= 0 */
  double width;         /* interface thickness W, > 0 */
  double diffusivity;   /* D of Eq. (2), >= 0; lambda = 4 D / W */
  double rho_l, rho_h;  /* phase densities (light, heavy), > 0 */
  double tau_l, tau_h;  /* phase relaxation times, > 1/2 */
} lbfast_phase_params;

/* Switch the handle to the two-component variant.  The library allocates
 * (and frees at destroy) 8 x N values of the compute type: phi and F (three
 * planes) for two time levels.  phi starts at 0. */
int lbfast_enable_two_phase(lbfast_t h, const lbfast_phase_params* pp);
/* Copy the phase field (N values, dtype LBF_F64 or LBF_F32, host or device)
 * in or out.  set also computes the force of the current time level, from
 * phi and (density contrast) the current moments: set the moments first. */
int lbfast_set_phase(lbfast_t h, const void* phi, int dtype, int on_device);
int lbfast_get_phase(lbfast_t h, void* phi, int dtype, int on_device);

/* Discrete adjoint (the paper does not treat differentiation; this is the
 * exact reverse mode of the discrete step of Eqs. (7)-(9) as implemented by
 * lbfast_step, for F64 and F32 storage and the lattices LBF_D3Q19 and
 * LBF_D3Q27; LBF_E_UNSUPPORTED for 16-bit storage and for LBF_D3Q27H).
 * The objective J is any function of the final state m(T); the caller gives
 * lambda_T = dJ/dm(T) and receives dJ/dF (gradient with respect to the
 * per-site force field, static in time) and optionally dJ/dm(0).  Gradients
 * with respect to the second-order planes are taken per stored component
 * (an off-diagonal plane stands for both symmetric entries).
 *
 * Checkpointing: lbfast_forward_checkpointed advances the state by nsteps,
 * saving the state at t = 0, k, 2k, ... (k = every) into ckpt_dev, which
 * holds ceil(nsteps/k) buffers of lbfast_buffer_bytes(p) bytes (device,
 * caller-owned, 256-byte aligned).  lbfast_adjoint then walks the segments
 * backwards: each is recomputed from its checkpoint into work_dev (k + 2
 * buffers of lbfast_buffer_bytes(p): the recomputed states and two adjoint
 * buffers; see lbfast_adjoint_work_bytes) and swept with one adjoint step
 * per time step.  A segment's end state is the next checkpoint and is not
 * recomputed, except in the last segment (the final state).  With every = 1 every state but the final one is a
 * checkpoint: the forward steps write straight into their slots (no copies)
 * and the adjoint reads each step's two states from ckpt_dev, recomputing
 * only the last step; the backward pass then costs one adjoint step per time
 * step, for nsteps buffers of checkpoint memory (500 steps of a 192^3 FP32
 * lattice: 142 GB).  The force (field or uniform), tau, lattice and
 * boundaries in use must be those of the forward run.
 *
 * Arrays (device, compute type: double for F64, float for F32 storage):
 *   lambda_T_dev  10 x N, read only;
 *   gF_dev        3 x N, overwritten with dJ/dF;
 *   lambda0_dev   10 x N, overwritten with dJ/dm(0), or NULL.
 * Both calls are asynchronous on the handle's stream; the handle's own
 * state is left at m(T).  nsteps = 0 gives gF = 0 and lambda0 = lambda_T. */
int lbfast_forward_checkpointed(lbfast_t h, int64_t nsteps, int64_t every, void* ckpt_dev);
/* Launch shape of the adjoint step: x-sites per lane (0 = automatic, 1, or 2
 * or 3 for F32 storage with nx divisible by it) and tile rows (0 = automatic,
 * 4, 6, 8 or 14; with two or three sites per lane 4 or 6, and 4 for
 * LBF_D3Q27).  Automatic: one site per lane, 8-row tiles (F64: 6).  Every
 * shape computes the same formulas; results may differ in the last bits. */
int lbfast_set_adjoint_launch(lbfast_t h, int sites, int tile_rows);
size_t lbfast_adjoint_work_bytes(lbfast_t h, int64_t every);
int lbfast_adjoint(lbfast_t h, int64_t nsteps, int64_t every, const void* ckpt_dev,
                   const void* lambda_T_dev, void* gF_dev, void* lambda0_dev, void* work_dev);

/* Message for the last failing call on this thread ("" if none). */
const char* lbfast_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBFAST_H_ */
