// phase.hip -- the phase field of the two-component variant (paper, section
// 2): the conservative Allen-Cahn equation, Eq. (2), advanced by
// forward-time centred-space differences, and the capillary force
// F^s = mu grad(phi), mu = 4 beta phi (phi - 1)(phi - 1/2) - kappa lap(phi),
// beta = 12 sigma / W, kappa = 3 sigma W / 2, plus rho(phi) g for a body
// acceleration g and, with density contrast, the pressure and viscous terms
// of the force split (rho, nu blended linearly in phi; the printed viscous
// term is garbled, this is -(nu omega / cs^2)(a2 - u u).grad(rho), the
// viscous stress written through the non-equilibrium coefficient of
// Eq. (6)).  Halfway walls in y take mirror images for the stencils, the
// flux normal to the wall reversed.
//
// Derivatives use the D3Q27-weighted stencils of section 2 (weights
// k_i / 216 with k = 64, 16, 4, 1 for |c|^2 = 0..3):
//   grad_a Psi = (1/cs^2) sum_i w_i c_ia Psi(x + c_i)   = (1/72) sum k_i c_ia Psi_i
//   lap Psi    = (2/cs^2) sum_{i!=0} w_i (Psi_i - Psi_0) = (1/36) sum k_i (Psi_i - Psi_0)
//   div V      = (1/cs^2) sum_i w_i c_i . V(x + c_i)
// (the printed Laplacian stencil is garbled; this is its Taylor-consistent
// reading, zero on constants).  Periodic grid.
//
// Two passes per step advance phi: the total flux V = phi u + lambda J (J the
// normalised compression flux) at every site, stored with phi as one 4-wide
// record, then phi' = phi - div(V) + D lap(phi).  A third pass gives the force
// from phi(t+1).  All three are z-marches over 64 x 8 column tiles that stage
// one plane (with halo) in LDS at a time and add each plane's contributions
// to the three destination planes it reaches, so a value is read from memory
// about once.  Algorithmic traffic at FP32: flux 32 B per lattice update
// (phi, u in; record out), update 20 B (record in; phi out), force 16 B (phi
// in, F out), against the fused step's 104.
#include "internal.hpp"
#include "lattice.hpp"

namespace lbf {
namespace {

constexpr int kPhaseThreads = 256;

// D3Q27 stencil weight numerators (w = k / 216) by |c|^2
__device__ constexpr int k27(int dx, int dy, int dz) {
  const int c2 = dx * dx + dy * dy + dz * dz;
  return c2 == 0 ? 64 : (c2 == 1 ? 16 : (c2 == 2 ? 4 : 1));
}

// per-site record of the update pass: the total phase flux
// V = phi u + lambda phi (1 - phi) grad(phi) / (|grad phi| + eps) (advection plus
// interface compression, so that Eq. (2) reads phi' = phi - div(V) + D lap(phi))
// and phi itself, interleaved so that a neighbour is one 4-wide load
template <typename C>
struct alignas(4 * sizeof(C)) Rec {
  C vx, vy, vz, phi;
};

// Output of the flux pass at one site, from phi and its derivatives: the
// record (V, phi) with u read from the state
template <int ST>
struct FluxEmit {
  using S = Storage<ST>;
  using C = typename S::C;
  const typename S::T* st;
  Rec<C>* V;
  int64_t N;
  C lambda, eps;
  float s1, s2, s3;
  __device__ __forceinline__ void operator()(int64_t s, C p, const C g[3], C) const {
    const C c = lambda * p * (C(1) - p) / (sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + eps);
    Rec<C> r;
    r.vx = p * S::load(st + N, s, s1) + c * g[0];
    r.vy = p * S::load(st + 2 * N, s, s2) + c * g[1];
    r.vz = p * S::load(st + 3 * N, s, s3) + c * g[2];
    r.phi = p;
    V[s] = r;
  }
};

// phi' = phi - div(V) + D lap(phi).  A workgroup owns a 64 x kUpdRows column
// tile and a chunk of z-planes and marches through z.  One plane of records
// (with a one-site halo) is staged in LDS at a time (double buffered, loaded
// one plane ahead into registers); every thread reads the 3 x 3 records
// around its column once and adds their contributions to the three
// destination planes they reach: p - 1 (complete after this plane, stored),
// p and p + 1 (rolling accumulators).  Each record is read from memory about
// once (plus halo) and from LDS nine times instead of 26.  The Laplacian's
// terms k (phi_n - phi_0) for destination p + 1 arrive before its phi_0: they
// are summed relative to the thread's own phi of plane p and corrected by the
// weight sum (36) times the difference once phi_0 is known, so FP32 adds only
// small differences.
constexpr int kUpdRows = 8;

template <typename C>
__global__ void __launch_bounds__(64 * kUpdRows) update_kernel(const Rec<C>* __restrict__ V,
                                                               C* __restrict__ out, int nx, int ny,
                                                               int nz, C D, int tiles_x,
                                                               int tiles_y, int zchunk,
                                                               bool walls_y) {
  constexpr int RY = kUpdRows + 2, RX = 66;
  constexpr int NT = 64 * kUpdRows;           // threads
  constexpr int NE = RY * RX;                 // staged records per plane
  constexpr int PER = (NE + NT - 1) / NT;     // staged records per thread
  constexpr int KZ = 16 + 4 * 4 + 4 * 1;      // sum of k over the 9 sites of an adjacent plane
  __shared__ Rec<C> t[2][RY][RX];
  const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
  int b = static_cast<int>(blockIdx.x);
  const int tx = b % tiles_x;
  b /= tiles_x;
  const int ty = b % tiles_y;
  const int zc = b / tiles_y;
  const int x0 = tx * 64, y0 = ty * kUpdRows;
  const int z0 = zc * zchunk, z1 = min(z0 + zchunk, nz);
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  // this thread's staged records: in-plane offset, LDS position, and whether
  // it is the mirror image beyond a y wall (flux normal to the wall reversed)
  int64_t off[PER];
  int pos[PER];
  bool act[PER], ghost[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + k * NT;
    act[k] = e < NE;
    const int ry = act[k] ? e / RX : 0, rx = act[k] ? e - ry * RX : 0;
    const int xw = pmod(x0 + rx - 1, nx), yr = y0 + ry - 1;
    ghost[k] = walls_y && (yr < 0 || yr >= ny);
    const int yw = walls_y ? clampi(yr, 0, ny - 1) : pmod(yr, ny);
    off[k] = static_cast<int64_t>(yw) * nx + xw;
    pos[k] = ry * RX + rx;
  }
  Rec<C> r[PER];
  auto fetch = [&](int z) {
    const int64_t zb = static_cast<int64_t>(wrap(z, nz)) * plane;
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (act[k]) r[k] = V[zb + off[k]];
  };
  auto put = [&](int z) {
    Rec<C>* dst = &t[z & 1][0][0];
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (act[k]) {
        Rec<C> v = r[k];
        if (ghost[k]) v.vy = -v.vy;
        dst[pos[k]] = v;
      }
  };
  const int x = x0 + lane, y = y0 + wy;
  const bool mine = x < nx && y < ny;
  // destination p - 1: divergence and Laplacian sums and its phi_0; p: the
  // same, with the Laplacian part from plane p - 1 relative to ref0; p + 1
  // is started afresh from each plane
  C dvm = 0, lm = 0, pm = 0;
  C dv0 = 0, l0 = 0, ref0 = 0;
  fetch(z0 - 1);
  for (int p = z0 - 1; p <= z1; ++p) {
    put(p);  // plane p (fetched one iteration ahead)
    __syncthreads();
    if (p < z1) fetch(p + 1);  // in flight while plane p is summed
    Rec<C> q[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) q[dy][dx] = t[p & 1][wy + dy][lane + dx];
    const C own = q[1][1].phi;
    C dvu = 0, lu = 0, dvc = 0, lc = 0, dvd = 0, ld = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const Rec<C>& n = q[dy + 1][dx + 1];
        C cv = 0;
        if (dx) cv += C(dx) * n.vx;
        if (dy) cv += C(dy) * n.vy;
        // seen from destination p + 1 this site is at dz = -1, from p - 1 at
        // dz = +1, from p at dz = 0
        const C ku = C(k27(dx, dy, 1));
        dvu += ku * (cv - n.vz);
        dvd += ku * (cv + n.vz);
        lu += ku * (n.phi - own);
        ld += ku * (n.phi - pm);
        if (dx || dy) {
          const C kc = C(k27(dx, dy, 0));
          dvc += kc * cv;
          lc += kc * (n.phi - own);
        }
      }
    // destination p - 1 is complete
    if (mine && p - 1 >= z0 && p - 1 < z1)
      out[static_cast<int64_t>(p - 1) * plane + static_cast<int64_t>(y) * nx + x] =
          pm - div_by<72>(dvm + dvd) + D * div_by<36>(lm + ld);
    // destination p: the part from p - 1, corrected to phi_0 = own
    dvm = dv0 + dvc;
    lm = l0 - C(KZ) * (own - ref0) + lc;
    pm = own;
    // destination p + 1, relative to own
    dv0 = dvu;
    l0 = lu;
    ref0 = own;
  }
}

// Output of the force pass at one site: F = mu grad(phi) + rho(phi) g, plus
// (contrast) the pressure and viscous terms - p* cs^2 grad(rho)
// - (nu omega / cs^2) (a2 - u u) . grad(rho), with p*, u, a2 of the state at
// the previous time level
template <int ST, bool CONTRAST>
struct ForceEmit {
  using S = Storage<ST>;
  using C = typename S::C;
  const typename S::T* st;
  C* F;
  int64_t N;
  PhaseArgs pa;
  __device__ __forceinline__ void operator()(int64_t s, C p, const C g[3], C l) const {
    const C beta = static_cast<C>(pa.beta), kappa = static_cast<C>(pa.kappa);
    const C rl = static_cast<C>(pa.rho_l), dr = static_cast<C>(pa.rho_h - pa.rho_l);
    const C mu = C(4) * beta * p * (p - C(1)) * (p - C(0.5)) - kappa * l;
    const C rho = rl + p * dr;
    C f[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] = mu * g[k] + rho * static_cast<C>(pa.Fb[k]);
    if constexpr (CONTRAST) {
      const C nl = static_cast<C>(pa.nu_l), dn = static_cast<C>(pa.nu_h - pa.nu_l);
      C m[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) m[k] = S::load(st + k * N, s, pa.scale[k]);
      // the non-equilibrium part a2 - u u (16-bit storage keeps it directly)
      if constexpr (!S::kNeq) {
#pragma unroll
        for (int k = 4; k < 10; ++k) m[k] -= m[1 + a2_a(k)] * m[1 + a2_b(k)];
      }
      const C nu = nl + p * dn;
      const C omega = C(1) / (C(3) * nu + C(0.5));
      const C gr[3] = {dr * g[0], dr * g[1], dr * g[2]};
      const C cv = C(3) * nu * omega;  // nu omega / cs^2
      const C cp = m[0] * C(1.0 / 3.0);
      // (a2 - u u) . grad(rho), rows xx xy xz / xy yy yz / xz yz zz
      f[0] += -cp * gr[0] - cv * (m[4] * gr[0] + m[7] * gr[1] + m[8] * gr[2]);
      f[1] += -cp * gr[1] - cv * (m[7] * gr[0] + m[5] * gr[1] + m[9] * gr[2]);
      f[2] += -cp * gr[2] - cv * (m[8] * gr[0] + m[9] * gr[1] + m[6] * gr[2]);
    }
    F[s] = f[0];
    F[N + s] = f[1];
    F[2 * N + s] = f[2];
  }
};

// grad(phi) and lap(phi) at every site, handed to an output functor: the
// same tiles, z-march, staging and 2.5-D accumulation as the update pass, on
// the scalar phi (a y wall's ghost is the mirror value)
template <typename C, class Emit>
__global__ void __launch_bounds__(64 * kUpdRows) grad_march_kernel(const C* __restrict__ phi,
                                                                   int nx, int ny, int nz,
                                                                   int tiles_x, int tiles_y,
                                                                   int zchunk, bool walls_y,
                                                                   Emit emit) {
  constexpr int RY = kUpdRows + 2, RX = 66;
  constexpr int NT = 64 * kUpdRows;
  constexpr int NE = RY * RX;
  constexpr int PER = (NE + NT - 1) / NT;
  constexpr int KZ = 16 + 4 * 4 + 4 * 1;  // sum of k over the 9 sites of an adjacent plane
  __shared__ C t[2][RY][RX];
  const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
  int b = static_cast<int>(blockIdx.x);
  const int tx = b % tiles_x;
  b /= tiles_x;
  const int ty = b % tiles_y;
  const int zc = b / tiles_y;
  const int x0 = tx * 64, y0 = ty * kUpdRows;
  const int z0 = zc * zchunk, z1 = min(z0 + zchunk, nz);
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  int64_t off[PER];
  int pos[PER];
  bool act[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + k * NT;
    act[k] = e < NE;
    const int ry = act[k] ? e / RX : 0, rx = act[k] ? e - ry * RX : 0;
    const int xw = pmod(x0 + rx - 1, nx), yr = y0 + ry - 1;
    const int yw = walls_y ? clampi(yr, 0, ny - 1) : pmod(yr, ny);
    off[k] = static_cast<int64_t>(yw) * nx + xw;
    pos[k] = ry * RX + rx;
  }
  C r[PER];
  auto fetch = [&](int z) {
    const int64_t zb = static_cast<int64_t>(wrap(z, nz)) * plane;
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (act[k]) r[k] = phi[zb + off[k]];
  };
  auto put = [&](int z) {
    C* dst = &t[z & 1][0][0];
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (act[k]) dst[pos[k]] = r[k];
  };
  const int x = x0 + lane, y = y0 + wy;
  const bool mine = x < nx && y < ny;
  // destination p - 1 (sums and phi_0) and p (sums from plane p - 1, the
  // Laplacian relative to ref0), as in the update pass
  C gxm = 0, gym = 0, gzm = 0, lm = 0, pm = 0;
  C gx0 = 0, gy0 = 0, gz0 = 0, l0 = 0, ref0 = 0;
  fetch(z0 - 1);
  for (int p = z0 - 1; p <= z1; ++p) {
    put(p);
    __syncthreads();
    if (p < z1) fetch(p + 1);
    C q[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) q[dy][dx] = t[p & 1][wy + dy][lane + dx];
    const C own = q[1][1];
    // sums over this plane's 3 x 3 sites with the weights of an adjacent
    // plane (ku) and of the own plane (kc, centre excluded)
    C axu = 0, ayu = 0, azu = 0, lu = 0, ld = 0, axc = 0, ayc = 0, lc = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const C n = q[dy + 1][dx + 1];
        const C ku = C(k27(dx, dy, 1));
        if (dx) axu += C(dx) * ku * n;
        if (dy) ayu += C(dy) * ku * n;
        azu += ku * n;
        lu += ku * (n - own);
        ld += ku * (n - pm);
        if (dx || dy) {
          const C kc = C(k27(dx, dy, 0));
          if (dx) axc += C(dx) * kc * n;
          if (dy) ayc += C(dy) * kc * n;
          lc += kc * (n - own);
        }
      }
    // destination p - 1 is complete: this plane is at dz = +1 from it
    if (mine && p - 1 >= z0 && p - 1 < z1) {
      const C g[3] = {div_by<72>(gxm + axu), div_by<72>(gym + ayu), div_by<72>(gzm + azu)};
      emit(static_cast<int64_t>(p - 1) * plane + static_cast<int64_t>(y) * nx + x, pm, g,
           div_by<36>(lm + ld));
    }
    // destination p: plane p - 1 (at dz = -1) plus this plane
    gxm = gx0 + axc;
    gym = gy0 + ayc;
    gzm = gz0;
    lm = l0 - C(KZ) * (own - ref0) + lc;
    pm = own;
    // destination p + 1: this plane at dz = -1
    gx0 = axu;
    gy0 = ayu;
    gz0 = -azu;
    l0 = lu;
    ref0 = own;
  }
}

// tiles and z-chunks of the staged passes: 64 x kUpdRows columns, chunks of
// >= 8 planes for about 512 workgroups
struct MarchGeom {
  int tiles_x, tiles_y, zchunk, blocks;
};
MarchGeom march_geom(int nx, int ny, int nz) {
  MarchGeom m;
  m.tiles_x = (nx + 63) / 64;
  m.tiles_y = (ny + kUpdRows - 1) / kUpdRows;
  const int cols = m.tiles_x * m.tiles_y;
  int nch = (512 + cols - 1) / cols;
  const int maxc = nz >= 8 ? nz / 8 : 1;
  nch = nch < 1 ? 1 : (nch > maxc ? maxc : nch);
  m.zchunk = (nz + nch - 1) / nch;
  m.blocks = cols * ((nz + m.zchunk - 1) / m.zchunk);
  return m;
}

int phase_grid(int64_t N) {
  const int64_t b = (N + kPhaseThreads - 1) / kPhaseThreads;
  return static_cast<int>(b < 16384 ? (b < 1 ? 1 : b) : 16384);
}

template <int ST>
hipError_t phase_step_st(const PhaseArgs& a, hipStream_t s) {
  using C = typename Storage<ST>::C;
  using T = typename Storage<ST>::T;
  const MarchGeom m = march_geom(a.nx, a.ny, a.nz);
  const FluxEmit<ST> flux{static_cast<const T*>(a.state), static_cast<Rec<C>*>(a.J), a.N,
                          static_cast<C>(a.lambda), static_cast<C>(a.eps), a.scale[1],
                          a.scale[2], a.scale[3]};
  hipLaunchKernelGGL((grad_march_kernel<C, FluxEmit<ST>>), dim3(m.blocks), dim3(64 * kUpdRows),
                     0, s, static_cast<const C*>(a.phi), a.nx, a.ny, a.nz, m.tiles_x, m.tiles_y,
                     m.zchunk, a.walls_y != 0, flux);
  hipLaunchKernelGGL((update_kernel<C>), dim3(m.blocks), dim3(64 * kUpdRows), 0, s,
                     static_cast<const Rec<C>*>(a.J), static_cast<C*>(a.phi_out), a.nx, a.ny,
                     a.nz, static_cast<C>(a.D), m.tiles_x, m.tiles_y, m.zchunk, a.walls_y != 0);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_phase_step(int storage, const PhaseArgs& a, hipStream_t s) {
  switch (storage) {
    case kF64: return phase_step_st<kF64>(a, s);
    case kF32: return phase_step_st<kF32>(a, s);
    case kF16S: return phase_step_st<kF16S>(a, s);
    case kBF16S: return phase_step_st<kBF16S>(a, s);
    default: return hipErrorInvalidValue;
  }
}

namespace {
template <int ST>
hipError_t force_st(const PhaseArgs& a, hipStream_t s) {
  using C = typename Storage<ST>::C;
  using T = typename Storage<ST>::T;
  const MarchGeom m = march_geom(a.nx, a.ny, a.nz);
  const C* phi = static_cast<const C*>(a.phi_out);
  const T* st = static_cast<const T*>(a.state);
  if (a.contrast)
    hipLaunchKernelGGL((grad_march_kernel<C, ForceEmit<ST, true>>), dim3(m.blocks),
                       dim3(64 * kUpdRows), 0, s, phi, a.nx, a.ny, a.nz, m.tiles_x, m.tiles_y,
                       m.zchunk, a.walls_y != 0,
                       ForceEmit<ST, true>{st, static_cast<C*>(a.F), a.N, a});
  else
    hipLaunchKernelGGL((grad_march_kernel<C, ForceEmit<ST, false>>), dim3(m.blocks),
                       dim3(64 * kUpdRows), 0, s, phi, a.nx, a.ny, a.nz, m.tiles_x, m.tiles_y,
                       m.zchunk, a.walls_y != 0,
                       ForceEmit<ST, false>{st, static_cast<C*>(a.F), a.N, a});
  return hipGetLastError();
}
}  // namespace

hipError_t launch_capillary_force(int storage, const PhaseArgs& a, hipStream_t s) {
  switch (storage) {
    case kF64: return force_st<kF64>(a, s);
    case kF32: return force_st<kF32>(a, s);
    case kF16S: return force_st<kF16S>(a, s);
    case kBF16S: return force_st<kBF16S>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbf

namespace lbf {
namespace {

template <typename From, typename To>
__global__ void convert_kernel(const From* __restrict__ src, To* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kPhaseThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kPhaseThreads)
    dst[i] = static_cast<To>(src[i]);
}

template <typename A, typename B>
hipError_t convert_t(const void* src, void* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((convert_kernel<A, B>), dim3(phase_grid(n)), dim3(kPhaseThreads), 0, s,
                     static_cast<const A*>(src), static_cast<B*>(dst), n);
  return hipGetLastError();
}

}  // namespace

// dst_is_user = 0: user (src_dtype) -> compute type of the storage;
// dst_is_user = 1: compute type -> user (src_dtype names the user type)
hipError_t launch_convert(int storage, int user_dtype, const void* src, int dst_is_user, void* dst,
                          int64_t n, hipStream_t s) {
  const bool c64 = storage == kF64, u64 = user_dtype == kF64;
  if (!dst_is_user) {
    if (c64) return u64 ? convert_t<double, double>(src, dst, n, s) : convert_t<float, double>(src, dst, n, s);
    return u64 ? convert_t<double, float>(src, dst, n, s) : convert_t<float, float>(src, dst, n, s);
  }
  if (c64) return u64 ? convert_t<double, double>(src, dst, n, s) : convert_t<double, float>(src, dst, n, s);
  return u64 ? convert_t<float, double>(src, dst, n, s) : convert_t<float, float>(src, dst, n, s);
}

}  // namespace lbf
