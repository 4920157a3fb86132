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
// record, then phi' = phi - div(V) + D lap(phi) by a z-march with the records
// staged in LDS.  The flux and force passes take one thread per site and read
// their 26 neighbours through the caches.  Algorithmic traffic at FP32: flux
// 32 B per lattice update (phi, u in; record out), update 20 B (record in;
// phi out), force 16 B (phi in, F out), against the fused step's 104.
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

// neighbour offsets of site (x, y, z): ox[d+1] etc.; periodic, or with
// halfway walls in y (walls_y) where the site beyond a wall is the mirror
// image of the one next to it
struct Nbr {
  int64_t ox[3], oy[3], oz[3];
  int64_t s;
};

__device__ __forceinline__ Nbr neighbours(int64_t s, int nx, int ny, int nz, bool walls_y) {
  Nbr n;
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  const int z = static_cast<int>(s / plane);
  const int64_t r = s - static_cast<int64_t>(z) * plane;
  const int y = static_cast<int>(r / nx);
  const int x = static_cast<int>(r - static_cast<int64_t>(y) * nx);
  for (int d = -1; d <= 1; ++d) {
    n.ox[d + 1] = wrap(x + d, nx);
    n.oy[d + 1] = static_cast<int64_t>(walls_y ? clampi(y + d, 0, ny - 1) : wrap(y + d, ny)) * nx;
    n.oz[d + 1] = static_cast<int64_t>(wrap(z + d, nz)) * plane;
  }
  n.s = s;
  return n;
}

__device__ __forceinline__ int64_t at(const Nbr& n, int dx, int dy, int dz) {
  return n.ox[dx + 1] + n.oy[dy + 1] + n.oz[dz + 1];
}

// grad and lap of a scalar field at one site
template <typename C>
__device__ __forceinline__ void grad_lap(const C* __restrict__ f, const Nbr& n, C g[3], C& lap) {
  const C f0 = f[n.s];
  C gx = 0, gy = 0, gz = 0, l = 0;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        const C v = f[at(n, dx, dy, dz)];
        const C k = C(k27(dx, dy, dz));
        gx += C(dx) * k * v;
        gy += C(dy) * k * v;
        gz += C(dz) * k * v;
        l += k * (v - f0);
      }
  g[0] = div_by<72>(gx);
  g[1] = div_by<72>(gy);
  g[2] = div_by<72>(gz);
  lap = div_by<36>(l);
}

// per-site record of the update pass: the total phase flux
// V = phi u + lambda phi (1 - phi) grad(phi) / (|grad phi| + eps) (advection plus
// interface compression, so that Eq. (2) reads phi' = phi - div(V) + D lap(phi))
// and phi itself, interleaved so that a neighbour is one 4-wide load
template <typename C>
struct alignas(4 * sizeof(C)) Rec {
  C vx, vy, vz, phi;
};

template <int ST>
__global__ void __launch_bounds__(kPhaseThreads) flux_kernel(
    const typename Storage<ST>::C* __restrict__ phi, const typename Storage<ST>::T* __restrict__ st,
    Rec<typename Storage<ST>::C>* __restrict__ V, int nx, int ny, int nz, int64_t N,
    typename Storage<ST>::C lambda, typename Storage<ST>::C eps, float s1, float s2, float s3,
    bool walls_y) {
  using S = Storage<ST>;
  using C = typename S::C;
  for (int64_t s = blockIdx.x * static_cast<int64_t>(kPhaseThreads) + threadIdx.x; s < N;
       s += static_cast<int64_t>(gridDim.x) * kPhaseThreads) {
    const Nbr n = neighbours(s, nx, ny, nz, walls_y);
    C g[3], l;
    grad_lap(phi, n, g, l);
    const C p = phi[s];
    const C c = lambda * p * (C(1) - p) / (sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + eps);
    Rec<C> r;
    r.vx = p * S::load(st + N, s, s1) + c * g[0];
    r.vy = p * S::load(st + 2 * N, s, s2) + c * g[1];
    r.vz = p * S::load(st + 3 * N, s, s3) + c * g[2];
    r.phi = p;
    V[s] = r;
  }
}

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

// F = mu grad(phi) + rho(phi) g, plus (contrast) the pressure and viscous
// terms - p* cs^2 grad(rho) - (nu omega / cs^2) (a2 - u u) . grad(rho), with
// p*, u, a2 of the state at the previous time level
template <int ST, bool CONTRAST>
__global__ void __launch_bounds__(kPhaseThreads) force_kernel(
    const typename Storage<ST>::C* __restrict__ phi, const typename Storage<ST>::T* __restrict__ st,
    typename Storage<ST>::C* __restrict__ F, int nx, int ny, int nz, int64_t N, PhaseArgs pa) {
  using S = Storage<ST>;
  using C = typename S::C;
  const C beta = static_cast<C>(pa.beta), kappa = static_cast<C>(pa.kappa);
  const C rl = static_cast<C>(pa.rho_l), dr = static_cast<C>(pa.rho_h - pa.rho_l);
  const C nl = static_cast<C>(pa.nu_l), dn = static_cast<C>(pa.nu_h - pa.nu_l);
  for (int64_t s = blockIdx.x * static_cast<int64_t>(kPhaseThreads) + threadIdx.x; s < N;
       s += static_cast<int64_t>(gridDim.x) * kPhaseThreads) {
    const Nbr n = neighbours(s, nx, ny, nz, pa.walls_y != 0);
    C g[3], l;
    grad_lap(phi, n, g, l);
    const C p = phi[s];
    const C mu = C(4) * beta * p * (p - C(1)) * (p - C(0.5)) - kappa * l;
    const C rho = rl + p * dr;
    C f[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] = mu * g[k] + rho * static_cast<C>(pa.Fb[k]);
    if constexpr (CONTRAST) {
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
}

int phase_grid(int64_t N) {
  const int64_t b = (N + kPhaseThreads - 1) / kPhaseThreads;
  return static_cast<int>(b < 16384 ? (b < 1 ? 1 : b) : 16384);
}

template <int ST>
hipError_t phase_step_st(const PhaseArgs& a, hipStream_t s) {
  using C = typename Storage<ST>::C;
  using T = typename Storage<ST>::T;
  const dim3 grid(phase_grid(a.N)), block(kPhaseThreads);
  hipLaunchKernelGGL((flux_kernel<ST>), grid, block, 0, s, static_cast<const C*>(a.phi),
                     static_cast<const T*>(a.state), static_cast<Rec<C>*>(a.J), a.nx, a.ny, a.nz,
                     a.N, static_cast<C>(a.lambda), static_cast<C>(a.eps), a.scale[1], a.scale[2],
                     a.scale[3], a.walls_y != 0);
  // update: 64 x 8 column tiles, z-chunks of >= 8 planes for ~512 workgroups
  const int tiles_x = (a.nx + 63) / 64, tiles_y = (a.ny + kUpdRows - 1) / kUpdRows;
  const int cols = tiles_x * tiles_y;
  int nch = (512 + cols - 1) / cols;
  const int maxc = a.nz >= 8 ? a.nz / 8 : 1;
  nch = nch < 1 ? 1 : (nch > maxc ? maxc : nch);
  const int zchunk = (a.nz + nch - 1) / nch;
  const int zchunks = (a.nz + zchunk - 1) / zchunk;
  hipLaunchKernelGGL((update_kernel<C>), dim3(cols * zchunks), dim3(64 * kUpdRows), 0, s,
                     static_cast<const Rec<C>*>(a.J), static_cast<C*>(a.phi_out), a.nx, a.ny,
                     a.nz, static_cast<C>(a.D), tiles_x, tiles_y, zchunk, a.walls_y != 0);
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
  const dim3 grid(phase_grid(a.N)), block(kPhaseThreads);
  if (a.contrast)
    hipLaunchKernelGGL((force_kernel<ST, true>), grid, block, 0, s,
                       static_cast<const C*>(a.phi_out), static_cast<const T*>(a.state),
                       static_cast<C*>(a.F), a.nx, a.ny, a.nz, a.N, a);
  else
    hipLaunchKernelGGL((force_kernel<ST, false>), grid, block, 0, s,
                       static_cast<const C*>(a.phi_out), static_cast<const T*>(a.state),
                       static_cast<C*>(a.F), a.nx, a.ny, a.nz, a.N, a);
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
