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
// One z-march advances phi: it computes the total flux V = phi u + lambda J
// (J the normalised compression flux) on the fly, keeping the tile's records
// in LDS, and then phi' = phi - div(V) + D lap(phi).  A second march gives
// the force from phi(t+1).  Algorithmic traffic at FP32: the phase update
// 20 B per lattice update (phi, u in; phi out), the force 16 B (phi in, F
// out), against the fused step's 104.
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

// per-site record staged by the phase update: the total phase flux
// V = phi u + lambda phi (1 - phi) grad(phi) / (|grad phi| + eps) (advection plus
// interface compression, so that Eq. (2) reads phi' = phi - div(V) + D lap(phi))
// and phi itself, interleaved so that a neighbour is one 4-wide load
template <typename C>
struct alignas(4 * sizeof(C)) Rec {
  C vx, vy, vz, phi;
};

// The z-marches below use 64 x kUpdRows column tiles.  Each stages one plane
// (with halo) in LDS at a time and adds that plane's contributions to the
// three destination planes it reaches: p - 1 (complete after this plane),
// and p and p + 1 (rolling accumulators).  So each value is read from memory
// about once (plus halo) and from LDS nine times instead of 26.
//
// The Laplacian's terms k (phi_n - phi_0) for destination p + 1 arrive before
// its phi_0.  They are summed relative to the thread's own phi of plane p and
// corrected, once phi_0 is known, by the weight sum (36) times the
// difference, so FP32 adds only small differences.
constexpr int kUpdRows = 8;

// The whole phase update in one z-march: phi' = phi - div(V) + D lap(phi)
// with V = phi u + lambda phi (1 - phi) grad(phi) / (|grad phi| + eps), no
// record written to memory.  A workgroup owns a 64 x kUpdRows column tile;
// each iteration q stages phi plane q with a two-site halo (PY x PX).  Its
// gradient contributions complete V(q - 1) at the tile's sites and a
// one-site ring (VY x VX record slots, u read there), with the rolling sums
// of the gradient march.  Those records are staged at iteration q + 1, and
// their divergence and Laplacian sums complete phi'(q - 2).  One barrier
// per plane: phi(q) and V(q - 2) are written to the buffers of parity q & 1
// before it and read after it; the other parity was last read before it.
// A y wall's ghost slot computes the mirror site's record from the mirror
// site's window and reverses v_y, so a ghost and its mirror hold the same
// numbers and the flux through the wall cancels exactly.
template <int ST>
__global__ void __launch_bounds__(64 * kUpdRows) phase_kernel(
    const typename Storage<ST>::C* __restrict__ phi, const typename Storage<ST>::T* __restrict__ st,
    typename Storage<ST>::C* __restrict__ out, int nx, int ny, int nz, int64_t N,
    typename Storage<ST>::C D, typename Storage<ST>::C lambda, typename Storage<ST>::C eps,
    float s1, float s2, float s3, int tiles_x, int tiles_y, int zchunk, bool walls_y) {
  using S = Storage<ST>;
  using C = typename S::C;
  constexpr int PY = kUpdRows + 4, PX = 68;  // phi plane, two-site halo
  constexpr int VY = kUpdRows + 2, VX = 66;  // record slots, one-site ring
  constexpr int NT = 64 * kUpdRows;
  constexpr int NP = PY * PX, NV = VY * VX;
  constexpr int PERP = (NP + NT - 1) / NT, PERV = (NV + NT - 1) / NT;
  constexpr int KZ = 16 + 4 * 4 + 4 * 1;  // sum of k over the 9 sites of an adjacent plane
  __shared__ C tp[2][NP];
  __shared__ Rec<C> tv[2][NV];
  const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
  int b = static_cast<int>(blockIdx.x);
  const int tx = b % tiles_x;
  b /= tiles_x;
  const int ty = b % tiles_y;
  const int zc = b / tiles_y;
  const int x0 = tx * 64, y0 = ty * kUpdRows;
  const int z0 = zc * zchunk, z1 = min(z0 + zchunk, nz);
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  // staged phi values: in-plane offset (a wall's ghost rows hold the clamped
  // row, which is the mirror image one site beyond the wall; rows further out
  // feed only slots that are never read for an owned site)
  int64_t poff[PERP];
  bool pact[PERP];
#pragma unroll
  for (int k = 0; k < PERP; ++k) {
    const int e = threadIdx.x + k * NT;
    pact[k] = e < NP;
    const int ry = pact[k] ? e / PX : 0, rx = pact[k] ? e - ry * PX : 0;
    const int yr = y0 + ry - 2;
    const int yw = walls_y ? clampi(yr, 0, ny - 1) : pmod(yr, ny);
    poff[k] = static_cast<int64_t>(yw) * nx + pmod(x0 + rx - 2, nx);
  }
  // record slots: the source site (the mirror site for a ghost), the top-left
  // of its 3 x 3 phi window in the staged plane, and whether v_y is reversed.
  // Rows: the source row ys lies in [y0 - 1, y0 + kUpdRows], so the window
  // rows ys - y0 + 1 .. ys - y0 + 3 lie in [0, PY).
  int64_t voff[PERV];
  int vwin[PERV];
  bool vact[PERV], vneg[PERV];
#pragma unroll
  for (int k = 0; k < PERV; ++k) {
    const int e = threadIdx.x + k * NT;
    vact[k] = e < NV;
    const int ry = vact[k] ? e / VX : 0, rx = vact[k] ? e - ry * VX : 0;
    const int yr = y0 + ry - 1;
    const int ys = walls_y ? clampi(yr, 0, ny - 1) : pmod(yr, ny);
    vneg[k] = walls_y && ys != yr;
    vwin[k] = (walls_y ? ys - y0 + 1 : ry) * PX + rx;
    voff[k] = static_cast<int64_t>(ys) * nx + pmod(x0 + rx - 1, nx);
  }
  // phi and u are loaded two planes ahead into two register sets; the set of
  // plane z is (z - z0) & 1, a compile-time index in the loop body below
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  C rp[2][PERP];
  auto fetch_phi = [&](auto P, int z) {
    constexpr int h = decltype(P)::value;
    const int64_t zb = static_cast<int64_t>(pmod(z, nz)) * plane;
#pragma unroll
    for (int k = 0; k < PERP; ++k)
      if (pact[k]) rp[h][k] = phi[zb + poff[k]];
  };
  C ux[2][PERV], uy[2][PERV], uz[2][PERV];
  auto fetch_u = [&](auto P, int z) {
    constexpr int h = decltype(P)::value;
    const int64_t zb = static_cast<int64_t>(pmod(z, nz)) * plane;
#pragma unroll
    for (int k = 0; k < PERV; ++k)
      if (vact[k]) {
        ux[h][k] = S::load(st + N, zb + voff[k], s1);
        uy[h][k] = S::load(st + 2 * N, zb + voff[k], s2);
        uz[h][k] = S::load(st + 3 * N, zb + voff[k], s3);
      }
  };
  // per slot: gradient sums of V(q) (m) and V(q + 1) (0), phi of V(q), and
  // the record V(q - 1) completed this iteration
  C gxm[PERV], gym[PERV], gzm[PERV], pv[PERV], gx0[PERV], gy0[PERV], gz0[PERV];
  Rec<C> rv[PERV];
#pragma unroll
  for (int k = 0; k < PERV; ++k) {
    gxm[k] = gym[k] = gzm[k] = pv[k] = gx0[k] = gy0[k] = gz0[k] = C(0);
    ux[0][k] = uy[0][k] = uz[0][k] = ux[1][k] = uy[1][k] = uz[1][k] = C(0);
    rv[k] = Rec<C>{C(0), C(0), C(0), C(0)};
  }
  const int x = x0 + lane, y = y0 + wy;
  const bool mine = x < nx && y < ny;
  // divergence and Laplacian sums of phi'(q - 3) (m) and phi'(q - 2) (0), the
  // Laplacian of the latter relative to ref0
  C dvm = 0, lm = 0, pm = 0;
  C dv0 = 0, l0 = 0, ref0 = 0;
  // iteration q; P = (q - z0) & 1 is the register set of plane q
  auto body = [&](int q, auto P) {
    constexpr int h = decltype(P)::value;
    using Other = std::integral_constant<int, 1 - h>;
    if (q <= z1 + 1) {
#pragma unroll
      for (int k = 0; k < PERP; ++k)
        if (pact[k]) tp[q & 1][threadIdx.x + k * NT] = rp[h][k];
    }
    if (q >= z0 + 1) {
#pragma unroll
      for (int k = 0; k < PERV; ++k)
        if (vact[k]) tv[q & 1][threadIdx.x + k * NT] = rv[k];
    }
    __syncthreads();
    if (q + 2 <= z1 + 1) fetch_phi(P, q + 2);  // in flight for two iterations
    if (q <= z1 + 1) {
      const C* w = tp[q & 1];
#pragma unroll
      for (int k = 0; k < PERV; ++k)
        if (vact[k]) {
          C n[3][3];
#pragma unroll
          for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) n[dy][dx] = w[vwin[k] + dy * PX + dx];
          C axu = 0, ayu = 0, azu = 0, axc = 0, ayc = 0;
#pragma unroll
          for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
              const C v = n[dy + 1][dx + 1];
              const C ku = C(k27(dx, dy, 1));
              if (dx) axu += C(dx) * ku * v;
              if (dy) ayu += C(dy) * ku * v;
              azu += ku * v;
              if (dx || dy) {
                const C kc = C(k27(dx, dy, 0));
                if (dx) axc += C(dx) * kc * v;
                if (dy) ayc += C(dy) * kc * v;
              }
            }
          // V(q - 1) is complete: this plane is at dz = +1 from it; its u is
          // in the other set
          const C g[3] = {div_by<72>(gxm[k] + axu), div_by<72>(gym[k] + ayu),
                          div_by<72>(gzm[k] + azu)};
          const C p = pv[k];
          const C c =
              lambda * p * (C(1) - p) / (sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + eps);
          rv[k].vx = p * ux[1 - h][k] + c * g[0];
          rv[k].vy = p * uy[1 - h][k] + c * g[1];
          rv[k].vz = p * uz[1 - h][k] + c * g[2];
          rv[k].phi = p;
          if (vneg[k]) rv[k].vy = -rv[k].vy;
          // V(q): plane q - 1 (at dz = -1) plus this plane; V(q + 1): this
          // plane at dz = -1
          gxm[k] = gx0[k] + axc;
          gym[k] = gy0[k] + ayc;
          gzm[k] = gz0[k];
          pv[k] = n[1][1];
          gx0[k] = axu;
          gy0[k] = ayu;
          gz0[k] = -azu;
        }
      // u of plane q + 1 (same set as plane q - 1), used two iterations on
      if (q + 1 >= z0 - 1 && q + 1 <= z1) fetch_u(Other{}, q + 1);
    }
    if (q >= z0 + 1) {
      // records V(q - 2): destination q - 3 completes
      const Rec<C>* t = tv[q & 1];
      Rec<C> r[3][3];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) r[dy][dx] = t[(wy + dy) * VX + lane + dx];
      const C own = r[1][1].phi;
      C dvu = 0, lu = 0, dvc = 0, lc = 0, dvd = 0, ld = 0;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const Rec<C>& n = r[dy + 1][dx + 1];
          C cv = 0;
          if (dx) cv += C(dx) * n.vx;
          if (dy) cv += C(dy) * n.vy;
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
      const int d = q - 3;
      if (mine && d >= z0 && d < z1)
        out[static_cast<int64_t>(d) * plane + static_cast<int64_t>(y) * nx + x] =
            pm - div_by<72>(dvm + dvd) + D * div_by<36>(lm + ld);
      dvm = dv0 + dvc;
      lm = l0 - C(KZ) * (own - ref0) + lc;
      pm = own;
      dv0 = dvu;
      l0 = lu;
      ref0 = own;
    }
  };
  // phi planes z0 - 2 .. z1 + 1 give V(z0 - 1) .. V(z1), which give phi'(z0)
  // .. phi'(z1 - 1)
  fetch_phi(I0{}, z0 - 2);
  fetch_phi(I1{}, z0 - 1);
  for (int q = z0 - 2; q <= z1 + 2; q += 2) {
    body(q, I0{});
    if (q + 1 <= z1 + 2) body(q + 1, I1{});
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
// same tiles, z-march, staging and 2.5-D accumulation as the phase update,
// on the scalar phi (a y wall's ghost is the mirror value)
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
  // Laplacian relative to ref0)
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
  hipLaunchKernelGGL((phase_kernel<ST>), dim3(m.blocks), dim3(64 * kUpdRows), 0, s,
                     static_cast<const C*>(a.phi), static_cast<const T*>(a.state),
                     static_cast<C*>(a.phi_out), a.nx, a.ny, a.nz, a.N, static_cast<C>(a.D),
                     static_cast<C>(a.lambda), static_cast<C>(a.eps), a.scale[1], a.scale[2],
                     a.scale[3], m.tiles_x, m.tiles_y, m.zchunk, a.walls_y != 0);
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
