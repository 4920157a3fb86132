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
// Derivatives use the D3Q27-weighted stencils of section 2 (stencil.hpp),
// and div V = (1/cs^2) sum_i w_i c_i . V(x + c_i).  Periodic grid.
//
// One z-march advances phi: it computes the total flux V = phi u + lambda J
// (J the normalised compression flux) on the fly, keeping the tile's records
// in LDS, and then phi' = phi - div(V) + D lap(phi).  A second march gives
// the force of a phase field that is set from outside (the first F(t)); while
// stepping, the fused step computes F(t+1) itself from phi(t+1).  Algorithmic
// traffic at FP32: the phase update 20 B per lattice update (phi, u in; phi
// out), the force march 16 B (phi in, F out).
#include <atomic>

#include "internal.hpp"
#include "lattice.hpp"
#include "stencil.hpp"

namespace lbf {
namespace {

constexpr int kPhaseThreads = 256;

// 1 / (sqrt(g2) + eps) for the interface normal: FP64 evaluates it exactly
// rounded; FP32 uses the hardware square root and reciprocal (about one unit in
// the last place each, against a sequence of some 16 instructions for the
// correctly rounded pair)
template <typename C>
__device__ __forceinline__ C inv_norm_eps(C g2, C eps) {
  if constexpr (std::is_same_v<C, float>)
    return __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(g2) + eps);
  else
    return C(1) / (sqrt(g2) + eps);
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
// 16 rows: the record ring and the phi halo are a smaller share of the tile
// than with 8 (measured 1% faster for the whole two-component step at 256^3)
constexpr int kUpdRows = 16;
// Loads ahead of use in the staged marches.  Iterations run in groups of
// kGroup planes, with two register banks: at the start of a group the next
// group's values are issued into one bank, and the current group is taken
// from the other.  So a value is loaded one to two groups before its use.
// Only the loads issued at the start of the group are ever in flight at a
// wait, even where the compiler's wait counting treats loads that cross
// the loop's back edge as just issued.  Every load is unconditional: an
// inactive slot reads offset 0, and a plane index past the chunk is clamped,
// which re-reads a cached plane.  So the loads form one fixed sequence.
constexpr int kGroup = 1;

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
  constexpr int KZ = kPlaneK;
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
  // Loads go through buffer resources of one plane with 32-bit in-plane byte
  // offsets (the host keeps a plane of doubles below 4 GiB).
  // staged phi values: in-plane offset (a wall's ghost rows hold the clamped
  // row, which is the mirror image one site beyond the wall; rows further out
  // feed only slots that are never read for an owned site)
  const uint32_t pbytes_c = static_cast<uint32_t>(plane * sizeof(C));
  const uint32_t pbytes_t = static_cast<uint32_t>(plane * sizeof(typename S::T));
  uint32_t poff[PERP];
  bool pact[PERP];
#pragma unroll
  for (int k = 0; k < PERP; ++k) {
    const int e = threadIdx.x + k * NT;
    pact[k] = e < NP;
    const int ry = pact[k] ? e / PX : 0, rx = pact[k] ? e - ry * PX : 0;
    const int yr = y0 + ry - 2;
    const int yw = walls_y ? clampi(yr, 0, ny - 1) : pmod(yr, ny);
    poff[k] = pact[k] ? static_cast<uint32_t>((yw * nx + pmod(x0 + rx - 2, nx)) * sizeof(C)) : 0u;
  }
  // record slots: the source site (the mirror site for a ghost), the top-left
  // of its 3 x 3 phi window in the staged plane, and whether v_y is reversed.
  // Rows: the source row ys lies in [y0 - 1, y0 + kUpdRows], so the window
  // rows ys - y0 + 1 .. ys - y0 + 3 lie in [0, PY).
  uint32_t voff[PERV];
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
    voff[k] = vact[k] ? static_cast<uint32_t>((ys * nx + pmod(x0 + rx - 1, nx)) *
                                              sizeof(typename S::T))
                      : 0u;
  }
  // register banks: slot i of a group starting at plane qs holds phi of
  // plane qs + i and u of plane qs + i - 1 (for V(qs + i - 1))
  constexpr int G = kGroup;
  C rp[2][G][PERP];
  C ux[2][G][PERV], uy[2][G][PERV], uz[2][G][PERV];
  auto load_group = [&](auto B, int qs) {
    constexpr int b = decltype(B)::value;
    static_for<G>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const int64_t zp = static_cast<int64_t>(pmod(min(qs + i, z1 + 1), nz)) * plane;
#pragma unroll
      for (int k = 0; k < PERP; ++k) rp[b][i][k] = buf_load<C>(plane_rsrc(phi + zp, pbytes_c), poff[k]);
      const int64_t zu = static_cast<int64_t>(pmod(clampi(qs + i - 1, z0 - 1, z1), nz)) * plane;
#pragma unroll
      for (int k = 0; k < PERV; ++k) {
        if constexpr (S::kGrouped) {
          // 16-bit storage: p*, u_x, u_y, u_z of a site are one 64-bit word
          using T4 = typename S::T __attribute__((ext_vector_type(4)));
          const uint64_t* st64 = reinterpret_cast<const uint64_t*>(st);
          const T4 h = __builtin_bit_cast(
              T4, buf_load<uint64_t>(plane_rsrc(st64 + zu, 4 * pbytes_t), 4 * voff[k]));
          ux[b][i][k] = S::decode(h.y, s1);
          uy[b][i][k] = S::decode(h.z, s2);
          uz[b][i][k] = S::decode(h.w, s3);
        } else {
          ux[b][i][k] = S::decode(buf_load<typename S::T>(plane_rsrc(st + N + zu, pbytes_t), voff[k]), s1);
          uy[b][i][k] = S::decode(buf_load<typename S::T>(plane_rsrc(st + 2 * N + zu, pbytes_t), voff[k]), s2);
          uz[b][i][k] = S::decode(buf_load<typename S::T>(plane_rsrc(st + 3 * N + zu, pbytes_t), voff[k]), s3);
        }
      }
    });
  };
  // per slot: gradient sums of V(q) (m) and V(q + 1) (0), phi of V(q), and
  // the record V(q - 1) completed this iteration
  C gxm[PERV], gym[PERV], gzm[PERV], pv[PERV], gx0[PERV], gy0[PERV], gz0[PERV];
  Rec<C> rv[PERV];
#pragma unroll
  for (int k = 0; k < PERV; ++k) {
    gxm[k] = gym[k] = gzm[k] = pv[k] = gx0[k] = gy0[k] = gz0[k] = C(0);
    rv[k] = Rec<C>{C(0), C(0), C(0), C(0)};
  }
  const int x = x0 + lane, y = y0 + wy;
  const bool mine = x < nx && y < ny;
  const uint32_t own_off = mine ? static_cast<uint32_t>((y * nx + x) * sizeof(C)) : 0u;
  // divergence and Laplacian sums of phi'(q - 3) (m) and phi'(q - 2) (0), the
  // Laplacian of the latter relative to ref0
  C dvm = 0, lm = 0, pm = 0;
  C dv0 = 0, l0 = 0, ref0 = 0;
  // iteration q, its values in slot I of bank B
  auto body = [&](int q, auto B, auto I) {
    constexpr int b = decltype(B)::value, i = decltype(I)::value;
    if (q <= z1 + 1) {
#pragma unroll
      for (int k = 0; k < PERP; ++k)
        if (pact[k]) tp[q & 1][threadIdx.x + k * NT] = rp[b][i][k];
    }
    if (q >= z0 + 1) {
#pragma unroll
      for (int k = 0; k < PERV; ++k)
        if (vact[k]) tv[q & 1][threadIdx.x + k * NT] = rv[k];
    }
    __syncthreads();
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
          C ss, ds, sd;
          window_sums(n, ss, ds, sd);
          // V(q - 1) is complete: this plane is at dz = +1 from it
          const C g[3] = {div_by<72>(gxm[k] + ds), div_by<72>(gym[k] + sd),
                          div_by<72>(gzm[k] + ss)};
          const C p = pv[k];
          const C c = lambda * p * (C(1) - p) *
                      inv_norm_eps(g[0] * g[0] + g[1] * g[1] + g[2] * g[2], eps);
          rv[k].vx = p * ux[b][i][k] + c * g[0];
          rv[k].vy = p * uy[b][i][k] + c * g[1];
          rv[k].vz = p * uz[b][i][k] + c * g[2];
          rv[k].phi = p;
          if (vneg[k]) rv[k].vy = -rv[k].vy;
          // V(q): plane q - 1 (at dz = -1) plus this plane; V(q + 1): this
          // plane at dz = -1
          gxm[k] = gx0[k] + C(4) * ds;
          gym[k] = gy0[k] + C(4) * sd;
          gzm[k] = gz0[k];
          pv[k] = n[1][1];
          gx0[k] = ds;
          gy0[k] = sd;
          gz0[k] = -ss;
        }
    }
    if (q >= z0 + 1) {
      // records V(q - 2): destination q - 3 completes
      const Rec<C>* t = tv[q & 1];
      C vx[3][3], vy[3][3], vz[3][3], ph[3][3];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const Rec<C> n = t[(wy + dy) * VX + lane + dx];
          vx[dy][dx] = n.vx;
          vy[dy][dx] = n.vy;
          vz[dy][dx] = n.vz;
          ph[dy][dx] = n.phi;
        }
      const C own = ph[1][1];
      // window sums of the records: a = sum k1 k1 (c_x v_x + c_y v_y) and
      // bz = sum k1 k1 v_z.  The destination one plane up sees this plane at
      // c_z = -1 and takes a - bz (dvu), the one below a + bz (dvd), this
      // plane's own 4 a (dvc).  Laplacian sums relative to own (lu), and to
      // pm, the phi of the destination below (ld).
      C ss, ds, sd;
      window_sums(vx, ss, ds, sd);
      const C ax = ds;
      window_sums(vy, ss, ds, sd);
      const C a = ax + sd;
      window_sums(vz, ss, ds, sd);
      const C bz = ss;
      const C dvu = a - bz, dvd = a + bz, dvc = C(4) * a;
      const C lu = window_lap(ph, own);
      const C ld = lu + C(KZ) * (own - pm), lc = C(4) * lu;
      const int d = q - 3;
      if (mine && d >= z0 && d < z1)
        buf_store<C>(pm - div_by<72>(dvm + dvd) + D * div_by<36>(lm + ld),
                     plane_rsrc(out + static_cast<int64_t>(d) * plane, pbytes_c), own_off);
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
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  load_group(B0{}, z0 - 2);
  // whole pairs of groups; iterations past z1 + 2 store nothing
  for (int q = z0 - 2; q <= z1 + 2; q += 2 * G) {
    load_group(B1{}, q + G);
    static_for<G>([&](auto I) { body(q + decltype(I)::value, B0{}, I); });
    load_group(B0{}, q + 2 * G);
    static_for<G>([&](auto I) { body(q + G + decltype(I)::value, B1{}, I); });
  }
}

// Output of the force pass at one site: F = mu grad(phi) + rho(phi) g, plus
// (contrast) the pressure and viscous terms - p* cs^2 grad(rho)
// - (nu omega / cs^2) (a2 - u u) . grad(rho), with p*, u, a2 of the state at
// the previous time level.  The state values a site needs are loaded ahead
// (prefetch) and handed back with its derivatives.
template <int ST, bool CONTRAST>
struct ForceEmit {
  using S = Storage<ST>;
  using C = typename S::C;
  struct Pre {
    C m[CONTRAST ? 10 : 1];
  };
  const typename S::T* st;
  C* F;
  int64_t N;
  PhaseArgs pa;
  __device__ __forceinline__ void prefetch(int64_t s, Pre& pre) const {
    if constexpr (CONTRAST) {
#pragma unroll
      for (int k = 0; k < 10; ++k) pre.m[k] = S::load(st, plane_elem<S>(k, s, N), pa.scale[k]);
    }
  }
  __device__ __forceinline__ void operator()(int64_t s, C p, const C g[3], C l,
                                             const Pre& pre) const {
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
      for (int k = 0; k < 10; ++k) m[k] = pre.m[k];
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
// same tiles, staging and 2.5-D accumulation as the phase update, on the
// scalar phi (a y wall's ghost is the mirror value).  Iteration p stages
// plane p and completes destination p - 1.  phi and the functor's per-site
// values are loaded in groups into two register banks, as in the phase
// update.
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
  constexpr int KZ = kPlaneK;
  constexpr int G = kGroup;
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
    off[k] = act[k] ? static_cast<int64_t>(yw) * nx + xw : 0;
    pos[k] = ry * RX + rx;
  }
  const int x = x0 + lane, y = y0 + wy;
  const bool mine = x < nx && y < ny;
  // the functor's values of a thread without a site are read at offset 0
  const int64_t own_off = mine ? static_cast<int64_t>(y) * nx + x : 0;
  // slot i of a group starting at plane ps: phi of plane ps + i and the
  // functor's values of destination ps + i - 1
  C r[2][G][PER];
  typename Emit::Pre pre[2][G];
  auto load_group = [&](auto B, int ps) {
    constexpr int b = decltype(B)::value;
    static_for<G>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const int64_t zb = static_cast<int64_t>(pmod(min(ps + i, z1), nz)) * plane;
#pragma unroll
      for (int k = 0; k < PER; ++k) r[b][i][k] = phi[zb + off[k]];
      emit.prefetch(static_cast<int64_t>(clampi(ps + i - 1, z0, z1 - 1)) * plane + own_off,
                    pre[b][i]);
    });
  };
  // destination p - 1 (sums and phi_0) and p (sums from plane p - 1, the
  // Laplacian relative to ref0)
  C gxm = 0, gym = 0, gzm = 0, lm = 0, pm = 0;
  C gx0 = 0, gy0 = 0, gz0 = 0, l0 = 0, ref0 = 0;
  auto body = [&](int p, auto B, auto I) {
    constexpr int b = decltype(B)::value, i = decltype(I)::value;
    {
      C* dst = &t[p & 1][0][0];
#pragma unroll
      for (int k = 0; k < PER; ++k)
        if (act[k]) dst[pos[k]] = r[b][i][k];
    }
    __syncthreads();
    C q[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) q[dy][dx] = t[p & 1][wy + dy][lane + dx];
    const C own = q[1][1];
    // this plane's separable sums with the weights of an adjacent plane; the
    // own plane's weights are 4 times those (centre excluded from the
    // Laplacian, where its term is zero)
    C azu, axu, ayu;
    window_sums(q, azu, axu, ayu);
    const C lu = window_lap(q, own);
    const C ld = lu + C(KZ) * (own - pm);
    const C axc = C(4) * axu, ayc = C(4) * ayu, lc = C(4) * lu;
    // destination p - 1 is complete: this plane is at dz = +1 from it
    if (mine && p - 1 >= z0 && p - 1 < z1) {
      const C g[3] = {div_by<72>(gxm + axu), div_by<72>(gym + ayu), div_by<72>(gzm + azu)};
      emit(static_cast<int64_t>(p - 1) * plane + own_off, pm, g, div_by<36>(lm + ld),
           pre[b][i]);
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
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  load_group(B0{}, z0 - 1);
  // whole pairs of groups; iterations past z1 emit nothing
  for (int p = z0 - 1; p <= z1; p += 2 * G) {
    load_group(B1{}, p + G);
    static_for<G>([&](auto I) { body(p + decltype(I)::value, B0{}, I); });
    load_group(B0{}, p + 2 * G);
    static_for<G>([&](auto I) { body(p + G + decltype(I)::value, B1{}, I); });
  }
}

// tiles and z-chunks of the staged passes: 64 x kUpdRows columns, z-chunks of
// >= 8 planes, about as many workgroups as the device holds at once
// (`target`), so that each CU runs as many marches as fit and they share
// the memory latency
struct MarchGeom {
  int tiles_x, tiles_y, zchunk, blocks;
};
MarchGeom march_geom(int nx, int ny, int nz, int target) {
  MarchGeom m;
  m.tiles_x = (nx + 63) / 64;
  m.tiles_y = (ny + kUpdRows - 1) / kUpdRows;
  const int cols = m.tiles_x * m.tiles_y;
  int nch = (target + cols - 1) / cols;
  const int maxc = nz >= 8 ? nz / 8 : 1;
  nch = nch < 1 ? 1 : (nch > maxc ? maxc : nch);
  m.zchunk = (nz + nch - 1) / nch;
  m.blocks = cols * ((nz + m.zchunk - 1) / m.zchunk);
  return m;
}

// workgroups of 64 x kUpdRows threads of kernel K resident on the current
// device at once (compute units x blocks per unit); 512 if the runtime does
// not say.  The answer depends only on the kernel and the device, so it is
// asked once per device and kept.
template <auto K>
int resident_blocks() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 512;
  }
  const bool slot = dev >= 0 && dev < 64;
  if (slot) {
    const int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(K),
                                                   64 * kUpdRows, 0) != hipSuccess ||
      cus < 1 || per < 1) {
    (void)hipGetLastError();
    return 512;
  }
  if (slot) cache[dev].store(cus * per, std::memory_order_relaxed);
  return cus * per;
}

int phase_grid(int64_t N) {
  const int64_t b = (N + kPhaseThreads - 1) / kPhaseThreads;
  return static_cast<int>(b < 16384 ? (b < 1 ? 1 : b) : 16384);
}

template <int ST>
hipError_t phase_step_st(const PhaseArgs& a, hipStream_t s) {
  using C = typename Storage<ST>::C;
  using T = typename Storage<ST>::T;
  const MarchGeom m = march_geom(a.nx, a.ny, a.nz, resident_blocks<phase_kernel<ST>>());
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
  const C* phi = static_cast<const C*>(a.phi_out);
  const T* st = static_cast<const T*>(a.state);
  auto launch = [&](auto contrast) {
    using E = ForceEmit<ST, decltype(contrast)::value>;
    const MarchGeom m = march_geom(a.nx, a.ny, a.nz, resident_blocks<grad_march_kernel<C, E>>());
    hipLaunchKernelGGL((grad_march_kernel<C, E>), dim3(m.blocks), dim3(64 * kUpdRows), 0, s, phi, a.nx, a.ny, a.nz,
                       m.tiles_x, m.tiles_y, m.zchunk, a.walls_y != 0,
                       E{st, static_cast<C*>(a.F), a.N, a});
  };
  if (a.contrast)
    launch(std::true_type{});
  else
    launch(std::false_type{});
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
