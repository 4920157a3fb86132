// step_kernel.hpp -- the fused stream-and-collide step of the moment-represented
// regularized LBM (Lauricella et al., arXiv 2609.09160, section 2: Eq. (7)
// followed by the correction of Eq. (8); section 3 for the fused pull kernel
// that never stores populations).
//
// What one launch computes, for every site x (destination):
//   1. at every source site y: the post-collision Hermite coefficients
//        P0 = p*,  P1 = u + F/2,
//        P2 = u u + (1 - omega)(a2 - u u) + (u F + F u)/2
//      (equilibrium + relaxed non-equilibrium of Eq. (6), plus half of the Guo
//      source of Eq. (9), whose Hermite coefficients are F and u F + F u);
//   2. the reconstructed populations of Eq. (4) at y,
//        f_i(y) = w_i [P0 - 1.5 tr P2 + 3 c_i.P1 + 4.5 c_i c_i : P2];
//   3. the pull f_i(x) = f_i(x - c_i) (periodic wrap, or halfway bounce-back
//      f_i(x) = f_{-i}(x) where x - c_i lies beyond a y wall);
//   4. the projection of Eq. (5): s0 = sum f, s1 = sum c f,
//      s2 = sum c c f - cs^2 s0 I;
//   5. the correction of Eq. (8) with F at x: u = s1 + F/2,
//      a2 = s2 + (F u + u F)/2 (updated u), a0 = s0.
//
// gfx950 mapping (own design; the paper's 8x8x8 shared-memory tiles are prior
// art for another GPU):
//   * a workgroup owns a 64 x TY column tile of the x-y plane and a chunk of
//     z-planes, and marches through z;
//   * wave w (0..TY+1) handles tile row w-1; waves 0 and TY+1 are the y-halo
//     rows and also compute the two x-halo columns (lanes 0..TY+1);
//   * per source plane, every thread collides its own site once and writes the
//     populations that leave its (x, y) column (16 for D3Q19, 24 for D3Q27)
//     to LDS; after a barrier each interior thread pulls the 3x3 column
//     neighbourhood from LDS;
//   * populations travelling along z stay in registers: the ones with c_z=+1
//     wait one plane, the ones with c_z=-1 complete the previous plane, so each
//     moment is read from HBM once per update (plus L2-resident halos) and
//     written once, with no population array anywhere;
//   * block ids are remapped so that each XCD (own L2) gets a contiguous range
//     of tiles, y-neighbours first: concurrently running tiles share halo rows.
#pragma once

#ifndef LBF_PREFETCH_DEPTH
#define LBF_PREFETCH_DEPTH 1
#endif

#include "internal.hpp"
#include "lattice.hpp"

namespace lbf {

// Steps 1-2 at one source site: post-collision coefficients and the
// reconstructed populations, kept in units of 1/D: g[i] = D f_i(y) with
// D f_i = k_i [P0 - 1.5 tr P2 + 3 c.P1 + 4.5 c c : P2], k_i = D w_i.
template <int Q, typename C>
__device__ __forceinline__ void source_pops(const C m[10], C Fx, C Fy, C Fz, C omega, C g[Q]) {
  using L = Lat<Q>;
  const C h = C(0.5);
  const C om1 = C(1) - omega;
  const C ux = m[1], uy = m[2], uz = m[3];
  const C P2xx = omega * ux * ux + om1 * m[4] + ux * Fx;
  const C P2yy = omega * uy * uy + om1 * m[5] + uy * Fy;
  const C P2zz = omega * uz * uz + om1 * m[6] + uz * Fz;
  const C P2xy = omega * ux * uy + om1 * m[7] + h * (ux * Fy + uy * Fx);
  const C P2xz = omega * ux * uz + om1 * m[8] + h * (ux * Fz + uz * Fx);
  const C P2yz = omega * uy * uz + om1 * m[9] + h * (uy * Fz + uz * Fy);
  // scaled coefficients of the reconstruction (cs^2 = 1/3)
  const C A = m[0] - C(1.5) * (P2xx + P2yy + P2zz);
  const C Vx = C(3) * (ux + h * Fx), Vy = C(3) * (uy + h * Fy), Vz = C(3) * (uz + h * Fz);
  const C Dx = C(4.5) * P2xx, Dy = C(4.5) * P2yy, Dz = C(4.5) * P2zz;
  const C Oxy = C(9) * P2xy, Oxz = C(9) * P2xz, Oyz = C(9) * P2yz;
  static_for<Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    C v = A;
    if constexpr (cx != 0) v += Dx;
    if constexpr (cy != 0) v += Dy;
    if constexpr (cz != 0) v += Dz;
    if constexpr (cx * cy == 1) v += Oxy;
    if constexpr (cx * cy == -1) v -= Oxy;
    if constexpr (cx * cz == 1) v += Oxz;
    if constexpr (cx * cz == -1) v -= Oxz;
    if constexpr (cy * cz == 1) v += Oyz;
    if constexpr (cy * cz == -1) v -= Oyz;
    if constexpr (cx == 1) v += Vx;
    if constexpr (cx == -1) v -= Vx;
    if constexpr (cy == 1) v += Vy;
    if constexpr (cy == -1) v -= Vy;
    if constexpr (cz == 1) v += Vz;
    if constexpr (cz == -1) v -= Vz;
    g[i] = (L::k(i) == 1.0) ? v : C(L::k(i)) * v;
  });
}

// Steps 4-5 at one destination site, split so that populations can be folded
// in as they arrive: Sums holds the running projections (in units of 1/D) on
// H0 (s0), H1 (j) and c c (p); finalize() turns them into the moments of the
// new time level and applies the force-consistent correction.
template <typename C>
struct Sums {
  C s0, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
};

template <typename C>
__device__ __forceinline__ void zero(Sums<C>& S) {
  S.s0 = S.jx = S.jy = S.jz = S.pxx = S.pyy = S.pzz = S.pxy = S.pxz = S.pyz = C(0);
}

// add population v travelling along direction i
template <int Q, int i, typename C>
__device__ __forceinline__ void accumulate(Sums<C>& S, C v) {
  using L = Lat<Q>;
  constexpr int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
  S.s0 += v;
  if constexpr (cx == 1) S.jx += v;
  if constexpr (cx == -1) S.jx -= v;
  if constexpr (cy == 1) S.jy += v;
  if constexpr (cy == -1) S.jy -= v;
  if constexpr (cz == 1) S.jz += v;
  if constexpr (cz == -1) S.jz -= v;
  if constexpr (cx != 0) S.pxx += v;
  if constexpr (cy != 0) S.pyy += v;
  if constexpr (cz != 0) S.pzz += v;
  if constexpr (cx * cy == 1) S.pxy += v;
  if constexpr (cx * cy == -1) S.pxy -= v;
  if constexpr (cx * cz == 1) S.pxz += v;
  if constexpr (cx * cz == -1) S.pxz -= v;
  if constexpr (cy * cz == 1) S.pyz += v;
  if constexpr (cy * cz == -1) S.pyz -= v;
}

template <int Q, typename C>
__device__ __forceinline__ void finalize(const Sums<C>& S, C Fx, C Fy, C Fz, C out[10]) {
  constexpr int D = Lat<Q>::D;
  const C h = C(0.5);
  const C ux = div_by<D>(S.jx) + h * Fx;
  const C uy = div_by<D>(S.jy) + h * Fy;
  const C uz = div_by<D>(S.jz) + h * Fz;
  out[0] = div_by<D>(S.s0);
  out[1] = ux;
  out[2] = uy;
  out[3] = uz;
  // H2 diagonal: sum c_a^2 f - cs^2 sum f = (3 sum c_a^2 f - sum f) / 3
  out[4] = div_by<3 * D>(C(3) * S.pxx - S.s0) + Fx * ux;
  out[5] = div_by<3 * D>(C(3) * S.pyy - S.s0) + Fy * uy;
  out[6] = div_by<3 * D>(C(3) * S.pzz - S.s0) + Fz * uz;
  out[7] = div_by<D>(S.pxy) + h * (Fx * uy + Fy * ux);
  out[8] = div_by<D>(S.pxz) + h * (Fx * uz + Fz * ux);
  out[9] = div_by<D>(S.pyz) + h * (Fy * uz + Fz * uy);
}

template <int Q, int ST, int TY, bool WALLY, bool FFIELD>
__global__ void __launch_bounds__(64 * (TY + 2)) step_kernel(const StepArgs a) {
  using L = Lat<Q>;
  using S = Storage<ST>;
  using C = typename S::C;
  using T = typename S::T;
  constexpr int NP = L::NP, NB = L::NB;
  constexpr int R = TY + 2;  // LDS rows: tile rows plus the two y-halo rows
  constexpr int W = 66;      // LDS columns: 64 lanes plus the two x-halo columns
  __shared__ C lds[NP][R][W];
  __shared__ C colbuf[NP][2][R];  // next plane's x-halo columns (halo waves)

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;  // LDS row of this wave's sites
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int64_t N = a.N;
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);
  const C* __restrict__ Ff = static_cast<const C*>(a.Ffield);
  const C omega = static_cast<C>(a.omega);

  // Hardware hands consecutive block ids to the 8 XCDs in turn; give each XCD
  // a contiguous range of logical tiles (y fastest, then x, then z chunk).
  const int nb = static_cast<int>(gridDim.x), b0 = static_cast<int>(blockIdx.x);
  const int q8 = nb >> 3, r8 = nb & 7, xcd = b0 & 7;
  int b = xcd * q8 + (xcd < r8 ? xcd : r8) + (b0 >> 3);
  const int tyi = b % a.tiles_y;
  b /= a.tiles_y;
  const int txi = b % a.tiles_x;
  const int zci = b / a.tiles_x;
  const int x0 = txi * 64, y0 = tyi * TY;
  const int z0 = zci * a.zchunk;
  const int z1 = min(z0 + a.zchunk, nz);

  // In-plane byte offsets are 32-bit (the host enforces nx*ny*8 < 2^32); the
  // per-plane base pointers are uniform, so every load and store is a scalar
  // base plus one vector offset.
  // own source site (every lane computes a valid, possibly wrapped, site)
  const int xs = pmod(x0 + lane, nx);
  const int ys = WALLY ? clampi(y0 + wv - 1, 0, ny - 1) : pmod(y0 + wv - 1, ny);
  const uint32_t off_s = (static_cast<uint32_t>(ys) * static_cast<uint32_t>(nx) + xs) * sizeof(T);
  // x-halo site: wave 0 takes the left column, wave R-1 the right one
  const bool do_halo = (wv == 0 || wv == R - 1) && lane < R;
  const int hcol = (wv == 0) ? 0 : W - 1;
  const int xh = pmod(wv == 0 ? x0 - 1 : x0 + 64, nx);
  const int yh = WALLY ? clampi(y0 - 1 + lane, 0, ny - 1) : pmod(y0 - 1 + lane, ny);
  const uint32_t off_h = (static_cast<uint32_t>(yh) * static_cast<uint32_t>(nx) + xh) * sizeof(T);
  // destination
  const bool interior = (wv >= 1 && wv <= TY);
  const int xd = x0 + lane, yd = y0 + wv - 1;
  const bool store_ok = interior && xd < nx && yd < ny;
  const uint32_t off_d = (static_cast<uint32_t>(yd) * static_cast<uint32_t>(nx) + xd) * sizeof(T);
  const bool wall_lo = WALLY && interior && yd == 0;
  const bool wall_hi = WALLY && interior && yd == ny - 1;

  // raw (still encoded) moments and force of one site, fetched a plane ahead
  struct Raw {
    T m[10];
    C F[3];
  };

  // the force field has the compute type; its byte offset scales accordingly
  constexpr uint32_t kFscale = sizeof(C) / sizeof(T);
  const uint32_t plane_bytes = static_cast<uint32_t>(plane * sizeof(T));
  // periodic plane index for zs >= -1 (zs is uniform: scalar arithmetic;
  // planes past the end of a padded chunk are fetched but never used)
  auto zwrap = [&](int zs) __attribute__((always_inline)) {
    zs = zs < 0 ? zs + nz : zs;
    zs = zs >= nz ? zs - nz : zs;
    return zs >= nz ? zs % nz : zs;
  };
  auto fetch = [&](const int zs, const uint32_t off, Raw& r) __attribute__((always_inline)) {
    const int64_t pb = static_cast<int64_t>(zwrap(zs)) * plane;
#pragma unroll
    for (int k = 0; k < 10; ++k)
      r.m[k] = buf_load<T>(plane_rsrc(src + (k * N + pb), plane_bytes), off);
    if constexpr (FFIELD) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
        r.F[k] = buf_load<C>(plane_rsrc(Ff + (k * N + pb), plane_bytes * kFscale), off * kFscale);
    }
  };
  auto collide = [&](const Raw& r, C g[Q], C Fo[3]) __attribute__((always_inline)) {
    C m[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = S::decode(r.m[k], a.scale[k]);
    if constexpr (FFIELD) {
      Fo[0] = r.F[0];
      Fo[1] = r.F[1];
      Fo[2] = r.F[2];
    } else {
      Fo[0] = static_cast<C>(a.F[0]);
      Fo[1] = static_cast<C>(a.F[1]);
      Fo[2] = static_cast<C>(a.F[2]);
    }
    source_pops<Q, C>(m, Fo[0], Fo[1], Fo[2], omega, g);
  };
  auto stage = [&](const C g[Q], const int row, const int col) __attribute__((always_inline)) {
    static_for<NP>([&](auto I) {
      constexpr int i = decltype(I)::value;
      lds[i][row][col] = g[i];
    });
  };
  // population i arriving at this thread's destination from the LDS plane;
  // on a wall row the ones that would come from beyond the wall are dropped
  // here and replaced by the reflections added in body_interior
  auto pulled = [&](auto I) __attribute__((always_inline)) -> C {
    constexpr int i = decltype(I)::value;
    C v = lds[i][wv - L::cy(i)][lane + 1 - L::cx(i)];
    if constexpr (WALLY && L::cy(i) == 1) v = wall_lo ? C(0) : v;
    if constexpr (WALLY && L::cy(i) == -1) v = wall_hi ? C(0) : v;
    return v;
  };

  // Interior waves, one source plane zs per call.  acc: running sums of
  // destination plane zs-1 (all but its c_z=-1 populations), completed and
  // stored here; up: the c_z=+1 populations that reach plane zs from zs-1;
  // Fd: force at the own site of plane zs-1.  rc holds this plane's moments,
  // rn receives the next plane's (one plane of latency hiding).
  constexpr int NU = (Q == 19) ? 5 : 9;  // populations with c_z = +1
  auto body_interior = [&](const int zs, Sums<C>& acc, C (&up)[NU], C (&Fd)[3], Raw& rc,
                           Raw& rn, const int ahead) __attribute__((always_inline)) {
    // unconditional (the last planes of a chunk fetch unused planes): a
    // conditional fetch makes the wait-count merge stall on the fresh loads
    fetch(zs + ahead, off_s, rn);
    C g[Q], Fs[3];
    collide(rc, g, Fs);
    stage(g, wv, lane + 1);
    __syncthreads();
    // c_z = -1 populations complete destination plane zs-1
    static_for<Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (L::cz(i) == -1) {
        if constexpr (i < NP)
          accumulate<Q, i>(acc, pulled(I));
        else
          accumulate<Q, i>(acc, g[i]);
      }
    });
    {
      // Every iteration issues the same ten stores (uniform memory-op counts
      // keep the wait counters precise); lanes with nothing to store -- planes
      // outside the chunk, ragged tails -- use an offset at the end of the
      // plane, which the buffer range check discards.
      C out[10];
      finalize<Q, C>(acc, Fd[0], Fd[1], Fd[2], out);
      const bool live = zs - 1 >= z0 && zs - 1 < z1;
      const int64_t pb = static_cast<int64_t>(live ? zs - 1 : z0) * plane;
      const uint32_t off = (store_ok && live) ? off_d : plane_bytes;
#pragma unroll
      for (int k = 0; k < 10; ++k)
        S::store_at(plane_rsrc(dst + (k * N + pb), plane_bytes), off, out[k], a.inv_scale[k]);
    }
    // destination plane zs: the c_z=+1 populations from zs-1, then c_z = 0
    zero(acc);
    {
      int u = 0;
      static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (L::cz(i) == 1) accumulate<Q, i>(acc, up[u++]);
      });
    }
    static_for<Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (L::cz(i) == 0) {
        if constexpr (i < NP)
          accumulate<Q, i>(acc, pulled(I));
        else
          accumulate<Q, i>(acc, g[i]);
      }
    });
    if constexpr (WALLY) {
      // halfway bounce-back: a population that would come from beyond the
      // wall is the opposite one leaving x itself at the same time level
      if (wall_lo)
        static_for<Q>([&](auto I) {
          constexpr int i = decltype(I)::value;
          if constexpr (L::cy(i) == 1) accumulate<Q, i>(acc, g[L::opp(i)]);
        });
      if (wall_hi)
        static_for<Q>([&](auto I) {
          constexpr int i = decltype(I)::value;
          if constexpr (L::cy(i) == -1) accumulate<Q, i>(acc, g[L::opp(i)]);
        });
    }
    Fd[0] = Fs[0];
    Fd[1] = Fs[1];
    Fd[2] = Fs[2];
    // c_z = +1 populations for destination plane zs+1
    {
      int u = 0;
      static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (L::cz(i) == 1) {
          if constexpr (i < NP)
            up[u++] = pulled(I);
          else
            up[u++] = g[i];
        }
      });
    }
    __syncthreads();
  };

  // Halo waves: their own y-halo row, plus one x-halo column site per lane
  // (lanes 0..R-1).  To balance the two phases of a plane against the
  // interior waves (collide, then pull + project), the column site of plane
  // zs+1 is collided during phase 2 of plane zs into colbuf, and copied into
  // the plane's column slots during phase 1 of zs+1 (same lane writes and
  // reads colbuf, so it needs no barrier of its own).
  const int hwave = (wv == 0) ? 0 : 1;
  // lanes without an x-halo site fetch at the plane end: zeros, no fault
  const uint32_t off_hf = do_halo ? off_h : plane_bytes;
  auto col_to_buf = [&](const Raw& r) __attribute__((always_inline)) {
    C g[Q], Fs[3];
    collide(r, g, Fs);
    if (do_halo)
      static_for<NP>([&](auto I) {
        constexpr int i = decltype(I)::value;
        colbuf[i][hwave][lane] = g[i];
      });
  };
  // rc: this plane's row site, rn: receives plane zs+ahead; hc: the column
  // site of plane zs+1, refilled after use with plane zs+1+U
  auto body_halo = [&](const int zs, Raw& rc, Raw& rn, Raw& hc, const int ahead) __attribute__((always_inline)) {
    fetch(zs + ahead, off_s, rn);
    if (do_halo)
      static_for<NP>([&](auto I) {
        constexpr int i = decltype(I)::value;
        lds[i][lane][hcol] = colbuf[i][hwave][lane];
      });
    {
      C g[Q], Fs[3];
      collide(rc, g, Fs);
      stage(g, wv, lane + 1);
    }
    __syncthreads();
    col_to_buf(hc);
    fetch(zs + 1 + (ahead + 1), off_hf, hc);
    __syncthreads();
  };

  // The role is uniform per wave; the two roles run separate loops so that
  // their loop-carried registers never coexist.  Both run the same padded
  // number of source planes (z0-1 .. z1, rounded up to a multiple of the
  // unroll U) with exactly two barriers each; padded planes compute values
  // that are never stored.  Every path through a loop trip issues the same
  // memory operations, which keeps the compiler's wait counts exact.
  constexpr int PF = LBF_PREFETCH_DEPTH;  // planes of moments in flight
  constexpr int U = PF + 1;               // rotating raw buffers = unroll
  const int trips = ((z1 - z0 + 2) + U - 1) / U;
  const bool interior_wave = __builtin_amdgcn_readfirstlane(static_cast<int>(interior)) != 0;
  if (interior_wave) {
    Sums<C> acc;
    zero(acc);
    C up[NU], Fd[3] = {C(0), C(0), C(0)};
#pragma unroll
    for (int u = 0; u < NU; ++u) up[u] = C(0);
    Raw rr[U];
    static_for<PF>([&](auto J) { fetch(z0 - 1 + J, off_s, rr[J]); });
#pragma unroll 1
    for (int t = 0; t < trips; ++t) {
      const int zb = z0 - 1 + t * U;
      static_for<U>([&](auto K) {
        constexpr int k = decltype(K)::value;
        body_interior(zb + k, acc, up, Fd, rr[k], rr[(k + PF) % U], PF);
      });
    }
  } else {
    Raw rr[U], hh[U];
    {
      Raw first;
      fetch(z0 - 1, off_hf, first);
      col_to_buf(first);  // columns of the first source plane
    }
    static_for<U>([&](auto J) { fetch(z0 + J, off_hf, hh[J]); });
    static_for<PF>([&](auto J) { fetch(z0 - 1 + J, off_s, rr[J]); });
#pragma unroll 1
    for (int t = 0; t < trips; ++t) {
      const int zb = z0 - 1 + t * U;
      static_for<U>([&](auto K) {
        constexpr int k = decltype(K)::value;
        body_halo(zb + k, rr[k], rr[(k + PF) % U], hh[k], PF);
      });
    }
  }
}

// LDS bytes of one workgroup: NP staged populations x (TY+2) rows x 66 columns
template <int Q, int ST, int TY>
constexpr size_t lds_bytes() {
  return sizeof(typename Storage<ST>::C) * Lat<Q>::NP * (TY + 2) * 66;
}
constexpr size_t kLdsLimit = 160 * 1024;

template <int Q, int ST, int TY, bool WALLY, bool FFIELD>
hipError_t launch_step_t(const StepArgs& a, hipStream_t stream) {
  if constexpr (lds_bytes<Q, ST, TY>() > kLdsLimit) {
    return hipErrorInvalidConfiguration;
  } else {
    const int nb = a.tiles_x * a.tiles_y * a.zchunks;
    hipLaunchKernelGGL((step_kernel<Q, ST, TY, WALLY, FFIELD>), dim3(nb), dim3(64 * (TY + 2)), 0,
                       stream, a);
    return hipGetLastError();
  }
}

// all (Q, tile rows, walls, force field) variants of one storage type
template <int ST>
hipError_t launch_step_storage(int Q, int tile_rows, bool walls_y, bool ffield, const StepArgs& a,
                               hipStream_t s) {
#define LBF_CASE(QQ, TYY)                                                          \
  if (Q == QQ && tile_rows == TYY) {                                              \
    if (walls_y)                                                                  \
      return ffield ? launch_step_t<QQ, ST, TYY, true, true>(a, s)                \
                    : launch_step_t<QQ, ST, TYY, true, false>(a, s);              \
    return ffield ? launch_step_t<QQ, ST, TYY, false, true>(a, s)                 \
                  : launch_step_t<QQ, ST, TYY, false, false>(a, s);               \
  }
  LBF_CASE(19, 4)
  LBF_CASE(19, 6)
  LBF_CASE(19, 8)
  LBF_CASE(19, 14)
  LBF_CASE(27, 4)
  LBF_CASE(27, 6)
  LBF_CASE(27, 8)
  LBF_CASE(27, 14)
#undef LBF_CASE
  return hipErrorInvalidValue;
}

}  // namespace lbf
