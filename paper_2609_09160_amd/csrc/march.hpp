// march.hpp -- the z-marching pull-stencil skeleton shared by the fused step
// (step_kernel.hpp) and its discrete adjoint (adjoint_kernel.hpp).
//
// Both kernels have the same shape: every site evaluates Q values that travel
// to its neighbours ("populations": value i leaves site y towards y + c_i),
// every site gathers the Q values that arrive from y - c_i (periodic wrap, or
// halfway bounce-back at the y walls: a value that would arrive from beyond a
// wall is replaced by the opposite value leaving the site itself), and
// projects them on the Hermite basis H0, H1, H2 (running sums s0, j, p).
// What the sites compute from their inputs and what they write from the sums
// is the physics policy P:
//
//   P::Q                      velocity set (19 or 27)
//   P::C, P::T                compute type, element type of the site offsets
//   P::Raw<OWN>               per-site inputs (OWN: the site is also a
//                             destination of this workgroup; halo sites
//                             only act as sources)
//   P::Carry                  per-site data a source hands to its own
//                             destination one plane later
//   P::fetch<OWN, S>(a, pb, off, plane_bytes, raw[S])   S consecutive sites
//   P::source<OWN, SEL>(a, raw, g[Q], carry)   g in units of 1/D (D =
//                             Lat<Q>::D); halo sites (SEL != kSelAll) only
//                             need the directions that enter the tile
//   P::finish<S>(a, sums[S], carry[S], pb, off, plane_bytes)   store S
//                             consecutive destinations
//   P::kStencil               the destinations also need the gradient and
//                             Laplacian of a scalar field (stencil.hpp):
//                             every source site hands P::scalar(raw), the
//                             skeleton stages it in LDS beside the values,
//                             accumulates the stencils along z and passes
//                             them to P::finish<S>(a, sums, carry, st[S], ...)
//
// gfx950 mapping (own design; the paper's 8x8x8 shared-memory tiles are prior
// art for another GPU):
//   * a workgroup owns a 64 S x TY column tile of the x-y plane (S = 1, 2 or
//     3 consecutive x-sites per lane, loaded and stored as one 1-, 2- or
//     3-wide access) and a chunk of z-planes, and marches through z;
//   * wave w (0..TY+1) handles tile row w-1; waves 0 and TY+1 are the y-halo
//     rows and also compute the two x-halo columns (lanes 0..TY+1);
//   * per source plane, every thread evaluates its own sites once and writes
//     the values that leave their (x, y) columns (16 for D3Q19, 24 for D3Q27)
//     to LDS; after a barrier each interior thread pulls the 3x3 column
//     neighbourhoods from LDS;
//   * values travelling along z stay in registers: the ones with c_z=+1 wait
//     one plane, the ones with c_z=-1 complete the previous plane, so each
//     input is read from HBM once per update (plus L2-resident halos) and each
//     output written once, with no population array anywhere;
//   * block ids can be remapped so that each XCD (own L2) gets a contiguous
//     range of tiles, y-neighbours first (a.xcd_remap); the host chooses the
//     order per storage form, from measurement.
#pragma once

#ifndef LBF_PREFETCH_DEPTH
#define LBF_PREFETCH_DEPTH 1
#endif

#include "internal.hpp"
#include "lattice.hpp"
#include "stencil.hpp"

namespace lbf {

// Which values a source site has to produce: all of them (sites the
// workgroup owns), or only those that enter the tile from a halo site: c_y =
// +1 from the halo row below, c_y = -1 from the row above, c_x = +1 from the
// halo column on the left, c_x = -1 from the one on the right.
enum { kSelAll = 0, kSelUp = 1, kSelDown = 2, kSelRight = 3, kSelLeft = 4 };
template <int SEL>
constexpr bool selected(int cx, int cy) {
  return SEL == kSelAll || (SEL == kSelUp && cy == 1) || (SEL == kSelDown && cy == -1) ||
         (SEL == kSelRight && cx == 1) || (SEL == kSelLeft && cx == -1);
}
template <int Q, int SEL>
constexpr bool selected_dir(int i) {
  return selected<SEL>(Lat<Q>::cx(i), Lat<Q>::cy(i));
}

// Values leaving one site along each direction, in units of 1/D, from the
// coefficients of the expansion
//   g_i = k_i [A + sum_a D_a c_ia^2 + sum_{a<b} O_ab c_ia c_ib + sum_a V_a c_ia],
// k_i = D w_i (only the directions SEL selects are written).
template <int Q, typename C, int SEL = kSelAll>
__device__ __forceinline__ void expand(C A, C Dx, C Dy, C Dz, C Oxy, C Oxz, C Oyz, C Vx, C Vy,
                                       C Vz, C g[Q]) {
  using L = Lat<Q>;
  static_for<Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr (!selected_dir<Q, SEL>(i)) return;
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

// Running projections of the arriving values (units of 1/D) on H0 (s0),
// H1 (j) and c c (p), so that values can be folded in as they arrive.
template <typename C>
struct Sums {
  C s0, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
};

template <typename C>
__device__ __forceinline__ void zero(Sums<C>& S) {
  S.s0 = S.jx = S.jy = S.jz = S.pxx = S.pyy = S.pzz = S.pxy = S.pxz = S.pyz = C(0);
}

// add value v arriving along direction i
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

template <class P, int TY, bool WALLY, int S>
__global__ void __launch_bounds__(64 * (TY + 2)) march_kernel(const StepArgs a) {
  constexpr int Q = P::Q;
  using L = Lat<Q>;
  using C = typename P::C;
  using T = typename P::T;
  using RawOwn = typename P::template Raw<true>;
  using RawHalo = typename P::template Raw<false>;
  using Carry = typename P::Carry;
  constexpr int NP = L::NP;
  constexpr int R = TY + 2;       // LDS rows: tile rows plus the two y-halo rows
  constexpr int TW = 64 * S;      // tile width: S consecutive x-sites per lane
  constexpr int W = TW + 2;       // LDS columns: the tile plus the two x-halo columns
  __shared__ C lds[NP][R][W];
  __shared__ C colbuf[NP][2][R];  // next plane's x-halo columns (halo waves)
  // the stencil's scalar of the source plane, and of the next plane's x-halo
  // columns (same rows and columns as the staged values)
  constexpr bool KS = P::kStencil;
  __shared__ C sgl[KS ? R : 1][KS ? W : 1];
  __shared__ C sgcol[KS ? 2 : 1][KS ? R : 1];

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;  // LDS row of this wave's sites
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int64_t plane = static_cast<int64_t>(nx) * ny;

  // Logical tile order: y fastest, then x, then z chunk.  Hardware hands
  // consecutive block ids to the 8 XCDs in turn; with a.xcd_remap each XCD
  // gets a contiguous range of tiles instead (y-neighbours on one L2).
  const int nb = static_cast<int>(gridDim.x), b0 = static_cast<int>(blockIdx.x);
  int b = b0;
  if (a.xcd_remap) {
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b0 & 7;
    b = xcd * q8 + (xcd < r8 ? xcd : r8) + (b0 >> 3);
  }
  const int tyi = b % a.tiles_y;
  b /= a.tiles_y;
  const int txi = b % a.tiles_x;
  const int zci = b / a.tiles_x;
  const int x0 = txi * TW, y0 = tyi * TY;
  const int z0 = zci * a.zchunk;
  const int z1 = min(z0 + a.zchunk, nz);

  // In-plane byte offsets are 32-bit (the host enforces nx*ny*8 < 2^32); the
  // per-plane base pointers are uniform, so every load and store is a scalar
  // base plus one vector offset.  With S = 2 the host guarantees an even nx,
  // so a lane's two sites never straddle the periodic wrap.
  // own source sites (every lane computes valid, possibly wrapped, sites)
  const int xs = pmod(x0 + S * lane, nx);
  const int ys = WALLY ? clampi(y0 + wv - 1, 0, ny - 1) : pmod(y0 + wv - 1, ny);
  const uint32_t off_s = (static_cast<uint32_t>(ys) * static_cast<uint32_t>(nx) + xs) * sizeof(T);
  // x-halo site: wave 0 takes the left column, wave R-1 the right one
  const bool do_halo = (wv == 0 || wv == R - 1) && lane < R;
  const int hcol = (wv == 0) ? 0 : W - 1;
  const int xh = pmod(wv == 0 ? x0 - 1 : x0 + TW, nx);
  const int yh = WALLY ? clampi(y0 - 1 + lane, 0, ny - 1) : pmod(y0 - 1 + lane, ny);
  const uint32_t off_h = (static_cast<uint32_t>(yh) * static_cast<uint32_t>(nx) + xh) * sizeof(T);
  // destinations
  const bool interior = (wv >= 1 && wv <= TY);
  const int xd = x0 + S * lane, yd = y0 + wv - 1;
  const bool store_ok = interior && xd < nx && yd < ny;
  const uint32_t off_d = (static_cast<uint32_t>(yd) * static_cast<uint32_t>(nx) + xd) * sizeof(T);
  const bool wall_lo = WALLY && interior && yd == 0;
  const bool wall_hi = WALLY && interior && yd == ny - 1;

  const uint32_t plane_bytes = static_cast<uint32_t>(plane * sizeof(T));
  // periodic plane index for zs >= -1 (zs is uniform: scalar arithmetic;
  // planes past the end of a padded chunk are fetched but never used)
  auto zwrap = [&](int zs) __attribute__((always_inline)) {
    zs = zs < 0 ? zs + nz : zs;
    zs = zs >= nz ? zs - nz : zs;
    return zs >= nz ? zs % nz : zs;
  };
  auto fetch_own = [&](const int zs, const uint32_t off, RawOwn (&r)[S]) __attribute__((always_inline)) {
    P::template fetch<true, S>(a, static_cast<int64_t>(zwrap(zs)) * plane, off, plane_bytes, r);
  };
  auto fetch_row = [&](const int zs, const uint32_t off, RawHalo (&r)[S]) __attribute__((always_inline)) {
    P::template fetch<false, S>(a, static_cast<int64_t>(zwrap(zs)) * plane, off, plane_bytes, r);
  };
  auto fetch_col = [&](const int zs, const uint32_t off, RawHalo (&r)[1]) __attribute__((always_inline)) {
    P::template fetch<false, 1>(a, static_cast<int64_t>(zwrap(zs)) * plane, off, plane_bytes, r);
  };
  auto stage = [&](auto SEL, const C g[Q], const int row, const int col)
                   __attribute__((always_inline)) {
    static_for<NP>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (selected_dir<Q, decltype(SEL)::value>(i)) lds[i][row][col] = g[i];
    });
  };
  using SelAll = std::integral_constant<int, kSelAll>;
  // value i arriving at the destination of own site s from the LDS plane; on
  // a wall row the ones that would come from beyond the wall are dropped here
  // and replaced by the reflections added in body_interior
  auto pulled = [&](auto I, const int s) __attribute__((always_inline)) -> C {
    constexpr int i = decltype(I)::value;
    C v = lds[i][wv - L::cy(i)][S * lane + s + 1 - L::cx(i)];
    if constexpr (WALLY && L::cy(i) == 1) v = wall_lo ? C(0) : v;
    if constexpr (WALLY && L::cy(i) == -1) v = wall_hi ? C(0) : v;
    return v;
  };

  // Interior waves, one source plane zs per call.  acc[s]: running sums of
  // destination plane zs-1 (all but its c_z=-1 values), completed and stored
  // here; up[s]: the c_z=+1 values that reach plane zs from zs-1; cd[s]: the
  // carry of the own site of plane zs-1.  rc holds this plane's inputs, rn
  // receives the next plane's (one plane of latency hiding).  The values along
  // the three column directions (rest, c_z = +-1) never leave the thread and
  // stay in registers (gc).
  constexpr int NU = (Q == 19) ? 5 : 9;  // directions with c_z = +1
  auto body_interior = [&](const int zs, Sums<C> (&acc)[S], C (&up)[S][NU], Carry (&cd)[S],
                           StencilRoll<C> (&sr)[S], RawOwn (&rc)[S], RawOwn (&rn)[S],
                           const int ahead) __attribute__((always_inline)) {
    // unconditional (the last planes of a chunk fetch unused planes): a
    // conditional fetch makes the wait-count merge stall on the fresh loads
    fetch_own(zs + ahead, off_s, rn);
    C gc[S][3];
    Carry cs[S];
    static_for<S>([&](auto SI) {
      constexpr int s = decltype(SI)::value;
      C g[Q];
      P::template source<true, kSelAll>(a, rc[s], g, cs[s]);
      stage(SelAll{}, g, wv, S * lane + s + 1);
      if constexpr (KS) sgl[wv][S * lane + s + 1] = P::scalar(rc[s]);
      gc[s][0] = g[L::kRest];
      gc[s][1] = g[L::kUp];
      gc[s][2] = g[L::kDown];
    });
    __syncthreads();
    auto own = [&](auto I, const int s) __attribute__((always_inline)) -> C {
      constexpr int i = decltype(I)::value;
      if constexpr (i < NP)
        return pulled(I, s);
      else
        return gc[s][i - NP];
    };
    // c_z = -1 values complete destination plane zs-1
    static_for<S>([&](auto SI) {
      constexpr int s = decltype(SI)::value;
      static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (L::cz(i) == -1) accumulate<Q, i>(acc[s], own(I, s));
      });
    });
    {
      // Every iteration issues the same stores (uniform memory-op counts keep
      // the wait counters precise); lanes with nothing to store -- planes
      // outside the chunk, ragged tails -- use an offset at the end of the
      // plane, which the buffer range check discards.
      const bool live = zs - 1 >= z0 && zs - 1 < z1;
      const int64_t pb = static_cast<int64_t>(live ? zs - 1 : z0) * plane;
      const uint32_t off = (store_ok && live) ? off_d : plane_bytes;
      if constexpr (KS) {
        // this plane's 3 x 3 windows complete the stencils of plane zs - 1
        StencilOut<C> so[S];
        static_for<S>([&](auto SI) {
          constexpr int s = decltype(SI)::value;
          const int col = S * lane + s;
          C n[3][3];
#pragma unroll
          for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) n[dy][dx] = sgl[wv - 1 + dy][col + dx];
          so[s] = sr[s].plane(n);
        });
        P::template finish<S>(a, acc, cd, so, pb, off, plane_bytes);
      } else {
        P::template finish<S>(a, acc, cd, pb, off, plane_bytes);
      }
    }
    static_for<S>([&](auto SI) {
      constexpr int s = decltype(SI)::value;
      // destination plane zs: the c_z=+1 values from zs-1, then c_z = 0
      zero(acc[s]);
      {
        int u = 0;
        static_for<Q>([&](auto I) {
          constexpr int i = decltype(I)::value;
          if constexpr (L::cz(i) == 1) accumulate<Q, i>(acc[s], up[s][u++]);
        });
      }
      static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (L::cz(i) == 0) accumulate<Q, i>(acc[s], own(I, s));
      });
      if constexpr (WALLY) {
        // halfway bounce-back: a value that would come from beyond the wall is
        // the opposite one leaving x itself at the same time level (its own
        // LDS slot: every direction with c_y != 0 is staged)
        const int col = S * lane + s + 1;
        if (wall_lo)
          static_for<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (L::cy(i) == 1) accumulate<Q, i>(acc[s], lds[L::opp(i)][wv][col]);
          });
        if (wall_hi)
          static_for<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (L::cy(i) == -1) accumulate<Q, i>(acc[s], lds[L::opp(i)][wv][col]);
          });
      }
      cd[s] = cs[s];
      // c_z = +1 values for destination plane zs+1
      {
        int u = 0;
        static_for<Q>([&](auto I) {
          constexpr int i = decltype(I)::value;
          if constexpr (L::cz(i) == 1) up[s][u++] = own(I, s);
        });
      }
    });
    __syncthreads();
  };

  // Halo waves: their own y-halo row, plus one x-halo column site per lane
  // (lanes 0..R-1).  To balance the two phases of a plane against the
  // interior waves (evaluate, then pull + project), the column site of plane
  // zs+1 is evaluated during phase 2 of plane zs into colbuf, and copied into
  // the plane's column slots during phase 1 of zs+1 (same lane writes and
  // reads colbuf, so it needs no barrier of its own).  A halo site evaluates
  // only the values that enter the tile (RS for the row, CS for the column:
  // wave 0 holds the row below and the left column, wave R-1 the row above and
  // the right column).
  const int hwave = (wv == 0) ? 0 : 1;
  // lanes without an x-halo site fetch at the plane end: zeros, no fault
  const uint32_t off_hf = do_halo ? off_h : plane_bytes;
  auto col_to_buf = [&](auto CS, const RawHalo& r) __attribute__((always_inline)) {
    constexpr int cs_sel = decltype(CS)::value;
    C g[Q];
    Carry cs;
    P::template source<false, cs_sel>(a, r, g, cs);
    if (do_halo) {
      static_for<NP>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (selected_dir<Q, cs_sel>(i)) colbuf[i][hwave][lane] = g[i];
      });
      if constexpr (KS) sgcol[hwave][lane] = P::scalar(r);
    }
  };
  // rc: this plane's row sites, rn: receives plane zs+ahead; hc: the column
  // site of plane zs+1, refilled after use with plane zs+1+U
  auto body_halo = [&](auto RS, auto CS, const int zs, RawHalo (&rc)[S], RawHalo (&rn)[S],
                       RawHalo (&hc)[1], const int ahead) __attribute__((always_inline)) {
    constexpr int rs_sel = decltype(RS)::value, cs_sel = decltype(CS)::value;
    fetch_row(zs + ahead, off_s, rn);
    if (do_halo) {
      static_for<NP>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (selected_dir<Q, cs_sel>(i)) lds[i][lane][hcol] = colbuf[i][hwave][lane];
      });
      if constexpr (KS) sgl[lane][hcol] = sgcol[hwave][lane];
    }
    static_for<S>([&](auto SI) {
      constexpr int s = decltype(SI)::value;
      C g[Q];
      Carry cs;
      P::template source<false, rs_sel>(a, rc[s], g, cs);
      stage(RS, g, wv, S * lane + s + 1);
      if constexpr (KS) sgl[wv][S * lane + s + 1] = P::scalar(rc[s]);
    });
    __syncthreads();
    col_to_buf(CS, hc[0]);
    fetch_col(zs + 1 + (ahead + 1), off_hf, hc);
    __syncthreads();
  };

  // The role is uniform per wave; the two roles run separate loops so that
  // their loop-carried registers never coexist.  Both run the same padded
  // number of source planes (z0-1 .. z1, rounded up to a multiple of the
  // unroll U) with exactly two barriers each; padded planes compute values
  // that are never stored.  Every path through a loop trip issues the same
  // memory operations, which keeps the compiler's wait counts exact.
  constexpr int PF = LBF_PREFETCH_DEPTH;  // planes of inputs in flight
  constexpr int U = PF + 1;               // rotating raw buffers = unroll
  const int trips = ((z1 - z0 + 2) + U - 1) / U;
  const bool interior_wave = __builtin_amdgcn_readfirstlane(static_cast<int>(interior)) != 0;
  if (interior_wave) {
    Sums<C> acc[S];
    C up[S][NU];
    Carry cd[S];
    StencilRoll<C> sr[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      zero(acc[s]);
      P::clear(cd[s]);
      sr[s].clear();
#pragma unroll
      for (int u = 0; u < NU; ++u) up[s][u] = C(0);
    }
    RawOwn rr[U][S];
    static_for<PF>([&](auto J) { fetch_own(z0 - 1 + J, off_s, rr[J]); });
#pragma unroll 1
    for (int t = 0; t < trips; ++t) {
      const int zb = z0 - 1 + t * U;
      static_for<U>([&](auto K) {
        constexpr int k = decltype(K)::value;
        body_interior(zb + k, acc, up, cd, sr, rr[k], rr[(k + PF) % U], PF);
      });
    }
  } else {
    auto halo_loop = [&](auto RS, auto CS) __attribute__((always_inline)) {
      RawHalo rr[U][S], hh[U][1];
      {
        RawHalo first[1];
        fetch_col(z0 - 1, off_hf, first);
        col_to_buf(CS, first[0]);  // columns of the first source plane
      }
      static_for<U>([&](auto J) { fetch_col(z0 + J, off_hf, hh[J]); });
      static_for<PF>([&](auto J) { fetch_row(z0 - 1 + J, off_s, rr[J]); });
#pragma unroll 1
      for (int t = 0; t < trips; ++t) {
        const int zb = z0 - 1 + t * U;
        static_for<U>([&](auto K) {
          constexpr int k = decltype(K)::value;
          body_halo(RS, CS, zb + k, rr[k], rr[(k + PF) % U], hh[k], PF);
        });
      }
    };
    // uniform per wave: each halo wave runs one of the two loops, with the
    // same trips and barriers
    if (wv == 0)
      halo_loop(std::integral_constant<int, kSelUp>{}, std::integral_constant<int, kSelRight>{});
    else
      halo_loop(std::integral_constant<int, kSelDown>{}, std::integral_constant<int, kSelLeft>{});
  }
}

// LDS bytes of one workgroup: NP staged values x (TY+2) rows x (64 S + 2)
// columns, plus the x-halo column buffer (NP x 2 x (TY+2)); a stencil's
// scalar takes one more such slot
template <int Q, typename C, int TY, int S, bool KS = false>
constexpr size_t march_lds_bytes() {
  return sizeof(C) * (Lat<Q>::NP + (KS ? 1 : 0)) * (TY + 2) * (64 * S + 2 + 2);
}
constexpr size_t kLdsLimit = 160 * 1024;

template <class P, int TY, bool WALLY, int S>
hipError_t launch_march_s(const StepArgs& a, hipStream_t stream) {
  if constexpr (march_lds_bytes<P::Q, typename P::C, TY, S, P::kStencil>() > kLdsLimit) {
    return hipErrorInvalidConfiguration;
  } else {
    const int nb = a.tiles_x * a.tiles_y * a.zchunks;
    hipLaunchKernelGGL((march_kernel<P, TY, WALLY, S>), dim3(nb), dim3(64 * (TY + 2)), 0, stream,
                       a);
    return hipGetLastError();
  }
}

// one, two or three consecutive x-sites per lane (a.lane_sites); the two-
// and three-site forms exist for tiles of up to 8 rows (taller ones measured
// slower), the three-site form (192-wide tiles) for 4-byte storage
template <class P, int TY, bool WALLY>
hipError_t launch_march(const StepArgs& a, hipStream_t stream) {
  if (a.lane_sites == 2) {
    if constexpr (TY <= 8) return launch_march_s<P, TY, WALLY, 2>(a, stream);
    return hipErrorInvalidValue;
  }
  if (a.lane_sites == 3) {
    if constexpr (TY <= 8 && sizeof(typename P::T) == 4 && P::kThreeSites)
      return launch_march_s<P, TY, WALLY, 3>(a, stream);
    return hipErrorInvalidValue;
  }
  if (a.lane_sites != 1) return hipErrorInvalidValue;
  return launch_march_s<P, TY, WALLY, 1>(a, stream);
}

}  // namespace lbf
