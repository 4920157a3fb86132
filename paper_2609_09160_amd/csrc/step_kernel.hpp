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
// D3Q27h (kD3Q27H) replaces step 2's second-order series by the complete
// D3Q27 Hermite basis (source_pops_full below); steps 3-5 are unchanged.
//
// The launch is the z-march of march.hpp (LDS-staged pull, populations never
// stored) with the Forward policy below.
#pragma once

#include "march.hpp"

namespace lbf {

// Steps 1-2 at one source site: post-collision coefficients and the
// reconstructed populations, kept in units of 1/D: g[i] = D f_i(y) with
// D f_i = k_i [P0 - 1.5 tr P2 + 3 c.P1 + 4.5 c c : P2], k_i = D w_i.
// m[4..9] hold, by NEQ: kTotal, the total a2; kDev, a2 - u u (deviation
// storage); kDevRelaxed, (1 - omega)(a2 - u u).
// HASF = false: no force anywhere (uniform zero force, no field); the force
// terms, identically zero, are left out.
enum { kTotal = 0, kDev = 1, kDevRelaxed = 2 };
template <int Q, typename C, int SEL = kSelAll, int NEQ = kTotal, bool HASF = true>
__device__ __forceinline__ void source_pops(const C m[10], C Fx, C Fy, C Fz, C omega, C g[Q]) {
  const C h = C(0.5);
  const C om1 = C(1) - omega;
  const C ux = m[1], uy = m[2], uz = m[3];
  // P2 = u u + (1 - omega)(a2 - u u) + (u F + F u)/2
  C P2xx, P2yy, P2zz, P2xy, P2xz, P2yz;
  if constexpr (NEQ == kDevRelaxed) {
    P2xx = ux * ux + m[4];
    P2yy = uy * uy + m[5];
    P2zz = uz * uz + m[6];
    P2xy = ux * uy + m[7];
    P2xz = ux * uz + m[8];
    P2yz = uy * uz + m[9];
  } else if constexpr (NEQ == kDev) {
    P2xx = ux * ux + om1 * m[4];
    P2yy = uy * uy + om1 * m[5];
    P2zz = uz * uz + om1 * m[6];
    P2xy = ux * uy + om1 * m[7];
    P2xz = ux * uz + om1 * m[8];
    P2yz = uy * uz + om1 * m[9];
  } else {
    P2xx = omega * ux * ux + om1 * m[4];
    P2yy = omega * uy * uy + om1 * m[5];
    P2zz = omega * uz * uz + om1 * m[6];
    P2xy = omega * ux * uy + om1 * m[7];
    P2xz = omega * ux * uz + om1 * m[8];
    P2yz = omega * uy * uz + om1 * m[9];
  }
  C Vx = C(3) * ux, Vy = C(3) * uy, Vz = C(3) * uz;
  if constexpr (HASF) {
    P2xx += ux * Fx;
    P2yy += uy * Fy;
    P2zz += uz * Fz;
    P2xy += h * (ux * Fy + uy * Fx);
    P2xz += h * (ux * Fz + uz * Fx);
    P2yz += h * (uy * Fz + uz * Fy);
    Vx = C(3) * (ux + h * Fx), Vy = C(3) * (uy + h * Fy), Vz = C(3) * (uz + h * Fz);
  }
  // scaled coefficients of the reconstruction (cs^2 = 1/3)
  const C A = m[0] - C(1.5) * (P2xx + P2yy + P2zz);
  const C Dx = C(4.5) * P2xx, Dy = C(4.5) * P2yy, Dz = C(4.5) * P2zz;
  const C Oxy = C(9) * P2xy, Oxz = C(9) * P2xz, Oyz = C(9) * P2yz;
  expand<Q, C, SEL>(A, Dx, Dy, Dz, Oxy, Oxz, Oyz, Vx, Vy, Vz, g);
}

// D3Q27h, steps 1-2 over the complete Hermite basis of D3Q27 (section 2,
// after Eq. (9): orders up to 6, coefficients of order >= 3 by the recursive
// closures of Shan et al. and Malaspinas).  Evaluated in tensor-product form
// rather than order by order: on D3Q27 the complete basis factorises per axis,
// the equilibrium coefficients u...u make the equilibrium part the product
// G_i = prod_a g(c_ia; u_a) of D1Q3 equilibria (unit density), and the
// recursive non-equilibrium closure, a sum over index pairs of a2neq times the
// remaining velocities, makes the relaxed part (1 - omega) (1/2) B : grad_u
// grad_u G_i with B = a2 - u u.  So
//   f_i = w_i p* + (G_i - w_i) + (1 - omega) N_i + S_i / 2,
// S_i the Guo term of Eq. (9) (orders 1 and 2 only).
//
// Per axis, scaled by 3 so that a product of three factors carries the 1/D
// units (D = 27), at c = -1, 0, 1 (array index c + 1):
//   W = 3 w1d(c)                  (1/2, 2, 1/2)
//   e = 3 g(c; u) - W             (3/2 (u^2 - u), -3 u^2, 3/2 (u^2 + u))
//   E = W + e,  d = 3 dg/du       (3 u - 3/2, -6 u, 3 u + 3/2)
//   s = (3/2) d2g/du2             (3/2, -3, 3/2).
// For one (c_x, c_y) column the three populations c_z = -1, 0, 1 are a
// quadratic in c_z, K0 + K1 c_z + K2 c_z^2; gathering the z factors' values
// into that form gives, with the column coefficients
//   Exy = E_x E_y,  P = E_x E_y - W_x W_y = e_x E_y + W_x e_y,
//   al  = B_xx s_x E_y + B_yy E_x s_y + B_xy d_x d_y,
//   gam = B_xz d_x E_y + B_yz E_x d_y,  bet = B_zz Exy + W_x W_y M_zz,
//   A   = W_x W_y [p* + 3/2 (c_x F_x + c_y F_y) + 9/2 (M_xx (c_x^2 - 1/3)
//         + M_yy (c_y^2 - 1/3)) + 9 M_xy c_x c_y],
//   Bf  = W_x W_y [3/2 F_z + 9 (M_xz c_x + M_yz c_y)],   M = (u F + F u)/2,
// and Q1 = P + al + A, Q2 = Exy + al, R = 3/2 u_z^2 Q2 + 3/2 bet + 3 u_z gam:
//   f(c_z = 0)  = 2 (Q1 - R),
//   f(c_z = +-1) = Q1 / 2 + R +- (3/2 u_z Q2 + 3/2 gam + Bf / 2).
// Every intermediate is a deviation of order u, B or F (the rest weights
// cancel in P), so FP32 keeps its precision relative to the flow.
template <typename C, int SEL = kSelAll, int NEQ = kTotal, bool HASF = true>
__device__ __forceinline__ void source_pops_full(const C m[10], C Fx, C Fy, C Fz, C omega,
                                                 C g[27]) {
  using L = Lat<27>;
  const C h = C(0.5);
  const C om1 = C(1) - omega;
  const C ux = m[1], uy = m[2], uz = m[3];
  // (1 - omega) a2neq
  C Bxx, Byy, Bzz, Bxy, Bxz, Byz;
  if constexpr (NEQ == kDevRelaxed) {
    Bxx = m[4], Byy = m[5], Bzz = m[6];
    Bxy = m[7], Bxz = m[8], Byz = m[9];
  } else if constexpr (NEQ == kDev) {
    Bxx = om1 * m[4], Byy = om1 * m[5], Bzz = om1 * m[6];
    Bxy = om1 * m[7], Bxz = om1 * m[8], Byz = om1 * m[9];
  } else {
    Bxx = om1 * (m[4] - ux * ux), Byy = om1 * (m[5] - uy * uy);
    Bzz = om1 * (m[6] - uz * uz), Bxy = om1 * (m[7] - ux * uy);
    Bxz = om1 * (m[8] - ux * uz), Byz = om1 * (m[9] - uy * uz);
  }
  // Hermite coefficient of the Guo term, (u F + F u) / 2 (zero without force)
  C Mxx = C(0), Myy = C(0), Mzz = C(0), Mxy = C(0), Mxz = C(0), Myz = C(0);
  if constexpr (HASF) {
    Mxx = ux * Fx, Myy = uy * Fy, Mzz = uz * Fz;
    Mxy = h * (ux * Fy + uy * Fx), Mxz = h * (ux * Fz + uz * Fx);
    Myz = h * (uy * Fz + uz * Fy);
  }
  constexpr C W[3] = {C(0.5), C(2), C(0.5)};
  constexpr C sv[3] = {C(1.5), C(-3), C(1.5)};
  // per-axis factors of x and y, and their products with the column terms
  C ex[3], Ex[3], dx[3], ey[3], Ey[3], dy[3];
  {
    const C uxx = ux * ux, uyy = uy * uy;
    ex[0] = C(1.5) * (uxx - ux), ex[1] = C(-3) * uxx, ex[2] = C(1.5) * (uxx + ux);
    ey[0] = C(1.5) * (uyy - uy), ey[1] = C(-3) * uyy, ey[2] = C(1.5) * (uyy + uy);
    dx[0] = C(3) * ux - C(1.5), dx[1] = C(-6) * ux, dx[2] = C(3) * ux + C(1.5);
    dy[0] = C(3) * uy - C(1.5), dy[1] = C(-6) * uy, dy[2] = C(3) * uy + C(1.5);
#pragma unroll
    for (int c = 0; c < 3; ++c) Ex[c] = W[c] + ex[c], Ey[c] = W[c] + ey[c];
  }
  // p* and the x, y parts of the force term: 3/2 c F_a + 9/2 M_aa (c^2 - 1/3)
  C fx[3] = {C(0), C(0), C(0)}, fy[3] = {C(0), C(0), C(0)};
  if constexpr (HASF) {
    fx[0] = C(-1.5) * Fx + C(3) * Mxx, fx[1] = C(-1.5) * Mxx, fx[2] = C(1.5) * Fx + C(3) * Mxx;
    fy[0] = C(-1.5) * Fy + C(3) * Myy, fy[1] = C(-1.5) * Myy, fy[2] = C(1.5) * Fy + C(3) * Myy;
  }
  const C h2 = C(1.5) * uz * uz, h1 = C(1.5) * uz;
  static_for<9>([&](auto J) {
    constexpr int cx = decltype(J)::value / 3, cy = decltype(J)::value % 3;
    if constexpr (!selected<SEL>(cx - 1, cy - 1)) return;
    constexpr C WW = W[cx] * W[cy];
    constexpr C sx = (cx - 1) * C(9), sy = (cy - 1) * C(9), sxy = (cx - 1) * (cy - 1) * C(9);
    const C Exy = Ex[cx] * Ey[cy];
    const C P = ex[cx] * Ey[cy] + W[cx] * ey[cy];
    const C al = Bxx * sv[cx] * Ey[cy] + Byy * sv[cy] * Ex[cx] + Bxy * dx[cx] * dy[cy];
    const C gam = Bxz * dx[cx] * Ey[cy] + Byz * dy[cy] * Ex[cx];
    C bet = Bzz * Exy, A = WW * m[0], Bf = C(0);
    if constexpr (HASF) {
      bet += WW * Mzz;
      A = WW * (m[0] + fx[cx] + fy[cy] + sxy * Mxy);
      Bf = WW * (C(1.5) * Fz + sx * Mxz + sy * Myz);
    }
    const C Q1 = P + al + A;
    const C Q2 = Exy + al;
    const C R = h2 * Q2 + C(1.5) * bet + C(2) * h1 * gam;
    const C even = h * Q1 + R;
    C odd = h1 * Q2 + C(1.5) * gam;
    if constexpr (HASF) odd += h * Bf;
    g[L::index(cx - 1, cy - 1, 0)] = C(2) * (Q1 - R);
    g[L::index(cx - 1, cy - 1, 1)] = even + odd;
    g[L::index(cx - 1, cy - 1, -1)] = even - odd;
  });
}

// Steps 4-5 at one destination site: the running projections (units of 1/D)
// become the moments of the new time level, with the force-consistent
// correction.
template <int Q, typename C, bool HASF = true>
__device__ __forceinline__ void finalize(const Sums<C>& S, C Fx, C Fy, C Fz, C out[10]) {
  constexpr int D = Lat<Q>::D;
  const C h = C(0.5);
  C ux = div_by<D>(S.jx), uy = div_by<D>(S.jy), uz = div_by<D>(S.jz);
  if constexpr (HASF) ux += h * Fx, uy += h * Fy, uz += h * Fz;
  out[0] = div_by<D>(S.s0);
  out[1] = ux;
  out[2] = uy;
  out[3] = uz;
  // H2 diagonal: sum c_a^2 f - cs^2 sum f = (3 sum c_a^2 f - sum f) / 3
  out[4] = div_by<3 * D>(C(3) * S.pxx - S.s0);
  out[5] = div_by<3 * D>(C(3) * S.pyy - S.s0);
  out[6] = div_by<3 * D>(C(3) * S.pzz - S.s0);
  out[7] = div_by<D>(S.pxy);
  out[8] = div_by<D>(S.pxz);
  out[9] = div_by<D>(S.pyz);
  if constexpr (HASF) {
    out[4] += Fx * ux;
    out[5] += Fy * uy;
    out[6] += Fz * uz;
    out[7] += h * (Fx * uy + Fy * ux);
    out[8] += h * (Fx * uz + Fz * ux);
    out[9] += h * (Fy * uz + Fz * uy);
  }
}

// The forward step as a physics policy of the z-march: a site reads its 10
// stored moments (and the force), its values are the post-collision
// populations, and a destination writes its 10 new moments.  FNEXT: the force
// changes every step (two-component flow, section 2); the source uses F(t)
// from a field, and the correction of Eq. (8) at the destination uses
// F(t+1), which the destination computes itself from the gradient and
// Laplacian of phi(t+1) (the march's scalar stencil) and writes out as the
// next step's F(t):
//   F = mu grad(phi) + rho(phi) g,  mu = 4 beta phi (phi - 1)(phi - 1/2) - kappa lap(phi),
// with density contrast also - p* cs^2 grad(rho) - (nu omega / cs^2)(a2 - u u).grad(rho)
// (p*, a2 - u u of the site at t; the printed viscous term is garbled, this
// is the viscous stress written through the non-equilibrium coefficient of
// Eq. (6)).
// VAR: density and viscosity follow the phase field (section 2): the source
// relaxes with omega(phi(t)) and applies F(t) / rho(phi(t)), the correction
// applies F(t+1) / rho(phi(t+1)).
// FULL: D3Q27h, the source populations over the complete Hermite basis.
// NOF: no force at all (a zero uniform force and no field): the Guo source and
// the force terms of the correction vanish and are not evaluated.
template <int Q_, int ST, bool FFIELD, bool FNEXT = false, bool VAR = false, bool FULL = false,
          bool NOF = false>
struct Forward {
  static_assert(FFIELD || !FNEXT, "a time-dependent force is a force field");
  static_assert(FNEXT || !VAR, "variable properties come with the two-component force");
  static_assert(!FULL || Q_ == 27, "the complete Hermite basis is the D3Q27 one");
  static_assert(!NOF || !FFIELD, "no force means no force field");
  static constexpr int Q = Q_;
  using S = Storage<ST>;
  using C = typename S::C;
  using T = typename S::T;
  // 192-wide tiles (three x-sites per lane) are built for the one-component
  // second-order sets in FP32 storage
  static constexpr bool kThreeSites = ST == kF32 && !FNEXT && !FULL;
  static constexpr bool kStencil = FNEXT;  // grad and lap of phi(t+1)
  // raw (still encoded) moments and force of one site, fetched a plane ahead;
  // with a time-dependent force also phi(t+1) (the stencil's scalar) and,
  // with variable properties, phi(t)
  template <bool OWN>
  struct Raw {
    T m[S::kPlanes];
    C F[3];
    C sc;
    C ph;
  };
  template <bool OWN>
  static __device__ __forceinline__ C scalar(const Raw<OWN>& r) {
    return r.sc;
  }
  // handed from the source to the destination of the same site: the force
  // of the correction (static force), or what the contrast terms of F(t+1)
  // take from the state at t, the symmetric M = p* cs^2 I + (nu omega / cs^2)
  // (a2 - u u) with nu, omega of phi(t+1) (xx yy zz xy xz yz), so that they
  // are -M.grad(rho)
  struct Carry {
    C F[3];
    C M[(FNEXT && VAR) ? 6 : 1];
  };
  static __device__ __forceinline__ void clear(Carry& c) {
    c.F[0] = c.F[1] = c.F[2] = C(0);
#pragma unroll
    for (int k = 0; k < ((FNEXT && VAR) ? 6 : 1); ++k) c.M[k] = C(0);
  }

  // the 16-bit values of one site in a group of four planes, or a pair
  using T4 = T __attribute__((ext_vector_type(4)));
  using T2 = T __attribute__((ext_vector_type(2)));
  // the force field has the compute type; its byte offset scales accordingly
  static constexpr uint32_t kFscale = sizeof(C) / sizeof(T);

  template <bool OWN, int NS>
  static __device__ __forceinline__ void fetch(const StepArgs& a, int64_t pb, uint32_t off,
                                               uint32_t plane_bytes, Raw<OWN> (&r)[NS]) {
    const T* __restrict__ src = static_cast<const T*>(a.src);
    // 16-bit storage: planes 4j .. 4j + 3 as one 64-bit word per site, then
    // a pair as one 32-bit word (plane_elem)
    constexpr int kQ4 = S::kGrouped ? (S::kPlanes & ~3) : 0;
    constexpr int kQ2 = S::kGrouped ? kQ4 + (S::kPlanes & 2) : 0;
    if constexpr (S::kGrouped) {
#pragma unroll
      for (int j = 0; j < kQ4 / 4; ++j) {
        uint64_t w[NS];
        buf_load_n<uint64_t, NS>(
            plane_rsrc(reinterpret_cast<const uint64_t*>(src) + (j * a.N + pb), 4 * plane_bytes),
            4 * off, w);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const T4 h = __builtin_bit_cast(T4, w[s]);
          r[s].m[4 * j] = h.x;
          r[s].m[4 * j + 1] = h.y;
          r[s].m[4 * j + 2] = h.z;
          r[s].m[4 * j + 3] = h.w;
        }
      }
      if constexpr (kQ2 > kQ4) {
        uint32_t w[NS];
        buf_load_n<uint32_t, NS>(
            plane_rsrc(reinterpret_cast<const uint32_t*>(src) + (kQ4 / 2 * a.N + pb),
                       2 * plane_bytes),
            2 * off, w);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const T2 h = __builtin_bit_cast(T2, w[s]);
          r[s].m[kQ4] = h.x;
          r[s].m[kQ4 + 1] = h.y;
        }
      }
    }
#pragma unroll
    for (int k = kQ2; k < S::kPlanes; ++k) {
      T v[NS];
      buf_load_n<T, NS>(plane_rsrc(src + (k * a.N + pb), plane_bytes), off, v);
#pragma unroll
      for (int s = 0; s < NS; ++s) r[s].m[k] = v[s];
    }
    if constexpr (FFIELD) {
      const C* __restrict__ Ff = static_cast<const C*>(a.Ffield);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        C v[NS];
        buf_load_n<C, NS>(plane_rsrc(Ff + (k * a.N + pb), plane_bytes * kFscale), off * kFscale, v);
#pragma unroll
        for (int s = 0; s < NS; ++s) r[s].F[k] = v[s];
      }
    }
    if constexpr (FNEXT) {
      C v[NS];
      buf_load_n<C, NS>(plane_rsrc(static_cast<const C*>(a.phi_dst) + pb, plane_bytes * kFscale),
                        off * kFscale, v);
#pragma unroll
      for (int s = 0; s < NS; ++s) r[s].sc = v[s];
    }
    if constexpr (VAR) {
      C v[NS];
      buf_load_n<C, NS>(plane_rsrc(static_cast<const C*>(a.phi_src) + pb, plane_bytes * kFscale),
                        off * kFscale, v);
#pragma unroll
      for (int s = 0; s < NS; ++s) r[s].ph = v[s];
    }
  }

  template <bool OWN, int SEL>
  static __device__ __forceinline__ void source(const StepArgs& a, const Raw<OWN>& r, C g[Q],
                                                Carry& c) {
    // Deviation storage keeps a2 - u u in m[4..9]: the source takes it as is,
    // and with one relaxation rate for all sites already multiplied by
    // (1 - omega) through the decode factor (1 - omega) s_k, exact as s_k is a
    // power of two, so that q (1 - omega) s_k rounds like (1 - omega)(q s_k).
    constexpr int kNeqMode = !S::kNeq ? kTotal : (VAR ? kDev : kDevRelaxed);
    C m[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      float sk = a.scale[k];
      if constexpr (kNeqMode == kDevRelaxed)
        sk = k >= 4 ? (1.0f - static_cast<float>(a.omega)) * sk : sk;
      m[k] = S::decode(r.m[k], sk);
    }
    if constexpr (S::kSplitU) {
#pragma unroll
      for (int k = 1; k < 4; ++k) m[k] = S::join(r.m[k], r.m[9 + k], a.scale[k]);
    }
    C F[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] = FFIELD ? r.F[k] : static_cast<C>(a.F[k]);
    C omega = static_cast<C>(a.omega);
    if constexpr (VAR) {
      // F / rho and omega of phi(t) at the source
      const C p = r.ph;
      const C inv_rho = C(1) / (static_cast<C>(a.rho_l) + p * static_cast<C>(a.rho_h - a.rho_l));
      const C nu = static_cast<C>(a.nu_l) + p * static_cast<C>(a.nu_h - a.nu_l);
      omega = C(1) / (C(3) * nu + C(0.5));
#pragma unroll
      for (int k = 0; k < 3; ++k) F[k] *= inv_rho;
      if constexpr (OWN) {
        // M for the contrast terms of F(t+1) from the state at t: p* cs^2 and
        // the non-equilibrium a2 - u u (deviation storage holds it directly)
        const C pn = r.sc;
        const C nun = static_cast<C>(a.nu_l) + pn * static_cast<C>(a.nu_h - a.nu_l);
        const C cv = C(3) * nun * (C(1) / (C(3) * nun + C(0.5)));
        const C cp = m[0] * C(1.0 / 3.0);
#pragma unroll
        for (int k = 4; k < 10; ++k)
          c.M[k - 4] = cv * (S::kNeq ? m[k] : m[k] - m[1 + a2_a(k)] * m[1 + a2_b(k)]) +
                       (k < 7 ? cp : C(0));
      }
    }
    if constexpr (!FNEXT) {
#pragma unroll
      for (int k = 0; k < 3; ++k) c.F[k] = F[k];
    }
    if constexpr (FULL)
      source_pops_full<C, SEL, kNeqMode, !NOF>(m, F[0], F[1], F[2], omega, g);
    else
      source_pops<Q, C, SEL, kNeqMode, !NOF>(m, F[0], F[1], F[2], omega, g);
  }

  // F(t+1) at a destination from the stencils of phi(t+1) (and, with
  // contrast, the site's state at t); rho(phi(t+1)) into rho
  static __device__ __forceinline__ void force_next(const StepArgs& a, const StencilOut<C>& st,
                                                    const Carry& c, C f[3], C& rho) {
    const C p = st.centre;
    const C beta = static_cast<C>(a.beta), kappa = static_cast<C>(a.kappa);
    const C rl = static_cast<C>(a.rho_l), dr = static_cast<C>(a.rho_h - a.rho_l);
    const C mu = C(4) * beta * p * (p - C(1)) * (p - C(0.5)) - kappa * st.lap;
    rho = rl + p * dr;
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] = mu * st.g[k] + rho * static_cast<C>(a.Fb[k]);
    if constexpr (VAR) {
      if (a.contrast) {
        const C gr[3] = {dr * st.g[0], dr * st.g[1], dr * st.g[2]};
        const C* M = c.M;  // xx yy zz xy xz yz
        f[0] -= M[0] * gr[0] + M[3] * gr[1] + M[4] * gr[2];
        f[1] -= M[3] * gr[0] + M[1] * gr[1] + M[5] * gr[2];
        f[2] -= M[4] * gr[0] + M[5] * gr[1] + M[2] * gr[2];
      }
    }
  }

  // two-component form: F(t+1) from the stencils, written out for the next
  // step, then the correction with it
  template <int NS>
  static __device__ __forceinline__ void finish(const StepArgs& a, const Sums<C> (&acc)[NS],
                                                const Carry (&c)[NS],
                                                const StencilOut<C> (&st)[NS], int64_t pb,
                                                uint32_t off, uint32_t plane_bytes) {
    static_assert(FNEXT, "the stencil form is the two-component step");
    Carry cf[NS];
    C fo[3][NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      C f[3], rho;
      force_next(a, st[s], c[s], f, rho);
      const C inv = VAR ? C(1) / rho : C(1);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        fo[k][s] = f[k];
        cf[s].F[k] = VAR ? f[k] * inv : f[k];
      }
    }
    C* __restrict__ Fo = static_cast<C*>(a.Fout);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      buf_store_nt_n<C, NS>(fo[k], plane_rsrc(Fo + (k * a.N + pb), plane_bytes * kFscale),
                            off * kFscale);
    finish(a, acc, cf, pb, off, plane_bytes);
  }

  template <int NS>
  static __device__ __forceinline__ void finish(const StepArgs& a, const Sums<C> (&acc)[NS],
                                                const Carry (&c)[NS], int64_t pb, uint32_t off,
                                                uint32_t plane_bytes) {
    T* __restrict__ dst = static_cast<T*>(a.dst);
    C out[NS][10];
    T q[NS][S::kPlanes];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      finalize<Q, C, !NOF>(acc[s], c[s].F[0], c[s].F[1], c[s].F[2], out[s]);
      if constexpr (S::kNeq) {
        // 16-bit storage.  p* and u round to nearest, or stochastically (8
        // bits each of one hash of the site index and this step's seed): the
        // planes that accumulate over the steps, where rounding to nearest
        // drops every change below half a unit in the last place and a slowly
        // evolving flow stalls.  a2 - u u, relaxed at every step, rounds to
        // nearest, with the velocity as it will be read back.
        // Without a force, p* and u are the sums times 1/D: they go to
        // storage units in one step, the sum times (inv_scale / D) as a hi +
        // lo pair, which rounds exactly as dividing first and scaling after
        // (the scales are powers of two) with one multiplication less.
        C un[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if constexpr (NOF) {
            const C t = k == 0 ? acc[s].s0 : (k == 1 ? acc[s].jx : (k == 2 ? acc[s].jy : acc[s].jz));
            un[k] = __builtin_fmaf(t, a.enc_hi[k], t * a.enc_lo[k]);
          } else {
            un[k] = out[s][k] * a.inv_scale[k];
          }
        }
        C ur[3];
        if constexpr (S::kSplitU) {
          // split velocity (always to nearest): u as hi and lo words
          q[s][0] = S::encode_unit(un[0]);
#pragma unroll
          for (int k = 1; k < 4; ++k) {
            S::split_unit(un[k], q[s][k], q[s][9 + k]);
            ur[k - 1] = S::join(q[s][k], q[s][9 + k], a.scale[k]);
          }
        } else {
          if (a.stochastic) {
            const uint32_t site = static_cast<uint32_t>(pb) + off / sizeof(T) + s;
            const uint32_t h = hash32(site ^ a.sr_seed);
#pragma unroll
            for (int k = 0; k < 4; ++k)
              q[s][k] = S::encode_unit_sr(un[k], (h >> (8 * k)) & 0xffu);
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) q[s][k] = S::encode_unit(un[k]);
          }
#pragma unroll
          for (int k = 0; k < 3; ++k) ur[k] = S::decode(q[s][1 + k], a.scale[1 + k]);
        }
#pragma unroll
        for (int k = 4; k < 10; ++k)
          q[s][k] = S::encode(out[s][k] - ur[a2_a(k)] * ur[a2_b(k)], a.inv_scale[k]);
      } else {
#pragma unroll
        for (int k = 0; k < 10; ++k) q[s][k] = S::encode(out[s][k], a.inv_scale[k]);
      }
    }
    constexpr int kQ4 = S::kGrouped ? (S::kPlanes & ~3) : 0;
    constexpr int kQ2 = S::kGrouped ? kQ4 + (S::kPlanes & 2) : 0;
    if constexpr (S::kGrouped) {
#pragma unroll
      for (int j = 0; j < kQ4 / 4; ++j) {
        uint64_t w[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          // built as vectors of halves, so that pairs convert in one instruction
          const T4 h = {q[s][4 * j], q[s][4 * j + 1], q[s][4 * j + 2], q[s][4 * j + 3]};
          w[s] = __builtin_bit_cast(uint64_t, h);
        }
        buf_store_nt_n<uint64_t, NS>(
            w, plane_rsrc(reinterpret_cast<uint64_t*>(dst) + (j * a.N + pb), 4 * plane_bytes),
            4 * off);
      }
      if constexpr (kQ2 > kQ4) {
        uint32_t w[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const T2 h = {q[s][kQ4], q[s][kQ4 + 1]};
          w[s] = __builtin_bit_cast(uint32_t, h);
        }
        buf_store_nt_n<uint32_t, NS>(
            w, plane_rsrc(reinterpret_cast<uint32_t*>(dst) + (kQ4 / 2 * a.N + pb), 2 * plane_bytes),
            2 * off);
      }
    }
#pragma unroll
    for (int k = kQ2; k < S::kPlanes; ++k) {
      T v[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) v[s] = q[s][k];
      buf_store_nt_n<T, NS>(v, plane_rsrc(dst + (k * a.N + pb), plane_bytes), off);
    }
  }
};

template <int Q, int ST, int TY, bool WALLY, bool FFIELD, bool FULL = false>
hipError_t launch_step_t(const StepArgs& a, hipStream_t stream) {
  if constexpr (FFIELD && TY <= 8) {
    // a force that changes every step (two-component flow), with or without
    // density and viscosity contrast
    if (a.Fout && a.phi_src)
      return launch_march<Forward<Q, ST, true, true, true, FULL>, TY, WALLY>(a, stream);
    if (a.Fout) return launch_march<Forward<Q, ST, true, true, false, FULL>, TY, WALLY>(a, stream);
  }
  if (a.Fout) return hipErrorInvalidValue;
  if constexpr (!FFIELD) {
    if (a.F[0] == 0.0 && a.F[1] == 0.0 && a.F[2] == 0.0)
      return launch_march<Forward<Q, ST, false, false, false, FULL, true>, TY, WALLY>(a, stream);
  }
  return launch_march<Forward<Q, ST, FFIELD, false, false, FULL>, TY, WALLY>(a, stream);
}

// all (lattice, tile rows, walls, force field) variants of one storage type
// for the second-order sets (lattice 19 or 27), and for D3Q27h (tile rows 4,
// 6 and 8; compiled in translation units of their own)
#define LBF_CASE(QQ, FULL, TYY)                                                   \
  if (tile_rows == TYY) {                                                         \
    if (walls_y)                                                                  \
      return ffield ? launch_step_t<QQ, ST, TYY, true, true, FULL>(a, s)          \
                    : launch_step_t<QQ, ST, TYY, true, false, FULL>(a, s);        \
    return ffield ? launch_step_t<QQ, ST, TYY, false, true, FULL>(a, s)           \
                  : launch_step_t<QQ, ST, TYY, false, false, FULL>(a, s);         \
  }
template <int ST>
hipError_t launch_step_storage(int lattice, int tile_rows, bool walls_y, bool ffield,
                               const StepArgs& a, hipStream_t s) {
  if (lattice == 19) {
    LBF_CASE(19, false, 4)
    LBF_CASE(19, false, 6)
    LBF_CASE(19, false, 8)
    LBF_CASE(19, false, 14)
  } else if (lattice == 27) {
    LBF_CASE(27, false, 4)
    LBF_CASE(27, false, 6)
    LBF_CASE(27, false, 8)
    LBF_CASE(27, false, 14)
  }
  return hipErrorInvalidValue;
}

template <int ST>
hipError_t launch_step_storage_full(int tile_rows, bool walls_y, bool ffield, const StepArgs& a,
                                    hipStream_t s) {
  LBF_CASE(27, true, 4)
  LBF_CASE(27, true, 6)
  LBF_CASE(27, true, 8)
  return hipErrorInvalidValue;
}
#undef LBF_CASE

}  // namespace lbf
