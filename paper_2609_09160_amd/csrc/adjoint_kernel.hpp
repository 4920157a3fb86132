// adjoint_kernel.hpp -- one step of the discrete adjoint of the fused
// moment-space step (the step of Eq. (7) followed by the correction of
// Eq. (8), with the Guo force of Eq. (9); the paper itself does not treat
// differentiation).
//
// Forward step, per destination x (F static per site, rho = 1):
//   source y:   P0 = p, P1 = u + F/2,
//               P2 = omega u u + (1 - omega) a2 + (u F + F u)/2
//   populations f_i(y) = w_i [P0 + 3 c_i.P1 + 4.5 H_i : P2],
//               H_i = c_i c_i - I/3 (full contraction)
//   pull        g_i(x) = f_i(x - c_i)      (bounce-back: f_{-i}(x))
//   project     s0 = sum g, s1 = sum c g, s2 = sum H g
//   correct     p' = s0, u' = s1 + F/2, a2' = s2 + (F u' + u' F)/2.
//
// Reverse mode with lambda = dJ/dm(t+1) (second-order planes by stored
// component), per site x' of time t+1 (the adjoint's "source"):
//   sigma0 = lambda_p, sigma2 = lambda_a2,
//   sigma1 = lambda_u + dA'/du'^T lambda_a2           (A' depends on u')
//   phi_i(x') = sigma0 + c_i.sigma1 + H_i : sigma2     (dJ/dg_i(x'))
//   dJ/dF(x') += sigma1/2 + dA'/dF^T lambda_a2        (needs u'(x'))
// and per site y of time t (the adjoint's "destination"), with
// psi_i(y) = phi_i(y + c_i) (bounce-back: phi_{-i}(y)):
//   pi0 = sum w psi, pi1 = 3 sum w c psi, pi2 = 4.5 sum w H psi (x2 off-diag)
//   lambda_p(t) = pi0, lambda_u(t) = pi1 + dP2/du^T pi2, lambda_a2(t) =
//   (1 - omega) pi2, dJ/dF(y) += pi1/2 + dP2/dF^T pi2    (needs u(t)(y)).
//
// The gather psi_i(y) = phi_i(y + c_i) is the forward pull run backwards:
// site x' sends w_i phi_{-i}(x') along +c_i, i.e. the values of the forward
// expansion with coefficients (A, D, O, V) = (sigma0 - tr sigma2 / 3,
// sigma2_aa, sigma2_ab, -sigma1), and the running sums of the skeleton then
// hold D pi0, -D pi1 / 3 and D sum w c c psi.  Bounce-back maps onto the
// skeleton's rule unchanged.  So the kernel is the z-march of march.hpp with
// the Adjoint policy below.
#pragma once

#include "march.hpp"

namespace lbf {

template <int Q_, typename C_, bool FFIELD>
struct Adjoint {
  static constexpr int Q = Q_;
  static constexpr bool kThreeSites = std::is_same_v<C_, float>;
  static constexpr bool kStencil = false;
  using C = C_;
  using T = C_;
  // lambda(t+1) and F of a site; destinations also read u(t+1), u(t) and
  // the dJ/dF accumulated so far (x[0..2], x[3..5], x[6..8])
  template <bool OWN>
  struct Raw {
    C l[10];
    C F[3];
    C x[OWN ? 9 : 1];
  };
  // handed from the site of t+1 to the same site of t: F, u(t), and dJ/dF
  // including this step's correction part
  struct Carry {
    C F[3];
    C u[3];
    C g[3];
  };
  static __device__ __forceinline__ void clear(Carry& c) {
#pragma unroll
    for (int k = 0; k < 3; ++k) c.F[k] = c.u[k] = c.g[k] = C(0);
  }

  template <bool OWN, int NS>
  static __device__ __forceinline__ void fetch(const StepArgs& a, int64_t pb, uint32_t off,
                                               uint32_t plane_bytes, Raw<OWN> (&r)[NS]) {
    auto load = [&](const C* base, C (&v)[NS]) __attribute__((always_inline)) {
      buf_load_n<C, NS>(plane_rsrc(base, plane_bytes), off, v);
    };
    const C* __restrict__ lam = static_cast<const C*>(a.src);
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      C v[NS];
      load(lam + (k * a.N + pb), v);
#pragma unroll
      for (int s = 0; s < NS; ++s) r[s].l[k] = v[s];
    }
    if constexpr (FFIELD) {
      const C* __restrict__ Ff = static_cast<const C*>(a.Ffield);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        C v[NS];
        load(Ff + (k * a.N + pb), v);
#pragma unroll
        for (int s = 0; s < NS; ++s) r[s].F[k] = v[s];
      }
    }
    if constexpr (OWN) {
      const C* __restrict__ sn = static_cast<const C*>(a.state_new);
      const C* __restrict__ so = static_cast<const C*>(a.state_old);
      const C* __restrict__ gf = static_cast<const C*>(a.gF);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        C v[NS];
        load(sn + ((1 + k) * a.N + pb), v);
#pragma unroll
        for (int s = 0; s < NS; ++s) r[s].x[k] = v[s];
        load(so + ((1 + k) * a.N + pb), v);
#pragma unroll
        for (int s = 0; s < NS; ++s) r[s].x[3 + k] = v[s];
        load(gf + (k * a.N + pb), v);
#pragma unroll
        for (int s = 0; s < NS; ++s) r[s].x[6 + k] = v[s];
      }
    }
  }

  template <bool OWN, int SEL>
  static __device__ __forceinline__ void source(const StepArgs& a, const Raw<OWN>& r, C g[Q],
                                                Carry& c) {
    const C h = C(0.5);
    C F[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] = FFIELD ? r.F[k] : static_cast<C>(a.F[k]);
    const C* l = r.l;
    // sigma1 = dJ/du' through u' itself and through a2' = s2 + (F u' + u' F)/2
    const C s1x = l[1] + l[4] * F[0] + h * (l[7] * F[1] + l[8] * F[2]);
    const C s1y = l[2] + l[5] * F[1] + h * (l[7] * F[0] + l[9] * F[2]);
    const C s1z = l[3] + l[6] * F[2] + h * (l[8] * F[0] + l[9] * F[1]);
    const C A = l[0] - div_by<3>(l[4] + l[5] + l[6]);
    expand<Q, C, SEL>(A, l[4], l[5], l[6], l[7], l[8], l[9], -s1x, -s1y, -s1z, g);
    if constexpr (OWN) {
      const C* un = r.x;  // u(t+1) at this site
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        c.F[k] = F[k];
        c.u[k] = r.x[3 + k];
      }
      c.g[0] = r.x[6] + h * s1x + l[4] * un[0] + h * (l[7] * un[1] + l[8] * un[2]);
      c.g[1] = r.x[7] + h * s1y + l[5] * un[1] + h * (l[7] * un[0] + l[9] * un[2]);
      c.g[2] = r.x[8] + h * s1z + l[6] * un[2] + h * (l[8] * un[0] + l[9] * un[1]);
    }
  }

  template <int NS>
  static __device__ __forceinline__ void finish(const StepArgs& a, const Sums<C> (&acc)[NS],
                                                const Carry (&cc)[NS], int64_t pb, uint32_t off,
                                                uint32_t plane_bytes) {
    constexpr int D = Lat<Q>::D;
    const C h = C(0.5);
    const C om = static_cast<C>(a.omega);
    const C om1 = C(1) - om;
    const C two_om = C(2) * om;
    C out[NS][13];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const Sums<C>& S = acc[s];
      const Carry& c = cc[s];
      // gradients with respect to the post-collision coefficients P0, P1, P2
      const C q0 = div_by<D>(S.s0);
      const C q1x = C(-3) * div_by<D>(S.jx);
      const C q1y = C(-3) * div_by<D>(S.jy);
      const C q1z = C(-3) * div_by<D>(S.jz);
      const C qxx = div_by<2 * D>(C(3) * (C(3) * S.pxx - S.s0));
      const C qyy = div_by<2 * D>(C(3) * (C(3) * S.pyy - S.s0));
      const C qzz = div_by<2 * D>(C(3) * (C(3) * S.pzz - S.s0));
      const C qxy = C(9) * div_by<D>(S.pxy);
      const C qxz = C(9) * div_by<D>(S.pxz);
      const C qyz = C(9) * div_by<D>(S.pyz);
      const C ux = c.u[0], uy = c.u[1], uz = c.u[2];
      const C Fx = c.F[0], Fy = c.F[1], Fz = c.F[2];
      C* o = out[s];
      o[0] = q0;
      o[1] = q1x + qxx * (two_om * ux + Fx) + qxy * (om * uy + h * Fy) + qxz * (om * uz + h * Fz);
      o[2] = q1y + qyy * (two_om * uy + Fy) + qxy * (om * ux + h * Fx) + qyz * (om * uz + h * Fz);
      o[3] = q1z + qzz * (two_om * uz + Fz) + qxz * (om * ux + h * Fx) + qyz * (om * uy + h * Fy);
      o[4] = om1 * qxx;
      o[5] = om1 * qyy;
      o[6] = om1 * qzz;
      o[7] = om1 * qxy;
      o[8] = om1 * qxz;
      o[9] = om1 * qyz;
      o[10] = c.g[0] + h * q1x + qxx * ux + h * (qxy * uy + qxz * uz);
      o[11] = c.g[1] + h * q1y + qyy * uy + h * (qxy * ux + qyz * uz);
      o[12] = c.g[2] + h * q1z + qzz * uz + h * (qxz * ux + qyz * uy);
    }
    C* __restrict__ lam = static_cast<C*>(a.dst);
    C* __restrict__ gf = static_cast<C*>(a.gF);
#pragma unroll
    for (int k = 0; k < 13; ++k) {
      C v[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) v[s] = out[s][k];
      C* base = k < 10 ? lam + (k * a.N + pb) : gf + ((k - 10) * a.N + pb);
      buf_store_nt_n<C, NS>(v, plane_rsrc(base, plane_bytes), off);
    }
  }
};

template <typename C>
hipError_t launch_adjoint_type(int Q, int tile_rows, bool walls_y, bool ffield,
                               const StepArgs& a, hipStream_t s) {
  // A destination reads 22 values: one site per lane fits 10-wave workgroups
  // (8-row tiles); two or three sites per lane (FP32) need the register room
  // of shorter tiles (4 or 6 rows: at most 2 waves per SIMD).
#define LBF_ADJ_CASE(QQ, TYY, SS)                                                     \
  if (Q == QQ && tile_rows == TYY && a.lane_sites == SS) {                            \
    if (walls_y)                                                                     \
      return ffield ? launch_march_s<Adjoint<QQ, C, true>, TYY, true, SS>(a, s)      \
                    : launch_march_s<Adjoint<QQ, C, false>, TYY, true, SS>(a, s);    \
    return ffield ? launch_march_s<Adjoint<QQ, C, true>, TYY, false, SS>(a, s)       \
                  : launch_march_s<Adjoint<QQ, C, false>, TYY, false, SS>(a, s);     \
  }
  LBF_ADJ_CASE(19, 4, 1)
  LBF_ADJ_CASE(19, 6, 1)
  LBF_ADJ_CASE(19, 8, 1)
  LBF_ADJ_CASE(19, 14, 1)
  LBF_ADJ_CASE(27, 4, 1)
  LBF_ADJ_CASE(27, 6, 1)
  LBF_ADJ_CASE(27, 8, 1)
  LBF_ADJ_CASE(27, 14, 1)
  if constexpr (std::is_same_v<C, float>) {
    LBF_ADJ_CASE(19, 4, 2)
    LBF_ADJ_CASE(19, 6, 2)
    LBF_ADJ_CASE(19, 4, 3)
    LBF_ADJ_CASE(19, 6, 3)
    LBF_ADJ_CASE(27, 4, 2)
    LBF_ADJ_CASE(27, 4, 3)
  }
#undef LBF_ADJ_CASE
  return hipErrorInvalidValue;
}

}  // namespace lbf
