// stencil.hpp -- the D3Q27-weighted finite-difference stencils of the phase
// field (paper, section 2), in the separable form the z-marching kernels use.
//
//   grad_a Psi = (1/cs^2) sum_i w_i c_ia Psi(x + c_i) = (1/72) sum k_i c_ia Psi_i
//   lap Psi    = (2/cs^2) sum_{i!=0} w_i (Psi_i - Psi_0) = (1/36) sum k_i (Psi_i - Psi_0)
//
// with k_i = 216 w_i = 64, 16, 4, 1 for |c_i|^2 = 0..3 (the printed Laplacian
// stencil is garbled; this is its Taylor-consistent reading, zero on
// constants).  The weights factor: k(dx, dy, dz) = k1(dx) k1(dy) k1(dz) with
// k1(0) = 4, k1(+-1) = 1, so a plane's sums with the weights of an adjacent
// plane are separable 3 x 3 sums, and with the own plane's weights they are 4
// times those.
#pragma once

#include "lattice.hpp"

namespace lbf {

template <typename C>
__device__ __forceinline__ C sum141(C a, C b, C c) {
  return a + C(4) * b + c;
}

// On a 3 x 3 window n[dy][dx] (offsets -1..1):
//   ss = sum k1 k1 n, ds = sum dx k1 k1 n, sd = sum dy k1 k1 n.
template <typename C>
__device__ __forceinline__ void window_sums(const C (&n)[3][3], C& ss, C& ds, C& sd) {
  C sx[3], dx[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    sx[r] = sum141(n[r][0], n[r][1], n[r][2]);
    dx[r] = n[r][2] - n[r][0];
  }
  ss = sum141(sx[0], sx[1], sx[2]);
  ds = sum141(dx[0], dx[1], dx[2]);
  sd = sx[2] - sx[0];
}

// sum k1 k1 (n - own), the centre being own: the differences are formed
// first, so that FP32 adds small numbers
template <typename C>
__device__ __forceinline__ C window_lap(const C (&n)[3][3], C own) {
  const C r0 = sum141(n[0][0] - own, n[0][1] - own, n[0][2] - own);
  const C r1 = (n[1][0] - own) + (n[1][2] - own);
  const C r2 = sum141(n[2][0] - own, n[2][1] - own, n[2][2] - own);
  return sum141(r0, r1, r2);
}

// sum of k1 k1 over the 9 sites of a plane
constexpr int kPlaneK = 16 + 4 * 4 + 4 * 1;

// Gradient, Laplacian and centre value of a scalar at one site.
template <typename C>
struct StencilOut {
  C g[3];
  C lap;
  C centre;
};

// Rolling 2.5-D accumulation of the stencils along z: planes arrive in order
// p = 0, 1, 2, ...; the window of plane p completes the site of plane p - 1
// and is added to those of planes p and p + 1.  The Laplacian sums of a site
// are kept relative to the value of the site below it (pm) and corrected by
// the weight sum times the difference once the site's own value is known.
template <typename C>
struct StencilRoll {
  C gxm, gym, gzm, lm, pm;  // site p - 1: sums of planes p - 2 and p - 1, its value
  C gx0, gy0, gz0, l0;      // site p: sums of plane p - 1, relative to pm

  __device__ __forceinline__ void clear() {
    gxm = gym = gzm = lm = pm = gx0 = gy0 = gz0 = l0 = C(0);
  }
  // add plane p (window n, centre n[1][1]) and return the site of plane p - 1
  __device__ __forceinline__ StencilOut<C> plane(const C (&n)[3][3]) {
    const C own = n[1][1];
    C az, ax, ay;
    window_sums(n, az, ax, ay);
    const C lu = window_lap(n, own);
    StencilOut<C> o;
    o.g[0] = div_by<72>(gxm + ax);
    o.g[1] = div_by<72>(gym + ay);
    o.g[2] = div_by<72>(gzm + az);
    o.lap = div_by<36>(lm + lu + C(kPlaneK) * (own - pm));
    o.centre = pm;
    // site p: plane p - 1 (at dz = -1) and this plane (own weights 4 k1 k1)
    gxm = gx0 + C(4) * ax;
    gym = gy0 + C(4) * ay;
    gzm = gz0;
    lm = l0 - C(kPlaneK) * (own - pm) + C(4) * lu;
    pm = own;
    // site p + 1: this plane at dz = -1
    gx0 = ax;
    gy0 = ay;
    gz0 = -az;
    l0 = lu;
    return o;
  }
};

}  // namespace lbf
