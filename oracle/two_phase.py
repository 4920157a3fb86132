"""Two-component variant of the oracle, FP64 (section 2 of the paper).

TEST INFRASTRUCTURE (see the package docstring).  Density and viscosity are
blended linearly in the phase field, rho = rho_L + phi (rho_H - rho_L),
nu = nu_L + phi (nu_H - nu_L), tau = nu / cs^2 + 1/2.  The total force is the
capillary force plus rho g (g: body acceleration) plus the pressure and
viscous terms of the force split (zero at equal densities), see
lbm_oracle.c.  Order of one step t -> t+1:
  1. phi(t+1) = FTCS step of Eq. (2) with u(t) (the reported velocity);
  2. F(t+1) from phi(t+1); its pressure and viscous terms use p*, u and a2 of
     time t (the newest level known before the step);
  3. populations: collide with F(t), rho(t), omega(t) (moments corrected
     with F(t)/rho(t), Guo source with F(t)/rho(t)), then stream; the
     reported moments at t+1 are corrected with F(t+1)/rho(t+1), so the
     correction uses the force of the updated time level.
Axes periodic, or walled (halfway bounce-back for the flow, mirror images
for the phase-field stencils).  Also: the Laplace measurement and the
layered-channel (two-layer Poiseuille) profile.
"""
import ctypes

import numpy as np

from . import PopulationOracle, _dp, _load

EPS_NORMAL = 1e-12  # n = grad(phi) / (|grad(phi)| + eps), FP64
CS2 = 1.0 / 3.0


def _bcp(bc):
    b = np.ascontiguousarray(np.asarray(bc, dtype=np.int32))
    return b, b.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def grad(phi, bc=(0, 0, 0)):
    """D3Q27-weighted gradient (section 2), [3, nz, ny, nx]."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    out = np.empty((3,) + phi.shape)
    b, bp = _bcp(bc)
    assert _load().oracle_grad(nx, ny, nz, bp, _dp(phi), _dp(out)) == 0
    return out


def lap(phi, bc=(0, 0, 0)):
    """D3Q27-weighted Laplacian, (2/cs^2) sum_{i != 0} w_i [Psi(x+c_i) - Psi(x)]."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    out = np.empty(phi.shape)
    b, bp = _bcp(bc)
    assert _load().oracle_lap(nx, ny, nz, bp, _dp(phi), _dp(out)) == 0
    return out


def phase_step(phi, u, D, W, eps=EPS_NORMAL, bc=(0, 0, 0)):
    """One FTCS step of the conservative Allen-Cahn equation, Eq. (2)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape((3,) + phi.shape))
    nz, ny, nx = phi.shape
    out = np.empty(phi.shape)
    b, bp = _bcp(bc)
    assert _load().oracle_phase_step(nx, ny, nz, bp, _dp(phi), _dp(u), D, W, eps,
                                     _dp(out)) == 0
    return out


def capillary_force(phi, sigma, W, Fb=None, bc=(0, 0, 0)):
    """F = mu grad(phi) (+ body force Fb, [3, ...] or a 3-vector)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    out = np.empty((3,) + phi.shape)
    fb = None if Fb is None else np.ascontiguousarray(
        np.broadcast_to(np.asarray(Fb, dtype=np.float64).reshape(3, 1, 1, 1) if np.size(Fb) == 3
                        else np.asarray(Fb, dtype=np.float64), (3,) + phi.shape))
    b, bp = _bcp(bc)
    assert _load().oracle_capillary_force(nx, ny, nz, bp, _dp(phi), sigma, W, _dp(fb),
                                          _dp(out)) == 0
    return out


class TwoPhaseOracle:
    """Flow (population oracle) + phase field on an (nx, ny, nz) grid.
    rho = (rho_L, rho_H), nu = (nu_L, nu_H) or None (one tau for both phases:
    the `tau` argument); g: body acceleration (3-vector) or None."""

    def __init__(self, Q, shape, tau, sigma, W, D, body_force=None, bc=(0, 0, 0),
                 rho=(1.0, 1.0), nu=None):
        self.shape = tuple(int(v) for v in shape)
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self.sigma, self.W, self.D = float(sigma), float(W), float(D)
        self.g = None if body_force is None else np.asarray(body_force, dtype=np.float64)
        self.bc = tuple(int(v) for v in bc)
        self.rho_lh = tuple(float(v) for v in rho)
        nu1 = CS2 * (tau - 0.5)
        self.nu_lh = (nu1, nu1) if nu is None else tuple(float(v) for v in nu)
        self.flow = PopulationOracle(Q, self.shape, tau, bc=bc)
        self.phi = np.zeros((nz, ny, nx))

    def rho(self, phi):
        return self.rho_lh[0] + phi * (self.rho_lh[1] - self.rho_lh[0])

    def omega(self, phi):
        nu = self.nu_lh[0] + phi * (self.nu_lh[1] - self.nu_lh[0])
        return 1.0 / (nu / CS2 + 0.5)

    def _force(self, phi, m):
        """F from phi and the moments m (pressure and viscous terms)."""
        Fb = None
        if self.g is not None:
            Fb = self.rho(phi)[None] * self.g.reshape(3, 1, 1, 1)
        F = capillary_force(phi, self.sigma, self.W, Fb, self.bc).reshape(3, self.N)
        if self.rho_lh[0] != self.rho_lh[1]:
            nx, ny, nz = self.shape
            b, bp = _bcp(self.bc)
            F = np.ascontiguousarray(F)
            mm = np.ascontiguousarray(np.asarray(m, dtype=np.float64).reshape(10, self.N))
            ph = np.ascontiguousarray(phi)
            assert _load().oracle_contrast_force(nx, ny, nz, bp, _dp(ph), _dp(mm),
                                                 self.rho_lh[0], self.rho_lh[1], self.nu_lh[0],
                                                 self.nu_lh[1], _dp(F)) == 0
        return np.ascontiguousarray(F)

    def _moments(self):
        nx, ny, nz = self.shape
        m = np.zeros((10, self.N))
        r = np.ascontiguousarray(self.rho(self.phi).reshape(self.N))
        assert _load().oracle_moments_var(self.flow.lattice, nx, ny, nz, _dp(r), _dp(self.flow.f),
                                          _dp(self.flow.F), _dp(m)) == 0
        return m

    def set_state(self, m, phi):
        """Moments m [10, nz, ny, nx] and phase field phi [nz, ny, nx] at t = 0."""
        nx, ny, nz = self.shape
        self.phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(
            self.shape[::-1]))
        m = np.ascontiguousarray(np.asarray(m, dtype=np.float64).reshape(10, self.N))
        self.flow.F = self._force(self.phi, m)
        r = np.ascontiguousarray(self.rho(self.phi).reshape(self.N))
        assert _load().oracle_init_var(self.flow.lattice, nx, ny, nz, _dp(r), _dp(m),
                                       _dp(self.flow.F), _dp(self.flow.f)) == 0

    def moments(self):
        nx, ny, nz = self.shape
        return self._moments().reshape(10, nz, ny, nx)

    def step(self, n=1):
        lib = _load()
        nx, ny, nz = self.shape
        b, bp = _bcp(self.bc)
        post = np.empty_like(self.flow.f)
        for _ in range(int(n)):
            m = self._moments()
            phi_new = phase_step(self.phi, m[1:4], self.D, self.W, bc=self.bc)
            F_new = self._force(phi_new, m)
            om = np.ascontiguousarray(self.omega(self.phi).reshape(self.N))
            r = np.ascontiguousarray(self.rho(self.phi).reshape(self.N))
            assert lib.oracle_collide_var(self.flow.lattice, nx, ny, nz, _dp(om), _dp(r),
                                          _dp(self.flow.f), _dp(self.flow.F), _dp(post)) == 0
            assert lib.oracle_stream(self.flow.lattice, nx, ny, nz, bp, _dp(post),
                                     _dp(self.flow.f)) == 0
            self.phi, self.flow.F = phi_new, F_new


def droplet(shape, R, W, center=None):
    """phi = 1/2 [1 - tanh(2 (r - R) / W)] around `center` (default: the
    middle of the grid), the planar equilibrium profile of Eq. (2) with
    lambda = 4 D / W; [nz, ny, nx]."""
    nx, ny, nz = shape
    cx, cy, cz = center if center is not None else (nx / 2, ny / 2, nz / 2)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
    return 0.5 * (1.0 - np.tanh(2.0 * (r - R) / W))


def layers(shape, W):
    """Two layers across a channel walled in y (halfway walls at y = -1/2 and
    ny - 1/2): phi = 0 (light phase) for eta < ny/2, 1 (heavy) above, eta =
    y + 1/2, as the tanh profile of width W; [nz, ny, nx]."""
    nx, ny, nz = shape
    eta = np.arange(ny) + 0.5
    prof = 0.5 * (1.0 + np.tanh(2.0 * (eta - ny / 2) / W))
    return np.broadcast_to(prof[None, :, None], (nz, ny, nx)).copy()


def layered_poiseuille(ny, g, rho, nu):
    """Steady two-layer channel profile (sharp interface at the middle): walls
    at eta = 0 and H = ny, layer 1 (rho[0], nu[0]) below H/2, layer 2 above,
    body acceleration g along the channel; mu_k u'' = -rho_k g, u continuous,
    mu u' continuous at the interface.  Returns u at eta = y + 1/2."""
    H, h = float(ny), ny / 2.0
    mu = [rho[0] * nu[0], rho[1] * nu[1]]
    c = [g / (2.0 * nu[0]), g / (2.0 * nu[1])]  # u_k = -c_k eta^2 + A_k eta + B_k
    # unknowns A1, A2, B2 (B1 = 0)
    M = np.array([[0.0, H, 1.0],                      # u2(H) = 0
                  [h, -h, -1.0],                      # u1(h) = u2(h)
                  [mu[0], -mu[1], 0.0]])              # mu1 u1'(h) = mu2 u2'(h)
    rhs = np.array([c[1] * H * H,
                    c[0] * h * h - c[1] * h * h,
                    mu[0] * 2 * c[0] * h - mu[1] * 2 * c[1] * h])
    A1, A2, B2 = np.linalg.solve(M, rhs)
    eta = np.arange(ny) + 0.5
    return np.where(eta < h, -c[0] * eta ** 2 + A1 * eta, -c[1] * eta ** 2 + A2 * eta + B2)


def laplace(m, phi, R, W, center=None):
    """Pressure jump across the droplet and the surface tension it implies:
    p = rho cs^2 p* (rho = 1), averaged inside r < R/2 and outside r > R + 3W;
    R_eff = (3 sum(phi) / (4 pi))^(1/3); sigma = dP R_eff / 2 (Laplace law).
    Returns (dP, R_eff, sigma)."""
    nz, ny, nx = phi.shape
    cx, cy, cz = center if center is not None else (nx / 2, ny / 2, nz / 2)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
    p = np.asarray(m[0]) / 3.0
    dP = float(p[r < R / 2].mean() - p[r > R + 3 * W].mean())
    R_eff = float((3.0 * phi.sum() / (4.0 * np.pi)) ** (1.0 / 3.0))
    return dP, R_eff, dP * R_eff / 2.0
