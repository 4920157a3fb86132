"""Two-component variant of the oracle, FP64 (section 2 of the paper).

TEST INFRASTRUCTURE (see the package docstring).  Equal phase densities and
viscosities (rho = 1, one tau), so the pressure and viscous force terms of the
force split vanish and the total force is the capillary force plus an
optional body force.  Order of one step t -> t+1:
  1. phi(t+1) = FTCS step of Eq. (2) with u(t) (the reported velocity);
  2. F(t+1) = mu(phi(t+1)) grad(phi(t+1)) + F^b;
  3. populations: collide with F(t) (moments corrected with F(t), Guo source
     with F(t)), then stream; the reported moments at t+1 are corrected with
     F(t+1), so the correction uses the force of the updated time level.
Periodic grid.  Also: the Laplace measurement of the pressure jump.
"""
import ctypes

import numpy as np

from . import PopulationOracle, _dp, _load

EPS_NORMAL = 1e-12  # n = grad(phi) / (|grad(phi)| + eps), FP64


def grad(phi):
    """D3Q27-weighted gradient (section 2), [3, nz, ny, nx]."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    out = np.empty((3,) + phi.shape)
    assert _load().oracle_grad(nx, ny, nz, _dp(phi), _dp(out)) == 0
    return out


def lap(phi):
    """D3Q27-weighted Laplacian, (2/cs^2) sum_{i != 0} w_i [Psi(x+c_i) - Psi(x)]."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    out = np.empty(phi.shape)
    assert _load().oracle_lap(nx, ny, nz, _dp(phi), _dp(out)) == 0
    return out


def phase_step(phi, u, D, W, eps=EPS_NORMAL):
    """One FTCS step of the conservative Allen-Cahn equation, Eq. (2)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape((3,) + phi.shape))
    nz, ny, nx = phi.shape
    out = np.empty(phi.shape)
    assert _load().oracle_phase_step(nx, ny, nz, _dp(phi), _dp(u), D, W, eps, _dp(out)) == 0
    return out


def capillary_force(phi, sigma, W, Fb=None):
    """F = mu grad(phi) (+ body force Fb [3, ...])."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    out = np.empty((3,) + phi.shape)
    fb = None if Fb is None else np.ascontiguousarray(
        np.broadcast_to(np.asarray(Fb, dtype=np.float64).reshape(3, 1, 1, 1) if np.size(Fb) == 3
                        else np.asarray(Fb, dtype=np.float64), (3,) + phi.shape))
    assert _load().oracle_capillary_force(nx, ny, nz, _dp(phi), sigma, W, _dp(fb), _dp(out)) == 0
    return out


class TwoPhaseOracle:
    """Flow (population oracle) + phase field on an (nx, ny, nz) periodic grid."""

    def __init__(self, Q, shape, tau, sigma, W, D, body_force=None):
        self.shape = tuple(int(v) for v in shape)
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self.sigma, self.W, self.D = float(sigma), float(W), float(D)
        self.Fb = body_force
        self.flow = PopulationOracle(Q, self.shape, tau)
        self.phi = np.zeros((nz, ny, nx))

    def _force(self, phi):
        return capillary_force(phi, self.sigma, self.W, self.Fb).reshape(3, self.N)

    def set_state(self, m, phi):
        """Moments m [10, nz, ny, nx] and phase field phi [nz, ny, nx] at t = 0."""
        self.phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(
            self.shape[::-1]))
        self.flow.F = np.ascontiguousarray(self._force(self.phi))
        self.flow.set_moments(m)

    def moments(self):
        return self.flow.moments()

    def step(self, n=1):
        lib = _load()
        nx, ny, nz = self.shape
        bc = np.zeros(3, dtype=np.int32)
        bcp = bc.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        post = np.empty_like(self.flow.f)
        for _ in range(int(n)):
            u = self.flow.moments()[1:4]
            phi_new = phase_step(self.phi, u, self.D, self.W)
            F_new = np.ascontiguousarray(self._force(phi_new))
            assert lib.oracle_collide(self.flow.Q, nx, ny, nz, self.flow.tau, _dp(self.flow.f),
                                      _dp(self.flow.F), _dp(post)) == 0
            assert lib.oracle_stream(self.flow.Q, nx, ny, nz, bcp, _dp(post),
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
