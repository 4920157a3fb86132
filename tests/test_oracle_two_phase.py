"""Pins of the two-component oracle (oracle/two_phase.py): the D3Q27-weighted
derivative stencils against their exact discrete Fourier symbols, exact
conservation of the phase field and of momentum with a force that changes
every step, the exact drift of a droplet under uniform advection, the
planar equilibrium of Eq. (2), the Laplace law, and (density and viscosity
contrast, walls) the steady layered channel against a 1-D solve of the
continuum equation."""
import numpy as np
import pytest


def _grid(n):
    return np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")  # z, y, x


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_stencils_exact_symbols(oracle_mod, axis):
    """For Psi = sin(k x_a + 0.3) on a periodic grid the stencils of section 2
    give exactly grad_a Psi = sin(k) cos(k x_a + 0.3), the other components
    zero, and lap Psi = 2 (cos k - 1) Psi (the symbol of the Taylor-consistent
    Laplacian with the D3Q27 weights; zero on constants).  A wrong weight, a
    missing 1/cs^2 or the printed centre term fails here."""
    from oracle import two_phase as T
    n = 16
    k = 2 * np.pi / n * 3
    X = _grid(n)[2 - axis]
    psi = np.sin(k * X + 0.3)
    g = T.grad(psi)
    assert np.abs(g[axis] - np.sin(k) * np.cos(k * X + 0.3)).max() <= 1e-14
    for b in range(3):
        if b != axis:
            assert np.abs(g[b]).max() <= 1e-14
    assert np.abs(T.lap(psi) - 2 * (np.cos(k) - 1) * psi).max() <= 1e-14
    assert np.abs(T.lap(np.full((n, n, n), 0.7))).max() <= 1e-15
    assert np.abs(T.grad(np.full((n, n, n), 0.7))).max() <= 1e-15


def test_phase_field_conserved(oracle_mod):
    """The flux form of Eq. (2) with antisymmetric stencils conserves sum(phi)
    exactly on a periodic grid, for any velocity and any phase field."""
    from oracle import two_phase as T
    rng = np.random.default_rng(3)
    phi = rng.uniform(0, 1, (12, 10, 14))
    u = 0.05 * rng.standard_normal((3, 12, 10, 14))
    p1 = T.phase_step(phi, u, 0.1, 4.0)
    assert abs(p1.sum() - phi.sum()) <= 1e-12 * phi.sum()


def test_droplet_drift_under_uniform_advection(oracle_mod):
    """With uniform u = (U, 0, 0), one FTCS step moves the first moment of a
    centred droplet by exactly U sum(phi): diffusion conserves it, and the
    interface-compression flux sums to zero by symmetry.  A sign error or a
    wrong factor in the advection term fails here."""
    from oracle import two_phase as T
    shape = (64, 32, 32)
    nx, ny, nz = shape
    phi = T.droplet(shape, 5, 4)
    U = 0.01
    u = np.zeros((3, nz, ny, nx))
    u[0] = U
    p1 = T.phase_step(phi, u, 0.1, 4.0)
    xs = (np.arange(nx) - nx / 2)[None, None, :]
    drift = float((xs * (p1 - phi)).sum())
    assert abs(drift - U * phi.sum()) <= 1e-8 * U * phi.sum()


def test_planar_interface_equilibrium(oracle_mod):
    """phi = 1/2 [1 - tanh(2 d / W)] is the equilibrium of Eq. (2) at rest
    (lambda = 4 D / W balances diffusion) and of the chemical potential
    (beta = 12 sigma/W, kappa = 3 sigma W/2 make mu vanish on it).  On the
    lattice, 400 steps move it by < 2e-2 (pure diffusion, or a compression
    term of the wrong sign or size, moves it by ~0.3) and the capillary force
    stays below 1e-3 (a factor 2 on kappa gives ~5e-3)."""
    from oracle import two_phase as T
    nx, ny, nz, W, L = 64, 4, 4, 4.0, 16
    x = np.arange(nx)[None, None, :] * np.ones((nz, ny, 1))
    phi0 = 0.5 * (1 - np.tanh(2 * (np.abs(x - nx / 2) - L) / W))
    u = np.zeros((3, nz, ny, nx))
    phi = phi0.copy()
    for _ in range(400):
        phi = T.phase_step(phi, u, 0.1, W)
    assert np.abs(phi - phi0).max() <= 2e-2
    assert np.abs(T.capillary_force(phi0, 0.03, W)).max() <= 1e-3


def test_momentum_with_time_dependent_force(oracle_mod):
    """Periodic grid: sum u(t+1) = sum u(t) + sum F(t)/2 + sum F(t+1)/2
    exactly, half of the force of each time level entering at the source
    (Guo term) and half in the correction of Eq. (8); sum p* is conserved."""
    from oracle import two_phase as T
    shape = (12, 10, 8)
    nx, ny, nz = shape
    rng = np.random.default_rng(4)
    phi = np.clip(T.droplet(shape, 3.5, 3.0) + 0.05 * rng.standard_normal((nz, ny, nx)), 0, 1)
    m = np.zeros((10, nz, ny, nx))
    m[1:4] = 0.01 * rng.standard_normal((3, nz, ny, nx))
    m[4:] = 1e-3 * rng.standard_normal((6, nz, ny, nx))
    o = T.TwoPhaseOracle(19, shape, 0.9, 0.05, 3.0, 0.1)
    o.set_state(m, phi)
    for _ in range(5):
        m0, F0 = o.moments(), o.flow.F.copy()
        o.step(1)
        m1, F1 = o.moments(), o.flow.F
        want = m0[1:4].sum(axis=(1, 2, 3)) + 0.5 * F0.sum(axis=1) + 0.5 * F1.sum(axis=1)
        assert np.abs(m1[1:4].sum(axis=(1, 2, 3)) - want).max() <= 1e-14 * nx * ny * nz
        assert abs(m1[0].sum() - m0[0].sum()) <= 1e-13


def test_laplace_law(oracle_mod):
    """Static droplet, D3Q19, 32^3, R = 8, W = 4, sigma = 0.03, D = 0.1,
    tau = 1, 600 steps: the pressure jump gives sigma = dP R_eff / 2 within
    10% of the input (the paper reports -6.8% at R = 64; the measurement
    procedure is this build's reading)."""
    from oracle import two_phase as T
    n, R, W, sigma = 32, 8, 4.0, 0.03
    o = T.TwoPhaseOracle(19, (n, n, n), 1.0, sigma, W, 0.1)
    o.set_state(np.zeros((10, n, n, n)), T.droplet((n, n, n), R, W))
    o.step(600)
    dP, R_eff, s = T.laplace(o.moments(), o.phi, R, W)
    assert dP > 0
    assert abs(s / sigma - 1) <= 0.10, (dP, R_eff, s)


def _diffuse_channel(phi_y, g, rho, nu):
    """Steady (mu u')' = -rho g across a channel with halfway walls (u = 0 at
    eta = 0 and ny), mu = rho nu blended from the given phi profile; second-
    order finite volumes on the lattice sites (a 1-D solve of the continuum
    equation, independent of the lattice Boltzmann arithmetic)."""
    ny = len(phi_y)
    r = rho[0] + phi_y * (rho[1] - rho[0])
    mu = r * (nu[0] + phi_y * (nu[1] - nu[0]))
    A = np.zeros((ny, ny))
    for y in range(ny):
        up = 0.5 * (mu[y] + mu[y + 1]) if y + 1 < ny else mu[y]
        dn = 0.5 * (mu[y] + mu[y - 1]) if y > 0 else mu[y]
        if y + 1 < ny:
            A[y, y + 1] += up
            A[y, y] -= up
        else:
            A[y, y] -= 2 * up  # ghost u = -u at the wall face
        if y > 0:
            A[y, y - 1] += dn
            A[y, y] -= dn
        else:
            A[y, y] -= 2 * dn
    return np.linalg.solve(A, -r * g)


def test_layered_channel_with_contrast(oracle_mod):
    """Two layers across a channel walled in y (the paper's layered
    Poiseuille case at small size): densities 0.5 / 1.5, viscosities 0.05 /
    0.4, sigma = 0.03, W = 4, body acceleration 1e-6, 6000 steps from rest.
    The steady profile solves (rho nu u')' = -rho g with rho, nu blended
    from the phase field; it matches a 1-D solve of that equation on the
    final phi profile to 2e-2 (measured 7e-3).  Dropping the viscous force
    term or flipping its sign gives errors of 20-70%."""
    from oracle import two_phase as T
    ny, g = 32, 1e-6
    shape = (4, ny, 4)
    o = T.TwoPhaseOracle(19, shape, 1.0, 0.03, 4.0, 0.1, body_force=(g, 0, 0), bc=(0, 1, 0),
                         rho=(0.5, 1.5), nu=(0.05, 0.4))
    o.set_state(np.zeros((10, 4, ny, 4)), T.layers(shape, 4.0))
    o.step(6000)
    u = o.moments()[1].mean(axis=(0, 2))
    want = _diffuse_channel(o.phi.mean(axis=(0, 2)), g, (0.5, 1.5), (0.05, 0.4))
    err = float(np.abs(u - want).max() / np.abs(want).max())
    assert err <= 2e-2, err
    assert np.abs(o.moments()[2:4]).max() <= 1e-3 * np.abs(u).max()


def test_phase_field_conserved_with_walls(oracle_mod):
    """Mirror images at the walls (normal flux components antisymmetric) keep
    the flux form of Eq. (2) exactly conservative for any velocity."""
    from oracle import two_phase as T
    rng = np.random.default_rng(8)
    phi = rng.uniform(0, 1, (7, 9, 6))
    u = 0.05 * rng.standard_normal((3, 7, 9, 6))
    for bc in ((0, 1, 0), (1, 1, 1)):
        p1 = T.phase_step(phi, u, 0.1, 4.0, bc=bc)
        assert abs(p1.sum() - phi.sum()) <= 1e-12 * phi.sum()
