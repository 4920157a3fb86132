"""Pins of the two-component oracle (oracle/two_phase.py): the D3Q27-weighted
derivative stencils against their exact discrete Fourier symbols, exact
conservation of the phase field and of momentum with a force that changes
every step, the exact drift of a droplet under uniform advection, the
planar equilibrium of Eq. (2), the Laplace law, and (density and viscosity
contrast, walls) the steady layered channel against a 1-D solve of the
continuum equation, the hydrostatic column (pressure force), uniform
acceleration across a contrast interface and closed forms on prescribed
fields (viscous and pressure forces), and the wall images of the stencils
on modes they continue exactly."""
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


def _column_state(ny, W, rho, g, P0):
    """Two layers across a channel walled in y, the heavy phase below, in the
    continuum hydrostatic equilibrium of body acceleration -g along y: p =
    rho cs^2 p* continuous, dp/dy = -rho g (trapezoid sums of rho)."""
    from oracle import two_phase as T
    shape = (4, ny, 4)
    phi = 1.0 - T.layers(shape, W)
    r = rho[0] + phi[0, :, 0] * (rho[1] - rho[0])
    p = P0 - g * np.concatenate([[0.0], np.cumsum(0.5 * (r[1:] + r[:-1]))])
    m = np.zeros((10, 4, ny, 4))
    m[0] = (p / (r / 3.0))[None, :, None]
    return shape, phi, m


def test_hydrostatic_column_pressure_force(oracle_mod):
    """Pressure force F^p = -p* cs^2 grad(rho) (section 2, force split): with
    it, the momentum equation at rest reads grad(rho cs^2 p*) = rho g, so the
    pressure p = rho cs^2 p* is continuous across an interface of density
    contrast and rises by rho_k g per site in each layer.  Walled column 4 x
    32 x 4, densities 0.5 / 1.5 (heavy below), viscosities 0.1 / 0.2, g =
    1e-5, background pressure 3e-3, 3000 steps from the continuum
    equilibrium: the state stays at rest (|u| <= 1e-6), the pressure jump
    across the interface (the two layers' linear fits extrapolated to the
    middle) is below 5e-2 of the background pressure (measured 2.4e-5 against
    3e-3) and the layer slopes are rho_k g within 6% (0.996 and 0.959).
    Without F^p the layers keep p* continuous instead, and p jumps by about
    the background pressure (-3.6e-3); with F^p of the wrong sign the column
    moves at 3e-4 and the jump is -7.2e-3."""
    from oracle import two_phase as T
    ny, W, rho, g, P0 = 32, 4.0, (0.5, 1.5), 1e-5, 3e-3
    shape, phi, m = _column_state(ny, W, rho, g, P0)
    o = T.TwoPhaseOracle(19, shape, 1.0, 0.0, W, 0.1, body_force=(0, -g, 0), bc=(0, 1, 0),
                         rho=rho, nu=(0.1, 0.2))
    o.set_state(m, phi)
    o.step(3000)
    mm = o.moments()
    assert np.abs(mm[1:4]).max() <= 1e-6
    php = o.phi.mean(axis=(0, 2))
    p = (rho[0] + php * (rho[1] - rho[0])) * mm[0].mean(axis=(0, 2)) / 3.0
    y = np.arange(ny)
    lo = np.polyfit(y[2:10], p[2:10], 1)
    hi = np.polyfit(y[22:30], p[22:30], 1)
    ym = ny / 2 - 0.5
    jump = np.polyval(hi, ym) - np.polyval(lo, ym)
    assert abs(jump) <= 5e-2 * P0, jump
    assert abs(lo[0] / (-rho[1] * g) - 1) <= 0.06, lo[0]
    assert abs(hi[0] / (-rho[0] * g) - 1) <= 0.06, hi[0]


def test_uniform_acceleration_across_contrast(oracle_mod):
    """A uniformly accelerated flow carries no shear, so the viscous force term
    F^nu must vanish on it even where the density varies.  Periodic 4 x 24 x
    4 box, a slab of the light phase between tanh interfaces normal to y
    (densities 0.5 / 1.5, viscosities 0.05 / 0.4), uniform velocity (0.01,
    0.02, -0.005) crossing the interfaces, p* = 0, a2 = u u, body
    acceleration (0, 1e-4, 0), no surface tension: the velocity stays
    u0 + g t at every site for 200 steps (1e-13; measured 3e-16) while the
    slab is carried along.  This fixes the non-equilibrium coefficient in
    F^nu to a2 - u u: subtracting the force part (F u + u F)/(2 rho) as
    well (a pre-correction coefficient read against the corrected u) leaves
    a viscous force on the interfaces and an error of 2.7e-6 here."""
    from oracle import two_phase as T
    nx, ny, nz, W = 4, 24, 4, 4.0
    eta = np.arange(ny) + 0.5
    prof = 0.5 * (1 + np.tanh(2 * (np.abs(eta - ny / 2) - 6) / W))
    phi = np.broadcast_to(prof[None, :, None], (nz, ny, nx)).copy()
    g = np.array([0.0, 1e-4, 0.0])
    u0 = np.array([0.01, 0.02, -0.005])
    m = np.zeros((10, nz, ny, nx))
    for a in range(3):
        m[1 + a] = u0[a]
    for k, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        m[4 + k] = u0[a] * u0[b]
    o = T.TwoPhaseOracle(19, (nx, ny, nz), 1.0, 0.0, W, 0.1, body_force=g, rho=(0.5, 1.5),
                         nu=(0.05, 0.4))
    o.set_state(m, phi)
    o.step(200)
    mm = o.moments()
    want = (u0 + 200 * g)[:, None, None, None]
    assert np.abs(mm[1:4] - want).max() <= 1e-13
    assert np.abs(mm[0]).max() <= 1e-13
    assert np.abs(o.phi - phi).max() > 0.5  # the interfaces did move


def test_contrast_force_closed_forms(oracle_mod):
    """The pressure and viscous terms of the force split on prescribed fields.
    phi = 0.5 + 0.4 sin(k y) (periodic, so the gradient stencil gives exactly
    sin(k) 0.4 cos(k y), pinned above), densities 0.5 / 1.5, viscosities
    0.05 / 0.4.  Viscous term: a2 = u u + A with A the non-equilibrium
    coefficient of a simple shear of rate gamma, A_xy = -(cs^2/omega) gamma
    (Eq. (6) without force); the continuum viscous term nu (grad u + grad
    u^T) . grad(rho) is then nu gamma d_y rho along x, nothing along y or z.
    Pressure term: a uniform p* = P gives -P cs^2 d_y rho along y, i.e. the
    part of grad(rho cs^2 p*) that the lattice equation does not carry."""
    from oracle import two_phase as T
    nx, ny, nz = 3, 16, 2
    N = nx * ny * nz
    k = 2 * np.pi / ny
    y = np.arange(ny)
    phi = np.broadcast_to((0.5 + 0.4 * np.sin(k * y))[None, :, None], (nz, ny, nx)).copy()
    rho, nu_lh = (0.5, 1.5), (0.05, 0.4)
    o = T.TwoPhaseOracle(19, (nx, ny, nz), 1.0, 0.0, 4.0, 0.1, rho=rho, nu=nu_lh)
    nu = nu_lh[0] + phi * (nu_lh[1] - nu_lh[0])
    omega = 1.0 / (3.0 * nu + 0.5)
    drho = (rho[1] - rho[0]) * 0.4 * np.sin(k) * np.cos(k * y)[None, :, None]
    u = np.array([0.01, -0.02, 0.015])
    gamma, P = 3e-3, 0.2
    m = np.zeros((10, nz, ny, nx))
    m[0] = P
    for a in range(3):
        m[1 + a] = u[a]
    for j, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        m[4 + j] = u[a] * u[b]
    m[7] += -(1.0 / 3.0) / omega * gamma
    F = o._force(phi, m).reshape(3, nz, ny, nx)
    assert np.abs(F[0] - nu * gamma * drho).max() <= 1e-15
    assert np.abs(F[1] - (-P / 3.0) * drho).max() <= 1e-15
    assert np.abs(F[2]).max() <= 1e-15


def _mirror_modes(ny):
    """Modes that the halfway-wall mirror images continue exactly: even
    cos(q (y + 1/2)) and odd sin(q (y + 1/2)), q = pi j / ny."""
    q = np.pi * 3 / ny
    eta = np.arange(ny) + 0.5
    return q, np.cos(q * eta), np.sin(q * eta)


def test_wall_ghosts_scalar_stencils(oracle_mod):
    """With walls in y the stencils read the mirror image of the wall-side
    site beyond the wall.  A scalar mode cos(q (y + 1/2)) with q = 3 pi / ny
    is continued exactly by those images, so on every row, the wall rows
    included, the stencils give their exact symbols: along y the averaging
    A(q) = 2/3 + cos(q)/3 and the derivative -sin(q) sin(q (y + 1/2)); the
    Laplacian 6 (A_x A_y A_z - 1) times the mode (the D3Q27 weights are the
    product of one-dimensional ones).  Zero, periodic or unreflected ghosts
    fail at the wall rows."""
    from oracle import two_phase as T
    nx, ny, nz = 8, 12, 6
    q, ev, _ = _mirror_modes(ny)
    kx, kz = 2 * np.pi / nx, 2 * np.pi * 2 / nz
    X = np.cos(kx * np.arange(nx) + 0.4)
    Z = np.sin(kz * np.arange(nz) + 0.1)
    psi = Z[:, None, None] * ev[None, :, None] * X[None, None, :]
    A = lambda k: 2.0 / 3.0 + np.cos(k) / 3.0  # noqa: E731
    bc = (0, 1, 0)
    gr = T.grad(psi, bc)
    Xd = -np.sin(kx) * np.sin(kx * np.arange(nx) + 0.4)
    Zd = np.sin(kz) * np.cos(kz * np.arange(nz) + 0.1)
    Yd = -np.sin(q) * np.sin(q * (np.arange(ny) + 0.5))
    want_x = A(kz) * A(q) * Z[:, None, None] * ev[None, :, None] * Xd[None, None, :]
    want_y = A(kz) * A(kx) * Z[:, None, None] * Yd[None, :, None] * X[None, None, :]
    want_z = A(q) * A(kx) * Zd[:, None, None] * ev[None, :, None] * X[None, None, :]
    for got, want in zip(gr, (want_x, want_y, want_z)):
        assert np.abs(got - want).max() <= 1e-14
    lap_want = 6.0 * (A(kx) * A(q) * A(kz) - 1.0) * psi
    assert np.abs(T.lap(psi, bc) - lap_want).max() <= 1e-14


def test_wall_ghosts_normal_flux(oracle_mod):
    """The flux of Eq. (2) through a wall: the image of the wall-normal flux
    component is reversed (no flux through the wall), the tangential ones are
    kept.  With phi = 1, D = 0 (so no diffusion and no compression) and a
    velocity whose wall-normal part is the odd mode sin(q (y + 1/2)) and whose
    tangential part is an even mode, one step gives phi' = 1 - div(u) with the
    exact symbols on every row: the normal part contributes sin(q) cos(q (y +
    1/2)) A_x A_z, the tangential x part A_y A_z times its x derivative."""
    from oracle import two_phase as T
    nx, ny, nz = 8, 12, 6
    q, ev, od = _mirror_modes(ny)
    kx = 2 * np.pi / nx
    X = np.cos(kx * np.arange(nx))
    A = lambda k: 2.0 / 3.0 + np.cos(k) / 3.0  # noqa: E731
    u = np.zeros((3, nz, ny, nx))
    u[1] = 0.01 * od[None, :, None] * X[None, None, :]
    u[0] = 0.02 * ev[None, :, None] * np.sin(kx * np.arange(nx))[None, None, :]
    phi = np.ones((nz, ny, nx))
    p1 = T.phase_step(phi, u, 0.0, 4.0, bc=(0, 1, 0))
    div_y = 0.01 * np.sin(q) * ev[None, :, None] * X[None, None, :] * A(kx) * A(0.0)
    dsx = np.sin(kx) * np.cos(kx * np.arange(nx))
    div_x = 0.02 * A(q) * A(0.0) * ev[None, :, None] * dsx[None, None, :]
    assert np.abs(p1 - (1.0 - div_y - div_x)).max() <= 1e-15
