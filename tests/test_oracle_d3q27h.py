"""Pins of the oracle's D3Q27h model: the D3Q27 velocity set with the series
of Eq. (4) over the complete Hermite basis (orders up to 6), coefficients of
order >= 3 from the recursive closures the paper cites in section 2 (Shan et
al. for the equilibrium, Malaspinas for the non-equilibrium part).

The oracle builds those terms from generic Hermite tensors and the two
recursions.  The pins below use none of that:
  * the full-basis equilibrium on D3Q27 equals w_i (p* - 1) plus the product
    of three one-dimensional D1Q3 equilibria g(c_a; u_a) (the tensor-product
    basis factorises, and the 1-D coefficients are 1, u, u^2);
  * the recursive non-equilibrium closure is, component by component, a sum
    over index pairs of a2neq times the remaining velocities, which is
    (1/2) A : grad_u grad_u of the equilibrium coefficients; so the relaxed
    part is (1 - omega) (1/2) A : grad_u grad_u of that product;
  * a shear wave advected by a uniform flow decays at the rest-frame rate
    (the third-order equilibrium terms the second-order sets lack are what
    makes the viscous stress Galilean invariant in this configuration).
"""
import numpy as np
import pytest



def _g(c, u):
    """D1Q3 equilibrium with unit density, velocity u, cs^2 = 1/3."""
    return np.where(c == 0, 2.0 / 3.0 - u * u, (1.0 / 3.0 + u * u + c * u) / 2.0)


def _dg(c, u):
    return np.where(c == 0, -2.0 * u, u + c / 2.0)


def _ddg(c):
    return np.where(c == 0, -2.0, 1.0)


def _closed_form(oracle_mod, m, F, tau):
    """w (p* - 1) + G(u) + (1 - omega) (1/2) A : grad grad G(u) + S / 2 with
    G = prod_a g(c_a; u_a), A = a2 - u u and S the Guo term of Eq. (9)."""
    c, w = oracle_mod.lattice_tables(27)
    p, u = m[0], m[1:4]
    a2 = np.array([[m[4], m[7], m[8]], [m[7], m[5], m[9]], [m[8], m[9], m[6]]])
    A = a2 - np.outer(u, u)
    e = [_g(c[:, a], u[a]) for a in range(3)]
    d = [_dg(c[:, a], u[a]) for a in range(3)]
    s = [_ddg(c[:, a]) for a in range(3)]
    G = e[0] * e[1] * e[2]
    N = np.zeros(27)
    for a in range(3):
        for b in range(3):
            if a == b:
                t = s[a] * e[(a + 1) % 3] * e[(a + 2) % 3]
            else:
                t = d[a] * d[b] * e[3 - a - b]
            N += 0.5 * A[a, b] * t
    S = w * (3.0 * ((c - u) @ F) + 9.0 * (c @ u) * (c @ F))
    return w * (p - 1.0) + G + (1.0 - 1.0 / tau) * N + 0.5 * S


def _site_state(rng, A_scale):
    m = np.zeros(10)
    m[0] = 0.01 * rng.standard_normal()
    m[1:4] = 0.1 * rng.standard_normal(3)
    A = A_scale * rng.standard_normal((3, 3))
    a2 = np.outer(m[1:4], m[1:4]) + A + A.T
    m[4:7] = np.diag(a2)
    m[7], m[8], m[9] = a2[0, 1], a2[0, 2], a2[1, 2]
    return m


def _post_collision(oracle_mod, lattice, m, F, tau):
    o = oracle_mod.PopulationOracle(lattice, (1, 1, 1), tau, force=F)
    o.set_moments(m.reshape(10, 1, 1, 1))
    return o.post_collision()[:, 0]


def test_equilibrium_is_product_of_1d_equilibria(oracle_mod):
    """a2 = u u, F = 0: the post-collision populations are the full-basis
    equilibrium, w_i (p* - 1) + prod_a g(c_ia; u_a), to round-off.  A wrong
    Hermite tensor, normalisation or multiplicity at any order 3..6 fails."""
    rng = np.random.default_rng(31)
    for _ in range(5):
        m = _site_state(rng, 0.0)
        got = _post_collision(oracle_mod, "27h", m, np.zeros(3), 0.8)
        want = _closed_form(oracle_mod, m, np.zeros(3), 0.8)
        assert np.abs(got - want).max() <= 2e-16


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.7])
def test_non_equilibrium_closure_second_derivative(oracle_mod, tau):
    """Random off-equilibrium a2 and a force: the post-collision populations
    equal the closed form with (1 - omega) (1/2) A : grad_u grad_u G, to
    round-off.  A wrong sign, a missing pair term or a wrong index in the
    recursive closure at any order fails (the high-order terms change the
    populations by ~1e-3 here, against a bar of 2e-16)."""
    rng = np.random.default_rng(32)
    for _ in range(5):
        m = _site_state(rng, 0.01)
        F = 1e-3 * rng.standard_normal(3)
        got = _post_collision(oracle_mod, "27h", m, F, tau)
        want = _closed_form(oracle_mod, m, F, tau)
        assert np.abs(got - want).max() <= 2e-16
        second = _post_collision(oracle_mod, 27, m, F, tau)
        assert np.abs(got - second).max() >= 1e-5


def test_added_orders_are_invisible_to_the_moments(oracle_mod):
    """The orders 3..6 are orthogonal to H0, H1 and H2 under the D3Q27
    weights: the D3Q27h and D3Q27 post-collision populations differ, but
    their projections on the ten stored moments agree to round-off.  At
    u = 0 every added coefficient vanishes and the two models coincide."""
    c, w = oracle_mod.lattice_tables(27)
    H2 = np.einsum("ia,ib->iab", c, c) - np.eye(3) / 3.0
    rng = np.random.default_rng(33)
    for _ in range(5):
        m = _site_state(rng, 0.01)
        F = 1e-3 * rng.standard_normal(3)
        diff = (_post_collision(oracle_mod, "27h", m, F, 0.7)
                - _post_collision(oracle_mod, 27, m, F, 0.7))
        assert np.abs(diff).max() >= 1e-5
        assert abs(diff.sum()) <= 1e-17
        assert np.abs(c.T @ diff).max() <= 1e-17
        assert np.abs(np.einsum("iab,i->ab", H2, diff)).max() <= 1e-17
        m[1:4] = 0.0
        still = (_post_collision(oracle_mod, "27h", m, F, 0.7)
                 - _post_collision(oracle_mod, 27, m, F, 0.7))
        assert np.abs(still).max() <= 1e-17


def test_advected_shear_wave_galilean_invariant(oracle_mod):
    """Shear wave u_y = 1e-4 sin(2 pi x / 32) carried by a uniform u_x = U0,
    tau = 0.8: the fitted viscosity (amplitude decay over t in [100, 400])
    deviates from its U0 = 0 value by < 2e-4 up to U0 = 0.2 with the full
    basis, while the second-order D3Q27 model shows the known O(U0^2) error
    (-12% at U0 = 0.2).  Dropping the third-order equilibrium terms, or
    giving them the wrong sign, puts the full-basis model back to (or beyond)
    the second-order error."""
    nx, tau = 32, 0.8
    nu, k = (tau - 0.5) / 3.0, 2 * np.pi / nx
    x = np.arange(nx)

    def fitted_nu(lattice, U0):
        uy = 1e-4 * np.sin(k * x)
        m = np.zeros((10, 1, 1, nx))
        m[1], m[2] = U0, uy
        m[4], m[5], m[7] = U0 * U0, uy * uy, U0 * uy
        o = oracle_mod.PopulationOracle(lattice, (nx, 1, 1), tau)
        o.set_moments(m)
        amp = []
        for t in (100, 300):
            o.step(t)
            amp.append(abs(np.sum(o.moments()[2, 0, 0] * np.exp(-1j * k * x))))
        return -np.log(amp[1] / amp[0]) / (300 * k * k)

    rest = fitted_nu("27h", 0.0)
    assert abs(rest / nu - 1) < 1e-3
    for U0 in (0.1, 0.2):
        assert abs(fitted_nu("27h", U0) / rest - 1) < 2e-4
    assert fitted_nu(27, 0.2) / rest - 1 < -0.1


def test_d3q27h_poiseuille_profile_unchanged(oracle_mod):
    """Body-force channel between y walls, u_x(y) only: the added orders
    change a2_xx (by ~0.3% here, through a3neq_xxy = 2 u_x a2neq_xy), which
    has no x-gradient to act through, and leave a2_xy and the velocity
    profile as in the second-order set, to round-off."""
    H, g, tau = 16, 1e-6, 0.9
    out = []
    for lat in (27, "27h"):
        o = oracle_mod.PopulationOracle(lat, (1, H, 1), tau, bc=(0, 1, 0), force=[g, 0, 0])
        o.set_moments(np.zeros((10, 1, H, 1)))
        o.step(3000)
        out.append(o.moments()[:, 0, :, 0])
    ux, axx, axy = (np.abs(out[0][k]).max() for k in (1, 4, 7))
    assert np.abs(out[1][1] - out[0][1]).max() <= 1e-12 * ux
    assert np.abs(out[1][7] - out[0][7]).max() <= 1e-10 * axy
    assert np.abs(out[1][4] - out[0][4]).max() >= 1e-4 * axx
