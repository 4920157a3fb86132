"""The seeded input recipes, on the CPU: the solenoidal throughput field is
divergence-free, band-limited to 1 <= |k| <= 8 and has the stated magnitude
RMS; its on-device synthesis (used at 512^3) equals the NumPy recipe; the
Taylor-Green state is the printed vortex of section 4; seeds reproduce."""
import numpy as np
import pytest

from paper_2609_09160_amd import inputs


def _spectrum(u):
    """Per-component FFT of u[3, nz, ny, nx] and the integer wave numbers."""
    nz, ny, nx = u.shape[1:]
    U = np.fft.fftn(u, axes=(1, 2, 3))
    kz, ky, kx = np.meshgrid(np.fft.fftfreq(nz, 1.0 / nz), np.fft.fftfreq(ny, 1.0 / ny),
                             np.fft.fftfreq(nx, 1.0 / nx), indexing="ij")
    return U, kx, ky, kz


@pytest.mark.parametrize("shape", [(32, 32, 32), (40, 24, 36)])
def test_solenoidal_field_recipe(shape):
    m = inputs.solenoidal_field(shape)
    u = m[1:4]
    # magnitude RMS as stated
    assert abs(np.sqrt((u ** 2).sum(axis=0).mean()) - 0.02) <= 1e-15
    # p* = 0 and a2 = u u (zero non-equilibrium stress)
    assert np.abs(m[0]).max() == 0.0
    for k, (a, b) in zip(range(4, 10), ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        assert np.array_equal(m[k], u[a] * u[b])
    U, kx, ky, kz = _spectrum(u)
    # divergence-free mode by mode: k . u_hat = 0
    div = kx * U[0] + ky * U[1] + kz * U[2]
    assert np.abs(div).max() <= 1e-12 * np.abs(U).max()
    # energy only in 1 <= |k| <= 8
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    outside = (k2 < 1) | (k2 > 64)
    assert (np.abs(U[:, outside]) ** 2).sum() <= 1e-24 * (np.abs(U) ** 2).sum()
    assert (np.abs(U[:, k2 == 64]) ** 2).sum() > 0  # the band edge is populated


def test_solenoidal_field_device_synthesis_equals_recipe():
    """The on-device path (torch matmuls; run here on the CPU device) returns
    the NumPy recipe's field to rounding."""
    torch = pytest.importorskip("torch")
    shape = (20, 18, 16)
    want = inputs.solenoidal_field(shape)
    got = inputs.solenoidal_field(shape, device="cpu").numpy()
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()
    assert isinstance(inputs.solenoidal_field(shape, device="cpu"), torch.Tensor)


def test_taylor_green_is_the_printed_vortex():
    n, U0 = 16, 0.01
    m = inputs.taylor_green(n, U0)
    i, j, k = 3, 5, 7  # x, y, z indices, 0-based
    x, y, z = (2 * np.pi * v / n for v in (i, j, k))
    assert m[1, k, j, i] == pytest.approx(U0 * np.sin(x) * np.cos(y) * np.cos(z), abs=1e-18)
    assert m[2, k, j, i] == pytest.approx(-U0 * np.cos(x) * np.sin(y) * np.cos(z), abs=1e-18)
    assert m[3].max() == 0.0
    p = U0 ** 2 / 16 * (np.cos(2 * x) + np.cos(2 * y)) * (2 + np.cos(2 * z))
    assert m[0, k, j, i] == pytest.approx(3.0 * p, abs=1e-18)  # p* = p / cs^2
    assert abs(m[0].mean()) <= 1e-20  # zero-mean pressure
    U, kx, ky, kz = _spectrum(m[1:4])
    assert np.abs(kx * U[0] + ky * U[1] + kz * U[2]).max() <= 1e-12 * np.abs(U).max()


def test_seeds_reproduce_and_differ():
    shape = (6, 5, 4)
    assert np.array_equal(inputs.random_state(shape, seed=3), inputs.random_state(shape, seed=3))
    assert not np.array_equal(inputs.random_state(shape, seed=3),
                              inputs.random_state(shape, seed=4))
    assert np.array_equal(inputs.random_force(shape, seed=160), inputs.random_force(shape, seed=160))
    assert np.array_equal(inputs.solenoidal_field(shape), inputs.solenoidal_field(shape))
    assert not np.array_equal(inputs.solenoidal_field(shape, seed=1), inputs.solenoidal_field(shape))
    noise = inputs.channel_noise(shape)
    assert np.abs(noise[1:4]).max() <= 1e-4 and np.abs(noise[0]).max() == 0.0
