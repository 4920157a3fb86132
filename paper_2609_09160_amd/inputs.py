"""Seeded synthetic inputs (moment states and force fields).

This module holds input recipes only -- no part of the lattice Boltzmann
update.  It serves both the GPU path and the CPU oracle: every test and the
benchmark draw arrays here and hand the same arrays to both sides.

All states are returned as FP64 NumPy arrays of shape [10, nz, ny, nx] in the
moment order [p*, ux, uy, uz, a2xx, a2yy, a2zz, a2xy, a2xz, a2yz].  States
"at equilibrium" set the second-order coefficient to its equilibrium value
u u (Eq. (6) of the paper), i.e. zero non-equilibrium stress at t = 0.
"""
import numpy as np

CS2 = 1.0 / 3.0


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def equilibrium_state(pstar, u):
    """[10, ...] state with a2 = u u from p*[...] and u[3, ...]."""
    pstar = np.asarray(pstar, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    return np.stack([pstar, u[0], u[1], u[2],
                     u[0] * u[0], u[1] * u[1], u[2] * u[2],
                     u[0] * u[1], u[0] * u[2], u[1] * u[2]])


def taylor_green(n, U0):
    """Taylor-Green vortex of section 4, Eq. (11), on an n^3 periodic box.

    x = 2 pi i / n with 0-based i (the paper's 1-based (i-1)); pressure with
    zero mean as printed; p* = p / (rho cs^2) with rho = 1.
    """
    t = 2.0 * np.pi * np.arange(n) / n
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    ux = U0 * np.sin(x) * np.cos(y) * np.cos(z)
    uy = -U0 * np.cos(x) * np.sin(y) * np.cos(z)
    uz = np.zeros_like(ux)
    p = U0 ** 2 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (2.0 + np.cos(2 * z))
    return equilibrium_state(p / CS2, np.stack([ux, uy, uz]))


def shear_wave(shape, U0, kmode=1):
    """u_x = U0 sin(k y), k = 2 pi kmode / ny; p* = 0; a2 = u u."""
    nx, ny, nz = shape
    k = 2.0 * np.pi * kmode / ny
    y = np.arange(ny)[None, :, None] * np.ones((nz, 1, nx))
    ux = U0 * np.sin(k * y)
    zero = np.zeros_like(ux)
    return equilibrium_state(zero, np.stack([ux, zero, zero]))


def solenoidal_field(shape, kmax=8, urms=0.02, seed=9160, device=None):
    """Random divergence-free velocity from Gaussian Fourier modes, 1<=|k|<=kmax.

    Integer wave vectors k (|k| <= kmax, excluding 0) get complex Gaussian
    coefficients (PCG64(seed)), projected with I - k k / |k|^2; the field is the
    real part of the inverse transform, scaled so that sqrt(<|u|^2>) = urms.
    p* = 0, a2 = u u.  Returns a NumPy array, or a torch FP64 tensor on
    `device` when given (synthesis on the device; same coefficients).
    """
    nx, ny, nz = shape
    rng = _rng(seed)
    K = 2 * kmax + 1
    kk = np.arange(-kmax, kmax + 1)
    kz, ky, kx = np.meshgrid(kk, kk, kk, indexing="ij")
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    coef = rng.standard_normal((3, K, K, K)) + 1j * rng.standard_normal((3, K, K, K))
    kvec = np.stack([kx, ky, kz]).astype(np.float64)
    keep = (k2 >= 1) & (k2 <= kmax * kmax)
    k2s = np.where(k2 == 0, 1, k2)
    kdotc = (kvec * coef).sum(axis=0)
    coef = np.where(keep[None], coef - kvec * kdotc[None] / k2s[None], 0.0)

    if device is None:
        Ex, Ey, Ez = (np.exp(1j * 2.0 * np.pi * kk[:, None] * np.arange(n)[None, :] / n)
                      for n in (nx, ny, nz))
        u = np.empty((3, nz, ny, nx))
        for a in range(3):
            t = np.einsum("zyx,zk->kyx", coef[a], Ez)          # [nz, K, K]
            t = np.einsum("kyx,yj->kjx", t, Ey)                # [nz, ny, K]
            u[a] = np.einsum("kjx,xi->kji", t, Ex).real        # [nz, ny, nx]
        u *= urms / np.sqrt((u ** 2).sum(axis=0).mean())
        return equilibrium_state(np.zeros((nz, ny, nx)), u)

    import torch
    kt = torch.as_tensor(kk, dtype=torch.float64, device=device)
    Ex, Ey, Ez = (torch.exp(1j * 2.0 * np.pi * kt[:, None]
                            * torch.arange(n, dtype=torch.float64, device=device)[None, :] / n)
                  for n in (nx, ny, nz))
    EzT = Ez.t().contiguous()
    out = torch.empty((10, nz, ny, nx), dtype=torch.float64, device=device)
    for a in range(3):
        # contiguous operands only: sum over kz, then ky, then kx
        c = torch.as_tensor(coef[a].reshape(K, K * K), device=device)
        t = (EzT @ c).reshape(nz, K, K)                                 # [nz, ky, kx]
        t = (t.permute(0, 2, 1).contiguous() @ Ey)                       # [nz, kx, ny]
        t = t.permute(0, 2, 1).contiguous() @ Ex                         # [nz, ny, nx]
        out[1 + a] = t.real
    u = out[1:4]
    ms = (u * u).sum(dim=0).mean()
    u.mul_(urms / torch.sqrt(ms))
    out[0].zero_()
    out[4] = u[0] * u[0]
    out[5] = u[1] * u[1]
    out[6] = u[2] * u[2]
    out[7] = u[0] * u[1]
    out[8] = u[0] * u[2]
    out[9] = u[1] * u[2]
    return out


def channel_noise(shape, amp=1e-4, seed=2609):
    """Rest state plus uniform noise U(-amp, amp) on each velocity component."""
    nx, ny, nz = shape
    u = _rng(seed).uniform(-amp, amp, size=(3, nz, ny, nx))
    return equilibrium_state(np.zeros((nz, ny, nx)), u)


def random_state(shape, seed, amp=1e-2, neq=1e-3):
    """Generic off-equilibrium state: Gaussian p*, u (std amp) and a2 = u u plus
    a random symmetric non-equilibrium part (std neq).  For parity tests."""
    nx, ny, nz = shape
    r = _rng(seed)
    p = amp * r.standard_normal((nz, ny, nx))
    u = amp * r.standard_normal((3, nz, ny, nx))
    m = equilibrium_state(p, u)
    m[4:] += neq * r.standard_normal((6, nz, ny, nx))
    return m


def random_force(shape, seed=160, std=1e-6):
    """Per-site Gaussian body-force field [3, nz, ny, nx]."""
    nx, ny, nz = shape
    return std * _rng(seed).standard_normal((3, nz, ny, nx))
