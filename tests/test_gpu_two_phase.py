"""The two-component variant on the GPU (phase field by the conservative
Allen-Cahn equation, capillary force, fused step with the force of each time
level) against the FP64 two-component oracle, and the Laplace law at the
256^3 droplet workload.

Bars: FP64 -- element-wise <= 1e-12 of each moment group's and of phi's
magnitude (equal phases, and density and viscosity contrast with walls).  FP32 -- against the oracle, p* and phi <= 1e-4 relative L2 after
100 steps, u <= 2e-3 (below), the pressure jump <= 1e-6 once the droplet is
static; at the 256^3 workload the pressure jump within 1e-4 of the FP64 run.
16-bit storage -- the pressure jump within 5e-3 (FP16) and 2e-2 (BF16) of the
FP64 run (below)."""
import numpy as np
import pytest

from gpu_util import group_rel_err, lattice_number, say

pytestmark = pytest.mark.gpu

SIGMA, W, DIFF = 0.03, 4.0, 0.1


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def gpu_two_phase(shape, tau, m0, phi0, steps, lattice=19, storage="f64", force=(0, 0, 0),
                  scale=None, every=None, sites=0, bc=(0, 0, 0), rho=(1.0, 1.0), taus=None):
    """Moments [10, nz, ny, nx] and phi [nz, ny, nx] (host float64) after
    `steps`; with `every`, also the per-plane max |v| sampled every `every`
    steps."""
    from paper_2609_09160_amd import Solver
    s = Solver(shape, tau, lattice=lattice, storage=storage, force=force, scale=scale, bc=bc)
    s.enable_two_phase(SIGMA, W, DIFF, rho=rho, tau=taus if taus is not None else tau)
    if sites:  # after enabling: the variant picks its own default shape
        s.set_launch(4, 0, sites)
    s.set_moments(np.ascontiguousarray(m0))
    s.set_phase(np.ascontiguousarray(phi0))
    peaks = np.zeros(10)
    if every:
        for _ in range(steps // every):
            s.step(every)
            m = s.moments()
            peaks = np.maximum(peaks, m.abs().amax(dim=(1, 2, 3)).cpu().numpy())
    else:
        s.step(steps)
    m, phi = s.moments().cpu().numpy(), s.phase().cpu().numpy()
    s.close()
    return m, phi, peaks


def oracle_two_phase(shape, tau, m0, phi0, steps, lattice=19, force=None, bc=(0, 0, 0),
                     rho=(1.0, 1.0), nu=None):
    from oracle import two_phase as T
    o = T.TwoPhaseOracle(lattice, shape, tau, SIGMA, W, DIFF, body_force=force, bc=bc, rho=rho,
                         nu=nu)
    o.set_state(m0, phi0)
    o.step(steps)
    return o.moments(), o.phi


def _droplet_state(shape, R, seed, noise=True):
    from oracle import two_phase as T
    nx, ny, nz = shape
    phi = T.droplet(shape, R, W)
    m = np.zeros((10, nz, ny, nx))
    if noise:
        rng = np.random.default_rng(seed)
        m[0] = 1e-3 * rng.standard_normal((nz, ny, nx))
        m[1:4] = 1e-3 * rng.standard_normal((3, nz, ny, nx))
        m[4:] = 1e-4 * rng.standard_normal((6, nz, ny, nx))
        for a, b, k in ((0, 0, 4), (1, 1, 5), (2, 2, 6), (0, 1, 7), (0, 2, 8), (1, 2, 9)):
            m[k] += m[1 + a] * m[1 + b]
    return m, phi


@pytest.mark.parametrize("sites", [1, 2])
@pytest.mark.parametrize("Q", [19, 27, "27h"])
def test_two_phase_parity_fp64(Q, sites):
    """70 x 21 x 18 (ragged), off-centre droplet R = 6 with a perturbed flow
    and a uniform body force, 30 steps, FP64, one or two x-sites per lane:
    moments and phi element-wise."""
    shape = (70, 21, 18)
    m0, _ = _droplet_state(shape, 6, seed=lattice_number(Q))
    from oracle import two_phase as T
    phi0 = T.droplet(shape, 6, W, center=(30.3, 10.1, 8.7))
    Fb = (2e-6, -1e-6, 5e-7)
    say(f"two-phase fp64 parity Q{Q} sites={sites}")
    got, gphi, _ = gpu_two_phase(shape, 0.8, m0, phi0, 30, lattice=Q, force=Fb, sites=sites)
    want, wphi = oracle_two_phase(shape, 0.8, m0, phi0, 30, lattice=Q, force=np.array(Fb))
    em = group_rel_err(got, want)
    ep = float(np.abs(gphi - wphi).max() / np.abs(wphi).max())
    say(f"  moments {em:.2e}, phi {ep:.2e}")
    assert em <= 1e-12 and ep <= 1e-12


@pytest.mark.parametrize("shape", [(7, 5, 3), (3, 2, 1), (65, 9, 2), (1, 17, 9)])
@pytest.mark.parametrize("walls", [False, True])
def test_two_phase_small_and_thin_grids(shape, walls):
    """Grids smaller than one 64 x 8 stencil tile, a single z-plane, two
    z-planes and a single x column, periodic or walled in y: the staged
    phase-field passes (one plane of records in LDS, rolling accumulators
    over three destination planes) wrap and mirror their halos within the
    grid.  Random phase field in [0.2, 0.8] and off-equilibrium flow, density
    and viscosity contrast, 5 steps, FP64: element-wise against the oracle."""
    if walls and shape[1] < 2:
        pytest.skip("a walled axis needs >= 2 sites")
    nx, ny, nz = shape
    rng = np.random.default_rng(sum(shape) + 7 * walls)
    phi0 = 0.2 + 0.6 * rng.random((nz, ny, nx))
    m0, _ = _droplet_state(shape, 1, seed=sum(shape))
    bc = (0, 1 if walls else 0, 0)
    g = (2e-6, -1e-6, 5e-7)
    say(f"two-phase small grid {shape} walls={walls}")
    got, gphi, _ = gpu_two_phase(shape, 1.0, m0, phi0, 5, force=g, bc=bc, rho=(0.5, 1.5),
                                 taus=(0.65, 1.7))
    want, wphi = oracle_two_phase(shape, 1.0, m0, phi0, 5, force=np.array(g), bc=bc,
                                  rho=(0.5, 1.5), nu=(0.05, 0.4))
    em = group_rel_err(got, want)
    ep = float(np.abs(gphi - wphi).max() / np.abs(wphi).max())
    say(f"  moments {em:.2e}, phi {ep:.2e}")
    assert em <= 1e-12 and ep <= 1e-12


@pytest.mark.parametrize("steps", [100, 600])
def test_two_phase_parity_fp32_laplace_32(steps):
    """The oracle's Laplace case (32^3, R = 8, tau = 1, from rest) in FP32
    against the FP64 oracle.  After 100 steps p* and phi agree to 1e-4
    (relative L2).  The velocity is the small residual of the balance between
    the capillary force and the pressure gradient, and mu itself is a
    difference of two terms ~100x larger than it, so FP32 rounding reaches u
    amplified by about that factor: u is held to 2e-3.  By 600 steps the
    droplet is static and its residual velocities are mostly that rounding, so
    the comparison is on what the method measures: the pressure jump (1e-6)
    and phi (1e-3)."""
    from oracle import two_phase as T
    n, R = 32, 8
    shape = (n, n, n)
    m0, phi0 = _droplet_state(shape, R, 0, noise=False)
    got, gphi, _ = gpu_two_phase(shape, 1.0, m0, phi0, steps, storage="f32")
    want, wphi = oracle_two_phase(shape, 1.0, m0, phi0, steps)
    e_p = float(np.linalg.norm(got[0] - want[0]) / np.linalg.norm(want[0]))
    e_u = float(np.linalg.norm(got[1:4] - want[1:4]) / np.linalg.norm(want[1:4]))
    e_phi = float(np.linalg.norm(gphi - wphi) / np.linalg.norm(wphi))
    dg = T.laplace(got, gphi, R, W)[0]
    dw = T.laplace(want, wphi, R, W)[0]
    say(f"fp32 32^3 droplet, {steps} steps: p* {e_p:.2e}, u {e_u:.2e} (|u|max "
        f"{np.abs(want[1:4]).max():.2e}), phi {e_phi:.2e}, dP rel {abs(dg / dw - 1):.2e}")
    if steps <= 100:
        assert e_p <= 1e-4 and e_u <= 2e-3 and e_phi <= 1e-4
    else:
        assert abs(dg / dw - 1) <= 1e-6 and e_phi <= 1e-3


_C4 = {}


def _c4(storage, scale=None):
    """The droplet workload: D3Q19 256^3 periodic, R = 40 centred, W = 4,
    sigma = 0.03, D = 0.1, equal densities, tau = 1, 5000 steps from rest."""
    if storage not in _C4:
        from oracle import two_phase as T
        n, R = 256, 40
        shape = (n, n, n)
        m0, phi0 = _droplet_state(shape, R, 0, noise=False)
        say(f"droplet 256^3 {storage}")
        m, phi, peaks = gpu_two_phase(shape, 1.0, m0, phi0, 5000, storage=storage, scale=scale,
                                      every=500 if storage == "f32" else None)
        dP, R_eff, sig = T.laplace(m, phi, R, W)
        _C4[storage] = dict(dP=dP, R_eff=R_eff, sigma=sig, peaks=peaks, mass=phi.sum())
        say(f"  dP {dP:.6e}, R_eff {R_eff:.4f}, sigma {sig:.5f}")
    return _C4[storage]


def test_laplace_256_fp32_and_fp64():
    """Laplace law at the droplet workload: sigma = dP R_eff / 2 within 10% of
    the input (the paper: -6.8% at R = 64); the FP32 pressure jump within
    1e-4 of the FP64 run, which the parity test above ties to the oracle
    (FP32 unit roundoff 6e-8 accumulated over 5000 steps: 4e-6 as a random
    walk, 3e-4 if every step's error had the same sign); total phase
    conserved."""
    r32, r64 = _c4("f32"), _c4("f64")
    say(f"sigma {r32['sigma']:.5f}, FP32 vs FP64 dP {abs(r32['dP'] / r64['dP'] - 1):.2e}")
    assert abs(r32["sigma"] / SIGMA - 1) <= 0.10
    assert abs(r32["dP"] / r64["dP"] - 1) <= 1e-4
    from oracle import two_phase as T
    m0 = T.droplet((256, 256, 256), 40, W).sum()
    assert abs(r64["mass"] / m0 - 1) <= 1e-12
    assert abs(r32["mass"] / m0 - 1) <= 1e-5


@pytest.mark.parametrize("storage,bar", [("f16s", 5e-3), ("bf16s", 2e-2)])
def test_laplace_256_16bit(storage, bar):
    """The same workload with 16-bit scaled moment storage (FP32 arithmetic;
    per-plane scales from the FP32 run's peak magnitudes with 4x headroom,
    the run starting at rest): pressure jump against the FP64 one.  Every
    moment is re-rounded each step (unit roundoff 2^-12 for FP16, 2^-9 for
    BF16) while the static droplet's pressure settles only through viscous
    damping of the flow over thousands of steps: measured 2.4e-3 (FP16) and
    1.1e-2 (BF16), held to about twice that."""
    peaks = _c4("f32")["peaks"]
    scale = []
    for v in peaks:
        e = int(np.ceil(np.log2(max(4.0 * v, 1e-30))))
        scale.append(2.0 ** (e - 15))
    r = _c4(storage, scale=scale)
    d = abs(r["dP"] / _c4("f64")["dP"] - 1)
    say(f"{storage}: dP relative to FP64 {d:.2e}")
    assert d <= bar


@pytest.mark.parametrize("sites", [1, 2])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("Q", [19, 27, "27h"])
def test_contrast_parity_fp64(Q, walls, sites):
    """Density and viscosity contrast (rho 0.5 / 1.5, nu 0.05 / 0.4), body
    acceleration, periodic or y walls, 70 x 21 x 18, off-centre droplet with
    a perturbed flow, 30 steps, FP64: moments and phi element-wise against
    the two-component oracle."""
    from oracle import two_phase as T
    shape = (70, 21, 18)
    m0, _ = _droplet_state(shape, 6, seed=lattice_number(Q) + 3)
    phi0 = T.droplet(shape, 6, W, center=(30.3, 10.1, 8.7))
    g = (2e-6, -1e-6, 5e-7)
    bc = (0, 1 if walls else 0, 0)
    say(f"contrast fp64 parity Q{Q} walls={walls} sites={sites}")
    got, gphi, _ = gpu_two_phase(shape, 1.0, m0, phi0, 30, lattice=Q, force=g, sites=sites, bc=bc,
                                 rho=(0.5, 1.5), taus=(0.65, 1.7))
    want, wphi = oracle_two_phase(shape, 1.0, m0, phi0, 30, lattice=Q, force=np.array(g), bc=bc,
                                  rho=(0.5, 1.5), nu=(0.05, 0.4))
    em = group_rel_err(got, want)
    ep = float(np.abs(gphi - wphi).max() / np.abs(wphi).max())
    say(f"  moments {em:.2e}, phi {ep:.2e}")
    assert em <= 1e-12 and ep <= 1e-12


def _diffuse_channel(phi_y, g, rho, nu):
    """Steady (mu u')' = -rho g across a channel with halfway walls, mu =
    rho nu blended from the phi profile (1-D finite volumes; see the oracle
    pin of the same case)."""
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
            A[y, y] -= 2 * up
        if y > 0:
            A[y, y - 1] += dn
            A[y, y] -= dn
        else:
            A[y, y] -= 2 * dn
    return np.linalg.solve(A, -r * g)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_layered_channel_128(storage):
    """The paper's layered Poiseuille benchmark at H = 128 (the paper: 512):
    walls in y, light phase (rho 0.5, nu 0.05) below the middle, heavy
    (rho 1.5, nu 0.4) above, sigma = 0.03, W = 4, body acceleration 1e-6
    along x, 80000 steps from rest to steady state.  The profile matches a
    1-D solve of (rho nu u')' = -rho g on the final phase profile to 1e-2;
    against the sharp-interface solution the largest error sits at the
    interface (the paper: 4.18e-2 at H = 512, D3Q19)."""
    from oracle import two_phase as T
    ny, g = 128, 1e-6
    shape = (8, ny, 8)
    m0 = np.zeros((10, 8, ny, 8))
    phi0 = T.layers(shape, W)
    say(f"layered channel {storage}")
    m, phi, _ = gpu_two_phase(shape, 1.0, m0, phi0, 80000, storage=storage, force=(g, 0, 0),
                              bc=(0, 1, 0), rho=(0.5, 1.5), taus=(0.65, 1.7))
    u = m[1].mean(axis=(0, 2))
    want = _diffuse_channel(phi.mean(axis=(0, 2)), g, (0.5, 1.5), (0.05, 0.4))
    sharp = T.layered_poiseuille(ny, g, (0.5, 1.5), (0.05, 0.4))
    e = float(np.abs(u - want).max() / np.abs(want).max())
    es = np.abs(u - sharp) / np.abs(sharp).max()
    say(f"  vs diffuse-interface solution {e:.2e}; vs sharp: max {es.max():.2e} at y = "
        f"{int(es.argmax())}")
    assert e <= 1e-2


def test_two_phase_argument_errors():
    import torch
    from paper_2609_09160_amd import LbfastError, Solver
    s = Solver((16, 16, 16), 1.0, storage="f32")
    with pytest.raises(LbfastError, match="E_ARG"):
        s.enable_two_phase(SIGMA, W, DIFF, rho=(0.0, 1.0))
    with pytest.raises(LbfastError, match="E_ARG"):
        s.enable_two_phase(SIGMA, W, DIFF, tau=(1.0, 0.5))
    with pytest.raises(LbfastError, match="E_STATE"):
        s.set_phase(np.zeros((16, 16, 16)))
    s.enable_two_phase(SIGMA, W, DIFF)
    with pytest.raises(LbfastError, match="E_STATE"):
        s.set_force_field(torch.zeros((3, 16, 16, 16), device="cuda"))
    with pytest.raises(LbfastError, match="UNSUPPORTED"):
        s.forward_checkpointed(4, 2)
    s.close()
