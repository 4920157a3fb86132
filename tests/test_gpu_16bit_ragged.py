"""16-bit storage on ragged grids: one step of the HIP path from a stored
16-bit state against the FP64 oracle's step from the same (decoded) state.

The grids have an odd nx (one site per lane: single-site group loads), an
even nx that leaves the last 128-wide tile partly empty (two sites per lane),
rows that do not fill the last tile, few z-planes, and walls in y: every
load and store of the grouped 16-bit layout (planes in groups of four per
64-bit word, a pair, a single plane) meets a tile edge or the periodic wrap.

Bars: the step rounds each stored value once, so each moment group (p*, u,
a2) is within twice one unit in the last place of its magnitude: 2e-3 for
FP16 (2^-10), 1.6e-2 for BF16 (2^-7 with stochastic rounding); the
split-velocity form keeps u to 2^-22, its u group is held to 2.5e-4."""
import numpy as np
import pytest

from paper_2609_09160_amd import inputs

from gpu_util import group_rel_err, say

pytestmark = pytest.mark.gpu

# (odd nx: one site per lane; nx = 200 and 250: two sites per lane by
# default, the last 128-wide tile partly empty)
CASES = [((37, 11, 6), (0, 0, 0), 19), ((200, 9, 5), (0, 1, 0), 19),
         ((250, 6, 4), (0, 0, 0), 27), ((35, 13, 5), (0, 1, 0), "27h")]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


@pytest.mark.parametrize("storage,bound,ubound", [("f16s", 2e-3, 2e-3), ("bf16s", 1.6e-2, 1.6e-2),
                                                  ("f16su", 2e-3, 2.5e-4)])
@pytest.mark.parametrize("shape,bc,Q", CASES)
def test_16bit_step_on_ragged_grids(storage, bound, ubound, shape, bc, Q):
    import oracle
    from paper_2609_09160_amd import Solver
    tau = 0.7
    m0 = inputs.random_state(shape, seed=sum(shape) + len(storage))
    s = Solver(shape, tau, lattice=Q, storage=storage, bc=bc)
    s.set_moments(m0)
    start = s.moments_host()
    s.step(1)
    got = s.moments_host()
    s.close()
    o = oracle.PopulationOracle(Q, shape, tau, bc=bc)
    o.set_moments(start)
    o.step(1)
    want = o.moments()
    eg = group_rel_err(got, want)
    eu = float(np.abs(got[1:4] - want[1:4]).max() / np.abs(want[1:4]).max())
    say(f"{storage} D3Q{Q} {shape} bc={bc}: groups {eg:.2e}, u {eu:.2e}")
    assert eg <= bound and eu <= ubound


@pytest.mark.parametrize("storage,bound", [("f16s", 2e-3), ("bf16s", 1.6e-2)])
@pytest.mark.parametrize("shape,bc,rho,taus", [((37, 11, 6), (0, 0, 0), (1.0, 1.0), None),
                                               ((200, 9, 5), (0, 1, 0), (0.5, 1.5), (0.65, 1.1))])
def test_16bit_two_component_step_on_ragged_grids(storage, bound, shape, bc, rho, taus):
    """The two-component step with a 16-bit state (the phase update reads u
    from the grouped words), one step from the stored state against the
    two-component oracle: moment groups as above, phi (FP32) within 1e-5."""
    from oracle import two_phase as T
    from paper_2609_09160_amd import Solver
    sigma, width, diff, tau = 0.03, 4.0, 0.1, 0.8
    nx, ny, nz = shape
    rng = np.random.default_rng(sum(shape))
    phi0 = T.droplet(shape, 3.0, width, center=(nx / 3, ny / 2, nz / 2))
    m0 = np.zeros((10, nz, ny, nx))
    m0[0] = 1e-3 * rng.standard_normal((nz, ny, nx))
    m0[1:4] = 1e-3 * rng.standard_normal((3, nz, ny, nx))
    m0[4:] = 1e-4 * rng.standard_normal((6, nz, ny, nx))
    for a, b, k in ((0, 0, 4), (1, 1, 5), (2, 2, 6), (0, 1, 7), (0, 2, 8), (1, 2, 9)):
        m0[k] += m0[1 + a] * m0[1 + b]
    s = Solver(shape, tau, storage=storage, bc=bc)
    s.enable_two_phase(sigma, width, diff, rho=rho, tau=taus if taus is not None else tau)
    s.set_moments(m0)
    s.set_phase(np.ascontiguousarray(phi0))
    start = s.moments_host()
    phi_start = s.phase().cpu().numpy().astype(np.float64)
    s.step(1)
    got, phi = s.moments_host(), s.phase().cpu().numpy().astype(np.float64)
    s.close()
    nu = None if taus is None else tuple((t - 0.5) / 3.0 for t in taus)
    o = T.TwoPhaseOracle(19, shape, tau, sigma, width, diff, bc=bc, rho=rho, nu=nu)
    o.set_state(start, phi_start)
    o.step(1)
    eg = group_rel_err(got, o.moments())
    ephi = float(np.abs(phi - o.phi).max() / np.abs(o.phi).max())
    say(f"{storage} two-component {shape} bc={bc} rho={rho}: groups {eg:.2e}, phi {ephi:.2e}")
    assert eg <= bound and ephi <= 1e-5
