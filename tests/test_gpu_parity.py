"""Parity of the HIP step (through the C ABI) with the FP64 CPU oracle.

Bars: FP64 storage -- max error <= 1e-12 relative to the magnitude of each
moment group (short runs) or of the whole state and of the velocity (long
runs, where a moment may decay far below the others); FP32 -- relative L2
error of the velocity <= 1e-5 after 1000 steps (the FP32 bar stated for the
method); sizes span several 64 x TY tiles and z-chunks with ragged tails in
x, y and z.
"""
import numpy as np
import pytest

from paper_2609_09160_amd import inputs

from gpu_util import (group_rel_err, gpu_run, lattice_number, oracle_run, say, state_rel_err,
                      u_rel_l2)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


@pytest.mark.parametrize("Q", [19, 27, "27h"])
def test_taylor_green_fp64(Q):
    """Taylor-Green vortex (section 4, Eq. (11)), 32^3, tau = 0.8, U0 = 0.01,
    200 steps, FP64: moments match the oracle to 1e-12."""
    n, tau = 32, 0.8
    m0 = inputs.taylor_green(n, 0.01)
    say(f"TG fp64 Q{Q}")
    got = gpu_run((n, n, n), tau, m0, 200, lattice=Q, storage="f64")
    want = oracle_run((n, n, n), tau, m0, 200, lattice=Q)
    err = group_rel_err(got, want)
    say(f"  max group rel err {err:.3e}")
    assert err <= 1e-12


SHAPES = [(130, 19, 21), (7, 5, 3), (1, 1, 1), (65, 9, 40), (64, 16, 2)]


@pytest.mark.parametrize("Q", [19, 27, "27h"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("forcing", ["uniform", "field"])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("sites", [1, 2])
def test_ragged_fp64(Q, shape, forcing, walls, sites):
    """Off-equilibrium random state, uniform or per-site force, periodic or
    y-walls, ragged sizes and small z-chunks, one or two x-sites per lane
    (two: 128-wide tiles, also wider than the grid): 6 steps, FP64, <= 1e-12."""
    if walls and shape[1] < 2:
        pytest.skip("a walled axis needs >= 2 sites")
    if sites == 2 and shape[0] % 2:
        pytest.skip("two sites per lane need an even nx")
    tau = 0.7
    bc = (0, 1 if walls else 0, 0)
    m0 = inputs.random_state(shape, seed=sum(shape) + lattice_number(Q))
    F = inputs.random_force(shape, seed=7, std=1e-4)
    Fu = (2e-5, -1e-5, 3e-5)
    say(f"ragged fp64 Q{Q} {shape} {forcing} walls={walls} sites={sites}")
    if forcing == "uniform":
        got = gpu_run(shape, tau, m0, 6, lattice=Q, bc=bc, force=Fu, launch=(0, 4, sites))
        want = oracle_run(shape, tau, m0, 6, lattice=Q, bc=bc, force=np.array(Fu))
    else:
        got = gpu_run(shape, tau, m0, 6, lattice=Q, bc=bc, Ffield=F, launch=(0, 4, sites))
        want = oracle_run(shape, tau, m0, 6, lattice=Q, bc=bc, force=F)
    err = group_rel_err(got, want)
    say(f"  err {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("Q", [19, 27])
@pytest.mark.parametrize("shape", [(195, 13, 20), (192, 6, 3), (3, 5, 4)])
@pytest.mark.parametrize("forcing", ["none", "uniform", "field"])
@pytest.mark.parametrize("walls", [False, True])
def test_three_sites_fp32(Q, shape, forcing, walls):
    """Three x-sites per lane (192-wide tiles, FP32 storage only): a full tile
    plus a ragged 3-site tail, one exact tile, and a grid narrower than one
    lane's sites times a wave; off-equilibrium random state, no force, a
    uniform or a per-site force, periodic or y-walls, 6 steps against the FP64
    oracle: max error <= 1e-6 of each moment group (FP32 storage rounding)."""
    tau = 0.7
    bc = (0, 1 if walls else 0, 0)
    m0 = inputs.random_state(shape, seed=sum(shape) + Q)
    F = inputs.random_force(shape, seed=8, std=1e-4)
    Fu = (2e-5, -1e-5, 3e-5)
    say(f"three sites fp32 Q{Q} {shape} {forcing} walls={walls}")
    kw = dict(lattice=Q, bc=bc, storage="f32", launch=(6, 0, 3))
    if forcing == "none":
        got = gpu_run(shape, tau, m0, 6, **kw)
        want = oracle_run(shape, tau, m0, 6, lattice=Q, bc=bc)
    elif forcing == "uniform":
        got = gpu_run(shape, tau, m0, 6, force=Fu, **kw)
        want = oracle_run(shape, tau, m0, 6, lattice=Q, bc=bc, force=np.array(Fu))
    else:
        got = gpu_run(shape, tau, m0, 6, Ffield=F.astype(np.float32), **kw)
        want = oracle_run(shape, tau, m0, 6, lattice=Q, bc=bc, force=F.astype(np.float32).astype(np.float64))
    err = group_rel_err(got, want)
    say(f"  err {err:.3e}")
    assert err <= 1e-6


@pytest.mark.parametrize("Q", [19, 27, "27h"])
def test_fp32_solenoidal_1000_steps(Q):
    """The 512^3 throughput workload's family at 64^3: random solenoidal field
    (|k| <= 8, rms 0.02), tau = 0.6, 1000 steps, FP32 storage: relative L2
    error of u against the FP64 oracle <= 1e-5."""
    n, tau = 64, 0.6
    m0 = inputs.solenoidal_field((n, n, n))
    say(f"fp32 solenoidal Q{Q}")
    got = gpu_run((n, n, n), tau, m0, 1000, lattice=Q, storage="f32")
    want = oracle_run((n, n, n), tau, m0, 1000, lattice=Q)
    e = u_rel_l2(got, want)
    say(f"  u rel L2 {e:.3e}")
    assert e <= 1e-5


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_channel_with_walls(storage, tol):
    """Channel of the Poiseuille workload at 32^3: walls in y, g_x = 1e-6,
    tau = 0.9, noise +-1e-4 (seed 2609), 2000 steps."""
    shape, tau = (32, 32, 32), 0.9
    m0 = inputs.channel_noise(shape)
    F = np.array([1e-6, 0.0, 0.0])
    say(f"channel {storage}")
    got = gpu_run(shape, tau, m0, 2000, storage=storage, bc=(0, 1, 0), force=F)
    want = oracle_run(shape, tau, m0, 2000, bc=(0, 1, 0), force=F)
    say("  per-group rel err " + str([group_rel_err(got[lo:hi], want[lo:hi])
                                       for lo, hi in ((0, 1), (1, 4), (4, 10))]))
    if storage == "f64":
        err = state_rel_err(got, want)
    else:
        err = u_rel_l2(got, want)
    say(f"  err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("Q", [19, 27, "27h"])
def test_launch_shape_invariance(Q):
    """Different tile heights, z-chunks and x-sites per lane agree to rounding
    (catches missing barriers or halo mistakes that depend on the tiling; the
    shapes are separately compiled, so the last bits may differ), and one
    launch shape is bitwise reproducible."""
    shape = (130, 37, 45)
    m0 = inputs.random_state(shape, seed=5)
    ref = gpu_run(shape, 0.65, m0, 3, lattice=Q, storage="f32", launch=(8, 0, 1))
    again = gpu_run(shape, 0.65, m0, 3, lattice=Q, storage="f32", launch=(8, 0, 1))
    assert np.array_equal(again, ref)
    scale = np.abs(ref).max()
    for launch in ((4, 0, 1), (6, 0, 1), (14, 0, 1), (8, 3, 1), (4, 7, 2), (6, 45, 2),
                   (8, 5, 2), (8, 1, 2), (4, 0, 2), (8, 0, 2)):
        if Q == "27h" and launch[0] > 8:
            continue  # D3Q27h is built for tiles of up to 8 rows
        got = gpu_run(shape, 0.65, m0, 3, lattice=Q, storage="f32", launch=launch)
        d = np.abs(got - ref).max()
        say(f"launch {launch}: max diff {d:.3e} (scale {scale:.3e})")
        assert d <= 1e-6 * scale


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_block_order_is_bitwise_neutral(storage):
    """The two workgroup orders over the XCDs compute bitwise the same state
    (the order is a scheduling choice; each site's arithmetic is unchanged)."""
    from paper_2609_09160_amd import Solver
    shape = (200, 37, 21)
    m0 = inputs.random_state(shape, seed=11)
    out = []
    for order in (1, 2):
        s = Solver(shape, 0.65, storage=storage, bc=(0, 1, 0))
        s.set_block_order(order)
        s.set_moments(m0)
        s.step(3)
        out.append(s.moments_host())
        s.close()
    assert np.array_equal(out[0], out[1])
