"""FP16 storage with the velocity split over two binary16 words (LBF_F16SU):
the stored words, the round trip, and the step against the FP64 oracle.
u = s (hi + 2^-11 lo) with hi the binary16 rounding of u/s and lo that of the
remainder times 2^11, so u keeps 22 significant bits while p* and a2 - u u
keep FP16's 11."""
import numpy as np
import pytest

from paper_2609_09160_amd import inputs

from gpu_util import gpu_run, group_rel_err, oracle_run, say, stored_planes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _solver(shape, **kw):
    from paper_2609_09160_amd import Solver
    return Solver(shape, kw.pop("tau", 0.7), storage="f16su", **kw)


def test_split_words_and_roundtrip():
    """The hi and lo words of each velocity plane are the binary16 roundings
    (numpy's float16, an independent conversion) of u/s and of the remainder
    times 2^11; reading back gives u to 2^-22 of its magnitude, p* to 2^-11,
    a2 to 2^-11 of its deviation from u u."""
    shape = (64, 24, 10)
    nx, ny, nz = shape
    N = nx * ny * nz
    m = inputs.random_state(shape, seed=31)
    s = _solver(shape)
    s.set_moments(m)
    sc = s.scales().astype(np.float64)
    ptr = s.state_ptr()
    buf = [b for b in s._bufs if b.data_ptr() == ptr]
    assert len(buf) == 1 and buf[0].numel() == 13 * N * 2
    words = stored_planes(buf[0].cpu().numpy().view(np.uint16), 13, N)
    for c in range(3):
        x = (m[1 + c].reshape(-1).astype(np.float32) * np.float32(1.0 / sc[1 + c]))
        hi = x.astype(np.float16)
        rem = (x - hi.astype(np.float32)) * np.float32(2048.0)
        lo = rem.astype(np.float16)
        bad = int((words[1 + c] != hi.view(np.uint16)).sum() + (words[10 + c] != lo.view(np.uint16)).sum())
        say(f"f16su u{c}: {bad} of {2 * N} words differ")
        assert bad == 0
    got = s.moments_host()
    for k in range(4):
        big = np.abs(m[k]) > 1e-3 * np.abs(m[k]).max()
        rel = np.abs(got[k] - m[k]) / np.abs(m[k])
        assert rel[big].max() <= (2.0 ** -11 if k == 0 else 2.0 ** -22)
    pairs = {4: (1, 1), 5: (2, 2), 6: (3, 3), 7: (1, 2), 8: (1, 3), 9: (2, 3)}
    for k, (a, b) in pairs.items():
        uu = got[a] * got[b]
        err = np.abs(got[k] - m[k])
        assert (err <= 2.0 ** -11 * np.abs(m[k] - uu) + 2.0 ** -22 * (np.abs(uu) + np.abs(m[k]))
                + 1e-30).all()
    s.close()


@pytest.mark.parametrize("shape,bc,force,sites", [
    ((70, 12, 9), (0, 0, 0), (0.0, 0.0, 0.0), 1),      # no force, one site per lane
    ((128, 10, 7), (0, 1, 0), (1e-5, -2e-5, 5e-6), 2),  # y walls, uniform force, two sites
    ((66, 9, 5), (0, 0, 0), None, 1),                   # per-site force field
])
def test_split_step_vs_oracle(shape, bc, force, sites):
    """Five steps from a random off-equilibrium state against the FP64 oracle
    run from the same stored state.  Each step rounds p* and a2 - u u to
    binary16 (2^-11 of a value) and u to 22 bits.  The velocity group then
    carries only what the p* and a2 roundings feed into it (about 1e-4 of its
    magnitude here, where p* is half as large as u): bounded by 2.5e-4, below
    one binary16 rounding of u (2^-11 = 4.9e-4), which FP16 storage proper
    adds at every step.  p* and a2 stay within 5e-3."""
    import torch
    m0 = inputs.random_state(shape, seed=41)
    Ff = None
    if force is None:
        rng = np.random.default_rng(7)
        nx, ny, nz = shape
        Ff = (1e-5 * rng.standard_normal((3, nz, ny, nx))).astype(np.float32)
        force = (0.0, 0.0, 0.0)
    s = _solver(shape, bc=bc, force=force)
    s.set_launch(0, 0, sites)
    s.set_moments(m0)
    start = s.moments_host()
    if Ff is not None:
        s.set_force_field(torch.as_tensor(Ff, device="cuda"))
    s.step(5)
    got = s.moments_host()
    s.close()
    import oracle
    o = oracle.PopulationOracle(19, shape, 0.7, bc=bc,
                                force=Ff.astype(np.float64) if Ff is not None else np.array(force))
    o.set_moments(start)
    o.step(5)
    want = o.moments()
    eu = float(np.abs(got[1:4] - want[1:4]).max() / np.abs(want[1:4]).max())
    eg = group_rel_err(got, want)
    say(f"f16su {shape} bc={bc} sites={sites}: u group {eu:.2e}, all groups {eg:.2e}")
    assert eu <= 2.5e-4 and eg <= 5e-3


def test_split_rejections():
    """Split storage: rounding to nearest, one component."""
    from paper_2609_09160_amd import LbfastError, Solver, _lib
    # the parameter check runs when the Solver sizes its buffers
    with pytest.raises(LbfastError, match="nearest"):
        Solver((32, 8, 8), 0.7, storage="f16su", rounding="stochastic")
    s = _solver((32, 8, 8))
    with pytest.raises(LbfastError) as e:
        s.enable_two_phase(0.03, 4.0, 0.1)
    assert e.value.code == _lib.LBF_E_UNSUPPORTED
    s.close()
