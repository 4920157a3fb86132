"""State handling of the C ABI on the GPU: conversions, determinism, restart,
reductions, conservation and error paths."""
import ctypes

import numpy as np
import pytest

from paper_2609_09160_amd import inputs

from gpu_util import say, stored_planes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _solver(shape, **kw):
    from paper_2609_09160_amd import Solver
    return Solver(shape, kw.pop("tau", 0.7), **kw)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_set_get_roundtrip(storage):
    """set then get returns the stored values: FP64 bit for bit, FP32 as the
    round-to-nearest FP32 image of the input; host and device paths agree."""
    import torch
    shape = (37, 11, 5)
    m = inputs.random_state(shape, seed=9)
    s = _solver(shape, storage=storage)
    s.set_moments(m)
    got = s.moments_host()
    want = m if storage == "f64" else m.astype(np.float32).astype(np.float64)
    assert np.array_equal(got, want)
    dev = s.moments().cpu().numpy()
    assert np.array_equal(dev, got)
    s.set_moments(torch.as_tensor(m, device="cuda"))
    assert np.array_equal(s.moments_host(), want)
    s.close()


@pytest.mark.parametrize("storage,bits", [("f16s", 11), ("bf16s", 8)])
def test_16bit_scaled_roundtrip(storage, bits):
    """16-bit storage keeps v/s_m rounded to nearest with a power-of-two scale
    per plane; p* and u are stored directly, the second-order planes as the
    deviation a2 - u u (u as stored).  Round-trip error of each stored value
    <= 2^-bits of its magnitude (normal range), plus FP32 rounding of u u."""
    shape = (40, 9, 6)
    m = inputs.random_state(shape, seed=10)
    s = _solver(shape, storage=storage)
    s.set_moments(m)
    sc = s.scales()
    assert all(float(v) > 0 and np.log2(float(v)).is_integer() for v in sc)
    got = s.moments_host()
    for k in range(4):
        big = np.abs(m[k]) > 1e-3 * np.abs(m[k]).max()
        rel = np.abs(got[k] - m[k]) / np.abs(m[k])
        assert rel[big].max() <= 2.0 ** -bits
    pairs = {4: (1, 1), 5: (2, 2), 6: (3, 3), 7: (1, 2), 8: (1, 3), 9: (2, 3)}
    for k, (a, b) in pairs.items():
        uu = got[a] * got[b]  # the stored velocities
        dev = m[k] - uu
        err = np.abs(got[k] - m[k])
        assert (err <= 2.0 ** -bits * np.abs(dev) + 2.0 ** -22 * (np.abs(uu) + np.abs(m[k]))
                + 1e-30).all()
    s.close()


def _ties(storage, n):
    """n binary32 values that lie exactly halfway between two neighbouring
    16-bit values (kept parts alternately even and odd), over many exponents."""
    i = np.arange(n, dtype=np.uint32)
    if storage == "bf16s":
        # exponents 100..139, 3 kept mantissa bits varying, dropped half = 0x8000
        bits = ((100 + i % 40) << 23) | ((i // 40 % 8) << 16) | 0x8000
        return bits.astype(np.uint32).view(np.float32)
    # float16: 1.k... between k * 2^-10 and (k + 1) * 2^-10, times 2^e
    k = (i % 64).astype(np.float64)
    e = (i // 64 % 12).astype(np.float64) - 6.0
    return ((1.0 + k * 2.0 ** -10 + 2.0 ** -11) * 2.0 ** e).astype(np.float32)


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_16bit_encoding_bit_exact(storage):
    """The stored words of the planes kept directly (p*, u) are v / s rounded to
    nearest even, bit for bit.  The expected words come from numpy's float16
    conversion for FP16 and from integer rounding of the binary32 pattern for
    BF16, both independent of the kernel's conversion instruction.  The p*
    plane holds exact ties at many exponents, where round-half-up or
    truncation would differ."""
    import torch
    shape = (64, 32, 16)
    nx, ny, nz = shape
    N = nx * ny * nz
    m = inputs.random_state(shape, seed=21)
    t = _ties(storage, 4096).astype(np.float64)
    p = m[0].reshape(-1)
    p[:t.size] = t
    m[0] = p.reshape(nz, ny, nx)
    s = _solver(shape, storage=storage, scale=[1.0] * 10)
    s.set_moments(m)
    assert np.array_equal(s.scales(), np.ones(10, dtype=np.float32))
    ptr = s.state_ptr()
    buf = [b for b in s._bufs if b.data_ptr() == ptr]
    assert len(buf) == 1
    words = stored_planes(buf[0][:10 * N * 2].cpu().numpy().view(np.uint16), 10, N)
    for k in range(4):
        x = m[k].reshape(-1).astype(np.float32)
        if storage == "f16s":
            want = x.astype(np.float16).view(np.uint16)
        else:
            u = x.view(np.uint32).astype(np.uint64)
            want = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
        bad = int((words[k] != want).sum())
        say(f"{storage} plane {k}: {bad} of {N} words differ")
        assert bad == 0
    # the step writes the same layout: p* and u read back from its stored
    # words on the host (scale 1) equal what the library decodes
    s.step(1)
    ptr = s.state_ptr()
    buf = [b for b in s._bufs if b.data_ptr() == ptr]
    words = stored_planes(buf[0][:10 * N * 2].cpu().numpy().view(np.uint16), 10, N)
    got = s.moments_host()
    for k in range(4):
        if storage == "f16s":
            host = words[k].view(np.float16).astype(np.float64)
        else:
            host = (words[k].astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        assert np.array_equal(host, got[k].reshape(-1)), f"{storage} plane {k} after a step"
    s.close()


def test_zero_steps_and_determinism():
    shape = (70, 13, 9)
    m = inputs.random_state(shape, seed=3)
    outs = []
    for _ in range(2):
        s = _solver(shape, storage="f32")
        s.set_moments(m)
        s.step(0)
        assert np.array_equal(s.moments_host(), m.astype(np.float32).astype(np.float64))
        s.step(7)
        outs.append(s.moments_host())
        s.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_restart_is_bitwise(storage):
    """n steps, get, set into a fresh solver, n steps == 2n steps (checkpoint)."""
    shape = (66, 10, 12)
    m = inputs.random_state(shape, seed=4)
    a = _solver(shape, storage=storage)
    a.set_moments(m)
    a.step(10)
    mid = a.moments_host()
    a.step(10)
    full = a.moments_host()
    b = _solver(shape, storage=storage)
    b.set_moments(mid)
    b.step(10)
    assert np.array_equal(b.moments_host(), full)
    a.close()
    b.close()


def test_reduce_matches_host_sums():
    """FP64 sums of the device state equal host sums of the fetched state."""
    shape = (65, 17, 9)
    m = inputs.random_state(shape, seed=6)
    s = _solver(shape, storage="f64")
    s.set_moments(m)
    s.step(3)
    red = s.reduce()
    h = s.moments_host()
    want = [h[0].sum(), h[1].sum(), h[2].sum(), h[3].sum(), 0.5 * (h[1:4] ** 2).sum()]
    for r, w, ref in zip(red, want, [np.abs(h[0]).sum(), np.abs(h[1]).sum(), np.abs(h[2]).sum(),
                                     np.abs(h[3]).sum(), abs(want[4])]):
        assert abs(r - w) <= 1e-12 * ref
    s.close()


def test_conservation_fp64():
    """Sum p* invariant; sum u grows by sum F each step (periodic, per-site F)."""
    import torch
    shape = (80, 24, 20)
    m = inputs.random_state(shape, seed=7)
    F = inputs.random_force(shape, seed=8, std=1e-5)
    s = _solver(shape, storage="f64", lattice=27)
    s.set_moments(m)
    s.set_force_field(torch.as_tensor(F, device="cuda"))
    r0 = s.reduce()
    s.step(50)
    r1 = s.reduce()
    assert abs(r1[0] - r0[0]) <= 1e-12 * np.abs(m[0]).sum()
    for a in range(3):
        assert abs(r1[1 + a] - (r0[1 + a] + 50 * F[a].sum())) <= 1e-12 * np.abs(m[1 + a]).sum()
    s.close()


@pytest.mark.parametrize("Q", [19, 27])
def test_conservation_512_fp32(Q):
    """The 512^3 FP32 workload, 1000 steps: mass and momentum sums drift only
    by FP32 rounding (relative to the sum of magnitudes)."""
    import torch
    n = 512
    m0 = inputs.solenoidal_field((n, n, n), device="cuda")
    s = _solver((n, n, n), storage="f32", lattice=Q, tau=0.6)
    s.set_moments(m0)
    del m0
    torch.cuda.empty_cache()
    r0 = s.reduce()
    s.step(1000)
    r1 = s.reduce()
    h = s.moments(dtype=torch.float32)
    mag_p = float(h[0].abs().sum(dtype=torch.float64))
    mag_u = float(h[1:4].abs().sum(dtype=torch.float64))
    del h
    say(f"Q{Q}: d sum p* = {r1[0] - r0[0]:.3e} (|p*| sum {mag_p:.3e}), "
        f"d sum u = {np.abs(r1[1:4] - r0[1:4]).max():.3e} (|u| sum {mag_u:.3e})")
    assert abs(r1[0] - r0[0]) <= 1e-6 * mag_p
    assert np.abs(r1[1:4] - r0[1:4]).max() <= 1e-6 * mag_u
    assert np.isfinite(r1).all()
    s.close()
    torch.cuda.empty_cache()


def test_nonfinite_state_is_reported():
    from paper_2609_09160_amd import LbfastError, _lib
    shape = (16, 8, 8)
    m = inputs.random_state(shape, seed=1)
    m[1, 3, 4, 5] = np.nan
    s = _solver(shape, storage="f32")
    s.set_moments(m)
    with pytest.raises(LbfastError) as e:
        s.reduce()
    assert e.value.code == _lib.LBF_E_NONFINITE
    s.close()


def test_fp16_scales_in_a_channel_start_up():
    """FP16 scales are fixed at the first set_moments.  A channel driven from
    noise (walls in y, 16 x 32 x 8, tau 0.9, g = 1e-4, u = +-1e-4 noise,
    seed 2609) grows its velocity about 900-fold in 3000 steps: with the
    automatic scales taken from the noise the stored velocity overflows FP16
    and lbfast_reduce reports LBF_E_NONFINITE.  With explicit scales sized for
    the developed flow it stays finite, and then the rounding matters: near
    steady state the velocity changes by less than half a unit in the last
    place per step, so rounding to nearest stalls the start-up (several
    percent behind the FP32 run), while stochastic rounding of p* and u keeps
    it within 1e-2."""
    from paper_2609_09160_amd import LbfastError, _lib
    shape = (16, 32, 8)
    nx, ny, nz = shape
    rng = np.random.default_rng(2609)
    m = np.zeros((10, nz, ny, nx))
    m[1:4] = rng.uniform(-1e-4, 1e-4, (3, nz, ny, nx))
    for k, (a, b) in enumerate(((1, 1), (2, 2), (3, 3), (1, 2), (1, 3), (2, 3))):
        m[4 + k] = m[a] * m[b]
    kw = dict(bc=(0, 1, 0), force=(1e-4, 0, 0))

    def run(storage, scale=None, rounding="nearest"):
        from paper_2609_09160_amd import Solver
        s = Solver(shape, 0.9, storage=storage, scale=scale, rounding=rounding, **kw)
        s.set_moments(m)
        s.step(3000)
        try:
            s.reduce()
            return s.moments_host(), None
        except LbfastError as e:
            return None, e.code
        finally:
            s.close()

    ref, _ = run("f32")
    umax = np.abs(ref[1]).max()
    assert umax > 300 * 1e-4
    _, code = run("f16s")
    assert code == _lib.LBF_E_NONFINITE
    errs = {}
    for rounding in ("nearest", "stochastic"):
        got, code = run("f16s", scale=[2.0 ** -14] * 10, rounding=rounding)
        assert code is None
        errs[rounding] = np.linalg.norm(got[1:4] - ref[1:4]) / np.linalg.norm(ref[1:4])
    say(f"channel start-up, FP16 vs FP32 u rel L2: {errs}")
    assert errs["nearest"] > 2e-2
    assert errs["stochastic"] <= 1e-2


def test_argument_errors_on_device():
    import torch
    from paper_2609_09160_amd import LbfastError, _lib
    s = _solver((16, 8, 8), storage="f32")
    with pytest.raises(LbfastError):
        s.step(-1)
    with pytest.raises(LbfastError):
        s.set_launch(5, 0)
    with pytest.raises(ValueError):
        s.set_moments(np.zeros((10, 3)))
    lib = _lib.load()
    F = torch.zeros(3 * 16 * 8 * 8, dtype=torch.float64, device="cuda")
    rc = lib.lbfast_set_force_field(s.h, ctypes.c_void_p(F.data_ptr()), _lib.LBF_F64)
    assert rc == _lib.LBF_E_ARG  # FP32 storage computes in FP32
    host = np.zeros(3 * 16 * 8 * 8, dtype=np.float32)
    rc = lib.lbfast_set_force_field(s.h, host.ctypes.data_as(ctypes.c_void_p), _lib.LBF_F32)
    assert rc == _lib.LBF_E_ARG  # not device memory
    s.close()
    big = _solver((8, 8, 8), storage="f64", lattice=27)
    with pytest.raises(LbfastError) as e:
        big.set_launch(14, 0)  # 24 x 16 x 68 doubles of LDS exceed 160 KiB
    assert e.value.code == _lib.LBF_E_UNSUPPORTED
    big.close()


def test_lane_sites_selection():
    """Two x-sites per lane need an even nx and tiles of at most 8 rows, three
    an nx divisible by 3 and FP32 storage; switching to them lowers a tile
    height whose LDS would not fit (FP64 D3Q27: 6-row tiles of 130 columns
    exceed 160 KiB, 4 rows fit).  The 192-wide default at nx = 192 (FP32)
    gives the same state as one site per lane, to FP32 rounding."""
    from paper_2609_09160_amd import LbfastError, _lib
    lib = _lib.load()
    odd = _solver((65, 8, 8), storage="f32")
    with pytest.raises(LbfastError) as e:
        odd.set_launch(0, 0, 2)
    assert e.value.code == _lib.LBF_E_UNSUPPORTED
    assert lib.lbfast_set_lane_sites(odd.h, 3) == _lib.LBF_E_UNSUPPORTED
    assert lib.lbfast_set_lane_sites(odd.h, 4) == _lib.LBF_E_ARG
    odd.close()
    h16 = _solver((192, 8, 8), storage="f16s")
    assert lib.lbfast_set_lane_sites(h16.h, 3) == _lib.LBF_E_UNSUPPORTED
    h16.close()
    m192 = inputs.random_state((192, 10, 9), seed=5)
    outs = []
    for sites in (0, 1):  # 0: the default (three sites per lane here)
        s3 = _solver((192, 10, 9), storage="f32")
        if sites:
            s3.set_launch(8, 0, sites)
        s3.set_moments(m192)
        s3.step(5)
        outs.append(s3.moments_host())
        s3.close()
    assert np.abs(outs[0] - outs[1]).max() <= 1e-6 * np.abs(outs[1]).max()
    s = _solver((64, 8, 8), storage="f32")
    s.set_launch(8, 0, 2)  # two sites per lane, 8-row tiles
    with pytest.raises(LbfastError) as e:
        s.set_launch(14, 0)  # not built with two sites per lane
    assert e.value.code == _lib.LBF_E_UNSUPPORTED
    s.close()
    big = _solver((64, 8, 8), storage="f64", lattice=27)
    big.set_launch(6, 0, 1)
    big.set_launch(0, 0, 2)  # falls back to 4-row tiles
    m = inputs.random_state((64, 8, 8), seed=2)
    big.set_moments(m)
    big.step(2)
    assert np.isfinite(big.moments_host()).all()
    big.close()
