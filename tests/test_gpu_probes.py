"""The library's copy probes (the bandwidth ceilings the step is measured
against) move every byte: exact copies at a full-tile size and at a ragged one
whose last block is partly empty."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,nplanes", [(1 << 16, 10), (2 * 70001, 10), (2 * 333, 3), (2, 1)])
def test_copy_probes_are_exact(n, nplanes):
    import torch
    from paper_2609_09160_amd import _lib
    lib = _lib.load()
    g = torch.Generator(device="cpu").manual_seed(n + nplanes)
    a = torch.rand(nplanes * n, generator=g).cuda()
    guard = torch.full((nplanes * n + 64,), -7.0, device="cuda")
    stream = torch.cuda.current_stream()
    S = ctypes.c_void_p(stream.cuda_stream)
    A, B = ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(guard.data_ptr())
    _lib.check(lib.lbfast_planes_probe(A, B, n, nplanes, S))
    torch.cuda.synchronize()
    assert torch.equal(guard[:nplanes * n], a)
    assert bool((guard[nplanes * n:] == -7.0).all())
    if (nplanes * n) % 4 == 0:
        guard.fill_(-7.0)
        _lib.check(lib.lbfast_copy_probe(A, B, nplanes * n // 4, S))
        torch.cuda.synchronize()
        assert torch.equal(guard[:nplanes * n], a)
        assert bool((guard[nplanes * n:] == -7.0).all())


@pytest.mark.parametrize("layout", [0, 1, 2, 3])
@pytest.mark.parametrize("nx,ny,nz,zchunk", [(128, 16, 5, 2), (256, 8, 3, 7)])
def test_zmarch_probe_is_exact(layout, nx, ny, nz, zchunk):
    """The marching copy moves every byte of the state in each layout,
    with a ragged last z-chunk, and nothing past it."""
    import torch
    from paper_2609_09160_amd import _lib
    lib = _lib.load()
    nbytes = (40 if layout == 0 else 20) * nx * ny * nz
    g = torch.Generator(device="cpu").manual_seed(layout * 7 + nx + nz)
    a = torch.randint(-2**31, 2**31 - 1, (nbytes // 4,), dtype=torch.int32, generator=g).cuda()
    guard = torch.full((nbytes // 4 + 64,), -7, dtype=torch.int32, device="cuda")
    S = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib.lbfast_zmarch_probe(ctypes.c_void_p(a.data_ptr()),
                                       ctypes.c_void_p(guard.data_ptr()), nx, ny, nz, layout,
                                       zchunk, S))
    torch.cuda.synchronize()
    assert torch.equal(guard[:nbytes // 4], a)
    assert bool((guard[nbytes // 4:] == -7).all())
